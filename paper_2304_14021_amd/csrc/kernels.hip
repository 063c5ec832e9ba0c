// HIP kernels (gfx950) of the all-at-once space-time solve, FFT path.
//
// Data: U [N_t][N_y][N_x] FP64 (caller's), S [N_t][k_y][k_x] in the working
// type W (float or double, the spectral scratch).  One outer iteration,
// correction form U <- U + P_alpha^{-1} r(U), is
//   k_rows_fwd   a1 + a2 (x): FP64 residual of a block of RB rows (with a
//                two-row halo for the 13-point stencil), then the orthonormal
//                DCT-II along x of those rows  ->  S
//   k_cols<fwd>  a2 (y): DCT-II along y of a tile of XB columns of one level
//   k_time_solve a3-a5: per tile of M spatial cosine modes, Gamma_alpha scaling,
//                FFT over time, shifted complex divide, inverse FFT,
//                Gamma_alpha^{-1} scaling (Section 2.1, eq. pintiter1;
//                Section 4.1, eqs. pintiter_CH and pintiter_CH_eyre)
//   k_cols<inv>  a6 (y): DCT-III along y
//   k_rows_inv   a6 (x): DCT-III along x, U += delta in FP64, partial norms
//   k_finalize   a7: fixed-order reduction, scalar averaged Jacobian, stop rule
// In 1D the "rows" are time levels and the column passes are skipped.  Every
// transform pass moves data global -> LDS (reordered and packed two real
// sequences per complex one) -> radix-8 Stockham FFT in LDS -> global, so each
// pass reads and writes its tile once.  All kernels return at once when the
// device stop flag is set, so iterations can be enqueued ahead of the host's
// check.
#include "pint.h"
#include "pint_kernels.hpp"
#include "fft_lds.hpp"
#include "stop_rule.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace pint {

thread_local hipEvent_t g_launch_ev0 = nullptr, g_launch_ev1 = nullptr;

// Neumann (ghost-reflection) index clamp.
__device__ __forceinline__ int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// Value at offset off of the predecessor of the first level: the datum u0,
// or wrap_alpha u_{N_t} for the alpha-circulant operator.
__device__ __forceinline__ double prev0(const ResidArgs& a, int off, size_t ns) {
  return a.wrap ? a.wrap_alpha * a.U[size_t(a.nt - 1) * ns + off] : a.u0[off];
}

template <typename T>
__device__ __forceinline__ T& comp(cx<T>& c, int i) {
  return i ? c.y : c.x;
}

// Copy a small read-only table into LDS (caller synchronizes before use).
template <typename T, int NT, int LEN>
__device__ __forceinline__ void table_to_lds(cx<T>* dst, const cx<T>* __restrict__ src) {
#pragma unroll
  for (int i = 0; i < cdiv_i(LEN, NT); ++i) {
    const int j = threadIdx.x + i * NT;
    if (LEN % NT == 0 || j < LEN) dst[j] = src[j];
  }
}

// ---------------------------------------------------------------------------
// a1 + a2(x).  DIM == 2: block b covers rows y0 .. y0+RB-1 of level
// n = b / (N/RB).  DIM == 1: block b covers levels b*RB .. b*RB+RB-1 (one
// row each).  The residual of level n is
//   r_n = -(u_n - u_{n-1})/dt + Lap_h g_n,
//   g   = c3 v^3 + c1 v + c1p u_{n-1} + c2 Lap_h v,  v = theta u_n + (1-theta) u_{n-1},
// which is the alpha = 0 row of eq. all-at-once1 (c3 = 0, c1 = -beta^2,
// c1p = 0, c2 = -eps^2; biharmonic c1 = 0, c2 = -1), of eq. nonlinear_G
// (theta = 1, c3 = 1, c1 = -1, c2 = -eps^2) and of eq. nonlinear_Q
// (theta = 1, c3 = 1, c1 = 0, c1p = -1, c2 = -eps^2).  Lap_h is the
// cell-centred Neumann Laplacian: neighbours outside the grid are reflected.
// With a.bcast the iterate is u0 at every level (first iteration from the
// broadcast initial guess), so u_n - u_{n-1} = 0.
// MODE 0 writes the x-DCT of r (type T) to S; MODE 1 writes r (FP64) to rout.
template <int DIM, int N, int RB>
struct rows_geom {
  static constexpr int NBL = DIM == 2 ? N / RB : 1;  // blocks per level
  static constexpr int H = DIM == 2 ? 2 : 0;         // v halo rows
  static constexpr int VR = RB + 2 * H;              // v rows (positions y0-2 .. y0+RB+1; LDS rows in 1D)
  static constexpr int GR = RB + (DIM == 2 ? 2 : 0); // g rows (positions y0-1 .. y0+RB; LDS rows in 1D)
  static constexpr int P = RB / 2;                   // packed complex sequences
  static constexpr int ES = P + 1;                   // odd stride of the complex scratch
};

// RT: the residual's arithmetic type (double; float for the unrefined mode).
template <typename T, typename TO, int DIM, int N, int RB, int NT, int MODE, typename RT>
__global__ __launch_bounds__(NT) void k_rows_fwd(ResidArgs a, TO* __restrict__ S, double* __restrict__ rout,
                                                  DctTables<T> dt) {
  if (a.done && *a.done) return;
  using Gm = rows_geom<DIM, N, RB>;
  constexpr int VR = Gm::VR, GR = Gm::GR, P = Gm::P, ES = Gm::ES, NBL = Gm::NBL;
  // 2D: v at RB + 2 rows per thread group of NT / N (see below); 1D: VR rows
  constexpr int VROWS = DIM == 2 ? RB + 2 * (NT / N) : VR;
  constexpr int VB = VROWS * N * int(sizeof(RT)), GB = GR * N * int(sizeof(RT)), ZB = N * ES * int(sizeof(cx<T>));
  constexpr int R0 = VB > ZB ? (VB > GB ? VB : GB) : (ZB > GB ? ZB : GB);
  constexpr int NV = DIM == 2 ? 1 : RB;
  // one buffer holds v, then g, then the packed DCT input (each phase keeps
  // its results in registers across the barrier before overwriting it)
  __shared__ __align__(16) unsigned char lds[R0];
  __shared__ double red[NT * NV];
  __shared__ cx<T> s_tw[N], s_wq[N];
  RT* V = reinterpret_cast<RT*>(lds);
  cx<T>* z = reinterpret_cast<cx<T>*>(lds);
  RT* G = reinterpret_cast<RT*>(lds);
  if (MODE == 0) {
    table_to_lds<T, NT, N>(s_tw, dt.tw);
    table_to_lds<T, NT, N>(s_wq, dt.wq);
  }
  const int tid = threadIdx.x;
  // XCD strips: workgroup p runs on XCD p mod 8; each XCD takes a contiguous
  // strip of NBL / 8 row blocks of every level, so halo rows shared by
  // neighbouring blocks stay in one L2 (the previous level's block of the
  // same rows already shares the XCD)
  const int b = [] {
    const int p = blockIdx.x;
    if constexpr (DIM == 2 && NBL % 8 == 0) {
      const int l = p / NBL, r = p - l * NBL;
      return l * NBL + (r & 7) * (NBL / 8) + (r >> 3);
    } else {
      return p;
    }
  }();
  const int lev = DIM == 2 ? b / NBL : b * RB;
  const int y0 = DIM == 2 ? (b - (b / NBL) * NBL) * RB : 0;
  const size_t ns = DIM == 2 ? size_t(N) * N : size_t(N);
  const bool bc = a.bcast != 0;
  const double th = a.theta, omth = 1.0 - a.theta;
  const RT thr = RT(th), omr = RT(omth);

  double rsq[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) rsq[q] = 0.0;
  if constexpr (DIM == 2) {
    // Thread t owns column x = t mod N of rows yb .. yb+OR-1 (group t / N of
    // the NT / N groups).  It holds that column's v at rows yb-2 .. yb+OR+1
    // and g at yb-1 .. yb+OR in registers, so the stencils' vertical
    // neighbours never leave the thread; the horizontal ones come from the
    // group's LDS rows (v at yb-1 .. yb+OR, then g at yb .. yb+OR-1).
    constexpr int GQ = NT / N, OR = RB / GQ, LR = OR + 2;
    static_assert(NT % N == 0 && RB % GQ == 0, "whole rows per thread group");
    const int x = tid & (N - 1), gq = tid / N;
    const int yb = y0 + gq * OR;
    const int xl = clampi(x - 1, N), xr = clampi(x + 1, N);
    RT* Vg = V + gq * LR * N;  // row j (-1 .. OR) of the group at Vg[(j + 1) N]
    const size_t lo = size_t(lev) * ns;
    // All loads first: u_n at rows yb-2 .. yb+OR+1, u_{n-1} at the own rows
    // and (theta < 1) at the four halo rows.  Level bases are uniform: u_n,
    // and u_{n-1} = sm * Pm (the predecessor of level 0 is u0, or wrap_alpha
    // u_{N_t} for the alpha-circulant operator); 32-bit offsets from them.
    const double* Pn = bc ? a.u0 : a.U + lo;
    const double* Pm = bc ? a.u0 : (lev > 0 ? a.U + lo - ns : (a.wrap ? a.U + size_t(a.nt - 1) * ns : a.u0));
    const double sm = (!bc && lev == 0 && a.wrap) ? a.wrap_alpha : 1.0;
    const bool halo_m = bc || omth != 0.0;
    double un[OR + 4], um[OR], uh[4];
#pragma unroll
    for (int j = 0; j < OR + 4; ++j) un[j] = Pn[unsigned(clampi(yb - 2 + j, N) * N + x)];
#pragma unroll
    for (int i = 0; i < OR; ++i) um[i] = Pm[unsigned((yb + i) * N + x)];
#pragma unroll
    for (int h = 0; h < 4; ++h)
      uh[h] = halo_m ? Pm[unsigned(clampi(yb - 2 + (h < 2 ? h : OR + h), N) * N + x)] : 0.0;
#pragma unroll
    for (int i = 0; i < OR; ++i) um[i] *= sm;
#pragma unroll
    for (int h = 0; h < 4; ++h) uh[h] *= sm;
    RT v[OR + 4], d[OR];
#pragma unroll
    for (int j = 0; j < OR + 4; ++j) {
      const int i = j - 2;
      const double m = i < 0 ? uh[j] : (i >= OR ? uh[j - OR] : um[i]);
      v[j] = thr * RT(un[j]) + omr * RT(m);
    }
#pragma unroll
    for (int i = 0; i < OR; ++i) d[i] = RT(un[i + 2]) - RT(um[i]);
#pragma unroll
    for (int j = 1; j < OR + 3; ++j) Vg[(j - 1) * N + x] = v[j];
    __syncthreads();
    // g at rows yb-1 .. yb+OR; a row outside the grid takes the value of its
    // reflection (the row inside), as the Neumann ghost of g
    RT g[LR];
#pragma unroll
    for (int j = 0; j < LR; ++j) {
      const RT vc = v[j + 1];
      RT lap = Vg[j * N + xl] + Vg[j * N + xr] - RT(2) * vc;
      lap += v[j] + v[j + 2] - RT(2) * vc;
      const int goff = clampi(yb - 1 + j, N) * N + x;
      const RT nl = a.jfield ? RT(a.jfield[goff]) * vc : RT(a.c3) * vc * vc * vc;
      RT gv = nl + RT(a.c1) * vc + RT(a.c2) * (lap * RT(a.inv_h2));
      if (a.c1p != 0.0) {
        const RT umg = RT(bc ? a.u0[goff] : (lev == 0 ? prev0(a, goff, ns) : a.U[lo - ns + goff]));
        gv += RT(a.c1p) * umg;
      }
      g[j] = gv;
      asm volatile("" ::: "memory");  // one row's LDS reads at a time (registers)
    }
    if (yb == 0) g[0] = g[1];
    if (yb + OR == N) g[LR - 1] = g[LR - 2];
    __syncthreads();  // every v read
#pragma unroll
    for (int i = 0; i < OR; ++i) Vg[(i + 1) * N + x] = g[i + 1];
    __syncthreads();
    RT rval[OR];
    const RT idt = RT(a.inv_dts ? a.inv_dts[lev] : a.inv_dt);
#pragma unroll
    for (int i = 0; i < OR; ++i) {
      const RT gc = g[i + 1];
      RT lap = Vg[(i + 1) * N + xl] + Vg[(i + 1) * N + xr] - RT(2) * gc;
      lap += g[i] + g[i + 2] - RT(2) * gc;
      const RT r = -d[i] * idt + lap * RT(a.inv_h2);
      rsq[0] += double(r) * double(r);
      rval[i] = r;
      asm volatile("" ::: "memory");
    }
    __syncthreads();  // every g read
#pragma unroll
    for (int i = 0; i < OR; ++i) {
      const int rr = gq * OR + i;
      if (MODE == 1) rout[lo + size_t(y0 + rr) * N + x] = double(rval[i]);
      else comp(z[dct_iperm<N>(x) * ES + (rr >> 1)], rr & 1) = T(rval[i]);
    }
  } else {
    // Phase 1: v at positions y0-2 .. y0+RB+1 (clamped rows) -> V.  The own
    // rows' time differences d = u_n - u_{n-1} stay in registers for phase 3
    // (same point-to-thread map).  All loads are issued before any is used.
    constexpr int HW = 2 * Gm::H * N, OW = RB * N;
    constexpr int ITH = cdiv_i(HW, NT), ITO = cdiv_i(OW, NT);
    RT d[ITO];
    {
      double hn[ITH > 0 ? ITH : 1], hm[ITH > 0 ? ITH : 1], on[ITO], om[ITO];
#pragma unroll
      for (int i = 0; i < ITH; ++i) {
        const int w = tid + i * NT;
        hn[i] = hm[i] = 0.0;
        if (HW % NT == 0 || w < HW) {
          const int hr = w / N, x = w - (w / N) * N;
          const int vr = hr < Gm::H ? hr : hr + RB;
          const int off = clampi(y0 - Gm::H + vr, N) * N + x;
          if (bc) {
            hn[i] = hm[i] = a.u0[off];
          } else {
            hn[i] = a.U[lev * ns + off];
            // v = theta u_n + (1 - theta) u_{n-1}: no u_{n-1} halo for theta = 1
            if (omth != 0.0) hm[i] = lev == 0 ? prev0(a, off, ns) : a.U[(lev - 1) * ns + off];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < ITO; ++i) {
        const int w = tid + i * NT;
        on[i] = om[i] = 0.0;
        if (OW % NT == 0 || w < OW) {
          const int rr = w / N, x = w - (w / N) * N;
          const int n = DIM == 2 ? lev : lev + rr;
          const int off = DIM == 2 ? (y0 + rr) * N + x : x;
          if (bc) {
            on[i] = om[i] = a.u0[off];
          } else {
            on[i] = a.U[n * ns + off];
            om[i] = n == 0 ? prev0(a, off, ns) : a.U[(n - 1) * ns + off];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < ITH; ++i) {
        const int w = tid + i * NT;
        if (HW % NT == 0 || w < HW) {
          const int hr = w / N, x = w - (w / N) * N;
          const int vr = hr < Gm::H ? hr : hr + RB;
          V[vr * N + x] = thr * RT(hn[i]) + omr * RT(hm[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < ITO; ++i) {
        const int w = tid + i * NT;
        d[i] = RT(on[i]) - RT(om[i]);
        if (OW % NT == 0 || w < OW) V[Gm::H * N + w] = thr * RT(on[i]) + omr * RT(om[i]);
      }
    }
    __syncthreads();
    // Phase 2: g at positions clamp(y0-1 .. y0+RB) -> registers -> G.
    constexpr int GW = GR * N, ITG = cdiv_i(GW, NT);
    RT gval[ITG];
#pragma unroll
    for (int i = 0; i < ITG; ++i) {
      const int idx = tid + i * NT;
      gval[i] = RT(0);
      if (!(GW % NT == 0 || idx < GW)) continue;
      const int gr = idx / N, x = idx - (idx / N) * N;
      int c, yg = 0;
      if (DIM == 2) {
        yg = clampi(y0 - 1 + gr, N);
        c = yg - (y0 - 2);  // V row holding position yg
      } else {
        c = gr;
      }
      const RT v = V[c * N + x];
      RT lap = V[c * N + clampi(x - 1, N)] + V[c * N + clampi(x + 1, N)] - RT(2) * v;
      if (DIM == 2) lap += V[(c - 1) * N + x] + V[(c + 1) * N + x] - RT(2) * v;
      const int goff = DIM == 2 ? yg * N + x : x;
      // cubic term, or the averaged Jacobian field times v (linearized operator)
      const RT nl = a.jfield ? RT(a.jfield[goff]) * v : RT(a.c3) * v * v * v;
      RT g = nl + RT(a.c1) * v + RT(a.c2) * (lap * RT(a.inv_h2));
      if (a.c1p != 0.0) {
        const int n = DIM == 2 ? lev : lev + gr;
        const RT um = RT(bc ? a.u0[goff] : (n == 0 ? prev0(a, goff, ns) : a.U[(n - 1) * ns + goff]));
        g += RT(a.c1p) * um;
      }
      gval[i] = g;
    }
    __syncthreads();  // every v read
#pragma unroll
    for (int i = 0; i < ITG; ++i) {
      const int idx = tid + i * NT;
      if (GW % NT == 0 || idx < GW) G[idx] = gval[i];
    }
    __syncthreads();
    // Phase 3: r on the own rows -> registers -> packed into z (same buffer).
    RT rval[ITO];
#pragma unroll
    for (int i = 0; i < ITO; ++i) {
      const int w = tid + i * NT;
      rval[i] = RT(0);
      if (!(OW % NT == 0 || w < OW)) continue;
      const int rr = w / N, x = w - (w / N) * N;
      const int gc = DIM == 2 ? rr + 1 : rr;
      const RT gv = G[gc * N + x];
      RT lap = G[gc * N + clampi(x - 1, N)] + G[gc * N + clampi(x + 1, N)] - RT(2) * gv;
      if (DIM == 2) lap += G[(gc - 1) * N + x] + G[(gc + 1) * N + x] - RT(2) * gv;
      const int nl = DIM == 2 ? lev : lev + rr;
      const RT r = -d[i] * RT(a.inv_dts ? a.inv_dts[nl] : a.inv_dt) + lap * RT(a.inv_h2);
#pragma unroll
      for (int qq = 0; qq < NV; ++qq)
        if (DIM == 2 || qq == rr) rsq[qq] += double(r) * double(r);
      rval[i] = r;
    }
    __syncthreads();  // every g read
#pragma unroll
    for (int i = 0; i < ITO; ++i) {
      const int w = tid + i * NT;
      if (!(OW % NT == 0 || w < OW)) continue;
      const int rr = w / N, x = w - (w / N) * N;
      if (MODE == 1) {
        const int n = DIM == 2 ? lev : lev + rr;
        const int off = DIM == 2 ? (y0 + rr) * N + x : x;
        rout[n * ns + off] = double(rval[i]);
      } else {
        comp(z[dct_iperm<N>(x) * ES + (rr >> 1)], rr & 1) = T(rval[i]);
      }
    }
  }
  __syncthreads();
  if (MODE == 0) {
    fft_lds<T, N, P, ES, NT, -1>(z, s_tw);
    constexpr int K = N / 2 + 1;
    TO* const Sl = S + size_t(lev) * (DIM == 2 ? ns : size_t(N));  // uniform base, 32-bit offsets
    // items k = 0 .. N/2 - 1 of each sequence; the thread of k = 0 also takes
    // k = N/2 (both pair with themselves), so no pass runs for a few lanes
    constexpr int H = N / 2;
    for (int w = tid; w < H * P; w += NT) {
      const int p = w / H, k0 = w - (w / H) * H;
      const unsigned r0 = unsigned((DIM == 2 ? y0 + 2 * p : 2 * p) * N), r1 = r0 + N;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if (e == 1 && k0 != 0) break;
        const int k = e ? H : k0;
        T x1k, x2k, x1n, x2n;
        dct2_split(z[k * ES + p], z[((N - k) & (N - 1)) * ES + p], s_wq[k], s_wq[(N - k) & (N - 1)], x1k, x2k,
                   x1n, x2n);
        Sl[r0 + k] = TO(x1k);
        Sl[r1 + k] = TO(x2k);
        if (k > 0 && k < H) {
          Sl[r0 + N - k] = TO(x1n);
          Sl[r1 + N - k] = TO(x2n);
        }
      }
    }
  }
  // Partial sums of r^2.
  bool ismax[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) ismax[q] = false;
  block_reduce<NT, NV>(red, rsq, ismax);
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int slot = DIM == 2 ? b : lev + q;  // [level][block] (NBL = 1 in 1D)
      a.part[size_t(slot) * PART_STRIDE + PART_RSQ] = rsq[q];
    }
  }
  if (DIM == 2 && a.one_level) {
    // level 0 stands for every level: its partial goes to each level's slot
    for (int n = 1 + tid; n < a.nt; n += NT) a.part[(size_t(n) * NBL + b) * PART_STRIDE + PART_RSQ] = rsq[0];
  }
}

// ---------------------------------------------------------------------------
// a6 (x) + update.  Same blocks as k_rows_fwd.  delta = DCT-III along x of
// the RB rows of S; U += delta in FP64 (with a.bcast: U = u0 + delta); partial
// sums of delta^2, U^2, 3U^2 and max|delta| per [level][block].  MODE 1 writes
// delta (FP64) to dout instead of updating U.
template <typename T, int DIM, int N, int RB, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_rows_inv(UpdArgs a, const T* __restrict__ S, double* __restrict__ dout,
                                                  DctTables<T> dt) {
  if (a.done && *a.done) return;
  using Gm = rows_geom<DIM, N, RB>;
  constexpr int P = Gm::P, ES = Gm::ES, NBL = Gm::NBL;
  constexpr int NV = DIM == 2 ? 1 : RB;
  __shared__ __align__(16) cx<T> z[N * ES];
  __shared__ double red[NT * 4 * NV];
  __shared__ cx<T> s_tw[N], s_wi[N];
  table_to_lds<T, NT, N>(s_tw, dt.tw);
  table_to_lds<T, NT, N>(s_wi, dt.wi);
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int lev = DIM == 2 ? b / NBL : b * RB;
  const int y0 = DIM == 2 ? (b - (b / NBL) * NBL) * RB : 0;
  const size_t ns = DIM == 2 ? size_t(N) * N : size_t(N);
  constexpr int K = N / 2 + 1;
  // this block's first level (uniform base): every offset below is 32-bit
  const size_t lo = size_t(lev) * ns;
  const T* Sl = S + (DIM == 2 ? lo : size_t(lev) * N);
  double* Ul = a.U + lo;
  {
    // items k = 0 .. N/2 - 1 with their partners N - k; the thread of k = 0
    // also takes k = N/2 (its own partner)
    constexpr int H = N / 2, W = H * P, IT = cdiv_i(W, NT);
    T x1k[IT], x2k[IT], x1n[IT], x2n[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      x1k[i] = x2k[i] = x1n[i] = x2n[i] = T(0);
      if (W % NT == 0 || w < W) {
        const int p = w / H, k = w - (w / H) * H;
        const unsigned r0 = unsigned((DIM == 2 ? y0 + 2 * p : 2 * p) * N);
        const unsigned r1 = r0 + N;
        x1k[i] = Sl[r0 + k];
        x2k[i] = Sl[r1 + k];
        // k = 0 has no partner: its second pair of values is row N/2's
        x1n[i] = Sl[r0 + (k ? N - k : H)];
        x2n[i] = Sl[r1 + (k ? N - k : H)];
      }
    }
    __syncthreads();  // s_tw / s_wi complete
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (W % NT == 0 || w < W) {
        const int p = w / H, k = w - (w / H) * H;
        cx<T> zk, zn;
        if (k > 0) {
          dct3_join(x1k[i], x2k[i], x1n[i], x2n[i], s_wi[k], zk, zn);
          z[k * ES + p] = zk;
          z[(N - k) * ES + p] = zn;
        } else {
          dct3_join(x1k[i], x2k[i], T(0), T(0), s_wi[0], zk, zn);
          z[p] = zk;
          dct3_join(x1n[i], x2n[i], x1n[i], x2n[i], s_wi[H], zk, zn);
          z[H * ES + p] = zk;
        }
      }
    }
  }
  __syncthreads();
  fft_lds<T, N, P, ES, NT, +1>(z, s_tw);
  double acc[4 * NV];
#pragma unroll
  for (int q = 0; q < 4 * NV; ++q) acc[q] = 0.0;
  const T inv_n = T(1) / T(N);
  {
    constexpr int W = RB * N, IT = cdiv_i(W, NT);
    constexpr int BATCH = IT < 8 ? IT : 8;
#pragma unroll
    for (int i0 = 0; i0 < IT; i0 += BATCH) {
      double uo[BATCH];
#pragma unroll
      for (int q = 0; q < BATCH; ++q) {
        const int idx = tid + (i0 + q) * NT;
        uo[q] = 0.0;
        if (MODE == 0 && i0 + q < IT && (W % NT == 0 || idx < W)) {
          const int rr = idx / N, x = idx - (idx / N) * N;
          const int off = DIM == 2 ? (y0 + rr) * N + x : x;
          uo[q] = a.bcast ? a.u0[unsigned(off)] : Ul[unsigned(DIM == 2 ? off : rr * int(ns) + x)];
        }
      }
#pragma unroll
      for (int q = 0; q < BATCH; ++q) {
        const int idx = tid + (i0 + q) * NT;
        if (!(i0 + q < IT && (W % NT == 0 || idx < W))) continue;
        const int rr = idx / N, x = idx - (idx / N) * N;
        const double del = double(comp(z[dct_iperm<N>(x) * ES + (rr >> 1)], rr & 1) * inv_n);
        const unsigned gi = unsigned(DIM == 2 ? (y0 + rr) * N + x : rr * int(ns) + x);
        if (MODE == 1) {
          dout[lo + gi] = del;
          continue;
        }
        // unrefined mode: the iterate is an FP32 quantity, updated in FP32
        const double u = a.round32 ? double(float(uo[q]) + float(del)) : uo[q] + del;
        Ul[gi] = u;
#pragma unroll
        for (int qq = 0; qq < NV; ++qq) {
          if (DIM == 2 || qq == rr) {
            acc[4 * qq + 0] += del * del;
            acc[4 * qq + 1] += u * u;
            acc[4 * qq + 2] += 3.0 * u * u;
            const double ad = del < 0 ? -del : del;
            acc[4 * qq + 3] = (ad != ad || ad > acc[4 * qq + 3]) ? ad : acc[4 * qq + 3];
          }
        }
      }
    }
  }
  if (MODE == 1) return;
  bool ismax[4 * NV];
#pragma unroll
  for (int q = 0; q < 4 * NV; ++q) ismax[q] = (q % 4) == 3;
  block_reduce<NT, 4 * NV>(red, acc, ismax);
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int slot = DIM == 2 ? b : lev + q;
      double* pp = a.part + size_t(slot) * PART_STRIDE;
      pp[PART_DSQ] = acc[4 * q + 0];
      pp[PART_USQ] = acc[4 * q + 1];
      pp[PART_U2] = acc[4 * q + 2];
      pp[PART_DMAX] = acc[4 * q + 3];
    }
  }
}

// ---------------------------------------------------------------------------
// a2 (y) forward / a6 (y) inverse: orthonormal DCT-II / DCT-III along y of a
// tile of XB columns of one level, from Sin (type T) to Sout (type TO; the
// same array when TO == T: the tile is read completely before it is written).  Columns 2c and 2c+1 are
// packed into one complex sequence; consecutive threads take consecutive c.
// PANEL: the spectral side (output of the forward, input of the inverse) is
// stored in panels of 2^tps modes; the other side is plain [level][mode].
template <bool PANEL, int N>
__device__ __forceinline__ size_t spec_off(int lev, int q, int tps, int nlev) {
  if constexpr (PANEL) return panel_index(lev, q, tps, nlev);
  else return size_t(lev) * (N * N) + q;
}

template <typename T, typename TO, int N, int XB, int NT, bool INV, bool PANEL>
__global__ __launch_bounds__(NT) void k_cols(const T* Sin, TO* Sout, const int* __restrict__ done,
                                              DctTables<T> dt, int tps, int nlev) {
  if (done && *done) return;
  constexpr int C = XB / 2, ES = C, NBX = N / XB, K = N / 2 + 1;
  __shared__ __align__(16) cx<T> z[N * ES];
  __shared__ cx<T> s_tw[N], s_w[N];
  table_to_lds<T, NT, N>(s_tw, dt.tw);
  table_to_lds<T, NT, N>(s_w, INV ? dt.wi : dt.wq);
  const int tid = threadIdx.x;
  // Tiles narrower than a 128-byte line share lines with their neighbours:
  // give each XCD (workgroups are dealt to the 8 XCDs round-robin) a
  // contiguous range of tiles so that shared lines go through one L2.
  const int nb = gridDim.x;
  constexpr bool NARROW = XB * int(sizeof(TO)) < 128 || XB * int(sizeof(T)) < 128;
  const int blk = (NARROW && (nb & 7) == 0) ? int(blockIdx.x & 7) * (nb >> 3) + int(blockIdx.x >> 3)
                                            : int(blockIdx.x);
  const int lev = blk / NBX;
  const int x0 = (blk - lev * NBX) * XB;
  // element (lev, q = row N + x); a pair (q, q + 1), q even, is contiguous in
  // both layouts
  const T* base = Sin + size_t(lev) * N * N + x0;
  TO* obase = Sout + size_t(lev) * N * N + x0;
  // FP32 sides move two complex values (four columns, 16 bytes) per access
  constexpr bool V2I = sizeof(T) == 4 && C % 2 == 0, V2O = sizeof(TO) == 4 && C % 2 == 0;
  constexpr int C2 = C / 2;
  if (!INV) {
    if constexpr (V2I) {
      constexpr int W = N * C2, IT = cdiv_i(W, NT);
      float4 x[IT];
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        if (W % NT == 0 || w < W) {
          const int m = w / C2, c = w - (w / C2) * C2;
          x[i] = *reinterpret_cast<const float4*>(base + size_t(dct_perm<N>(m)) * N + 4 * c);
        }
      }
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        if (W % NT == 0 || w < W) {
          const int m = w / C2, c = w - (w / C2) * C2;
          *reinterpret_cast<float4*>(z + m * ES + 2 * c) = x[i];
        }
      }
    } else {
      constexpr int W = N * C, IT = cdiv_i(W, NT);
      cx<T> x[IT];
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        if (W % NT == 0 || w < W) {
          const int m = w / C, c = w - (w / C) * C;
          x[i] = *reinterpret_cast<const cx<T>*>(base + size_t(dct_perm<N>(m)) * N + 2 * c);
        }
      }
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        if (W % NT == 0 || w < W) z[(w / C) * ES + (w - (w / C) * C)] = x[i];
      }
    }
    __syncthreads();
    fft_lds<T, N, C, ES, NT, -1>(z, s_tw);
    if constexpr (V2O) {
      for (int w = tid; w < K * C2; w += NT) {
        const int k = w / C2, c = 2 * (w - (w / C2) * C2);
        const int kn = (N - k) & (N - 1);
        T a1k, a2k, a1n, a2n, b1k, b2k, b1n, b2n;
        dct2_split(z[k * ES + c], z[kn * ES + c], s_w[k], s_w[kn], a1k, a2k, a1n, a2n);
        dct2_split(z[k * ES + c + 1], z[kn * ES + c + 1], s_w[k], s_w[kn], b1k, b2k, b1n, b2n);
        *reinterpret_cast<float4*>(Sout + spec_off<PANEL, N>(lev, k * N + x0 + 2 * c, tps, nlev)) =
            make_float4(float(a1k), float(a2k), float(b1k), float(b2k));
        if (k > 0 && k < N / 2)
          *reinterpret_cast<float4*>(Sout + spec_off<PANEL, N>(lev, kn * N + x0 + 2 * c, tps, nlev)) =
              make_float4(float(a1n), float(a2n), float(b1n), float(b2n));
      }
    } else {
      for (int w = tid; w < K * C; w += NT) {
        const int k = w / C, c = w - (w / C) * C;
        T x1k, x2k, x1n, x2n;
        dct2_split(z[k * ES + c], z[((N - k) & (N - 1)) * ES + c], s_w[k], s_w[(N - k) & (N - 1)], x1k, x2k,
                   x1n, x2n);
        *reinterpret_cast<cx<TO>*>(Sout + spec_off<PANEL, N>(lev, k * N + x0 + 2 * c, tps, nlev)) =
            mk(TO(x1k), TO(x2k));
        if (k > 0 && k < N / 2)
          *reinterpret_cast<cx<TO>*>(Sout + spec_off<PANEL, N>(lev, (N - k) * N + x0 + 2 * c, tps, nlev)) =
              mk(TO(x1n), TO(x2n));
      }
    }
  } else {
    if constexpr (V2I) {
      constexpr int W = K * C2, IT = cdiv_i(W, NT);
      float4 xk[IT], xn[IT];
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        xk[i] = xn[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (w < W) {
          const int k = w / C2, c = 2 * (w - (w / C2) * C2);
          xk[i] = *reinterpret_cast<const float4*>(Sin + spec_off<PANEL, N>(lev, k * N + x0 + 2 * c, tps, nlev));
          if (k)
            xn[i] = *reinterpret_cast<const float4*>(Sin + spec_off<PANEL, N>(lev, (N - k) * N + x0 + 2 * c, tps, nlev));
        }
      }
      __syncthreads();  // s_tw / s_w complete
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        if (w < W) {
          const int k = w / C2, c = 2 * (w - (w / C2) * C2);
          cx<T> ak, an, bk, bn;
          dct3_join(T(xk[i].x), T(xk[i].y), T(xn[i].x), T(xn[i].y), s_w[k], ak, an);
          dct3_join(T(xk[i].z), T(xk[i].w), T(xn[i].z), T(xn[i].w), s_w[k], bk, bn);
          *reinterpret_cast<float4*>(z + k * ES + c) = make_float4(ak.x, ak.y, bk.x, bk.y);
          if (k > 0 && k < N / 2) *reinterpret_cast<float4*>(z + (N - k) * ES + c) = make_float4(an.x, an.y, bn.x, bn.y);
        }
      }
    } else {
      constexpr int W = K * C, IT = cdiv_i(W, NT);
      cx<T> xk[IT], xn[IT];
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        xk[i] = xn[i] = mk(T(0), T(0));
        if (w < W) {
          const int k = w / C, c = w - (w / C) * C;
          xk[i] = *reinterpret_cast<const cx<T>*>(Sin + spec_off<PANEL, N>(lev, k * N + x0 + 2 * c, tps, nlev));
          if (k) xn[i] = *reinterpret_cast<const cx<T>*>(Sin + spec_off<PANEL, N>(lev, (N - k) * N + x0 + 2 * c, tps, nlev));
        }
      }
      __syncthreads();  // s_tw / s_w complete
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int w = tid + i * NT;
        if (w < W) {
          const int k = w / C, c = w - (w / C) * C;
          cx<T> zk, zn;
          dct3_join(xk[i].x, xk[i].y, xn[i].x, xn[i].y, s_w[k], zk, zn);
          z[k * ES + c] = zk;
          if (k > 0 && k < N / 2) z[(N - k) * ES + c] = zn;
        }
      }
    }
    __syncthreads();
    fft_lds<T, N, C, ES, NT, +1>(z, s_tw);
    const T inv_n = T(1) / T(N);
    if constexpr (V2O) {
      for (int w = tid; w < N * C2; w += NT) {
        const int m = w / C2, c = 2 * (w - (w / C2) * C2);
        const cx<T> v = scale(z[m * ES + c], inv_n), u = scale(z[m * ES + c + 1], inv_n);
        *reinterpret_cast<float4*>(obase + size_t(dct_perm<N>(m)) * N + 2 * c) =
            make_float4(float(v.x), float(v.y), float(u.x), float(u.y));
      }
    } else {
      for (int w = tid; w < N * C; w += NT) {
        const int m = w / C, c = w - (w / C) * C;
        const cx<T> v = scale(z[m * ES + c], inv_n);
        *reinterpret_cast<cx<TO>*>(obase + size_t(dct_perm<N>(m)) * N + 2 * c) = mk(TO(v.x), TO(v.y));
      }
    }
  }
}

// Stand-alone x-DCT of RB rows (stage entry point): plain copy in, DCT, out.
template <typename T, int DIM, int N, int RB, int NT, bool INV>
__global__ __launch_bounds__(NT) void k_rows_dct(const T* __restrict__ in, T* __restrict__ out, DctTables<T> dt) {
  using Gm = rows_geom<DIM, N, RB>;
  constexpr int P = Gm::P, ES = Gm::ES, K = N / 2 + 1;
  __shared__ __align__(16) cx<T> z[N * ES];
  const int tid = threadIdx.x;
  const size_t row0 = size_t(blockIdx.x) * RB;  // rows are contiguous in both 1D and 2D layouts
  if (!INV) {
    for (int idx = tid; idx < RB * N; idx += NT) {
      const int rr = idx / N, x = idx - (idx / N) * N;
      comp(z[dct_iperm<N>(x) * ES + (rr >> 1)], rr & 1) = in[(row0 + rr) * N + x];
    }
    __syncthreads();
    fft_lds<T, N, P, ES, NT, -1>(z, dt.tw);
    for (int w = tid; w < K * P; w += NT) {
      const int p = w / K, k = w - (w / K) * K;
      T x1k, x2k, x1n, x2n;
      dct2_split(z[k * ES + p], z[((N - k) & (N - 1)) * ES + p], dt.wq[k], dt.wq[(N - k) & (N - 1)], x1k, x2k,
                 x1n, x2n);
      const size_t r0 = (row0 + 2 * p) * N, r1 = r0 + N;
      out[r0 + k] = x1k;
      out[r1 + k] = x2k;
      if (k > 0 && k < N / 2) {
        out[r0 + N - k] = x1n;
        out[r1 + N - k] = x2n;
      }
    }
  } else {
    for (int w = tid; w < K * P; w += NT) {
      const int p = w / K, k = w - (w / K) * K;
      const size_t r0 = (row0 + 2 * p) * N, r1 = r0 + N;
      cx<T> zk, zn;
      dct3_join(in[r0 + k], in[r1 + k], k ? in[r0 + N - k] : T(0), k ? in[r1 + N - k] : T(0), dt.wi[k], zk, zn);
      z[k * ES + p] = zk;
      if (k > 0 && k < N / 2) z[(N - k) * ES + p] = zn;
    }
    __syncthreads();
    fft_lds<T, N, P, ES, NT, +1>(z, dt.tw);
    const T inv_n = T(1) / T(N);
    for (int idx = tid; idx < RB * N; idx += NT) {
      const int rr = idx / N, x = idx - (idx / N) * N;
      out[(row0 + rr) * N + x] = comp(z[dct_iperm<N>(x) * ES + (rr >> 1)], rr & 1) * inv_n;
    }
  }
}

// ---------------------------------------------------------------------------
// a3-a5.  One workgroup per tile of M consecutive spatial modes k (M even):
// the M real sequences over time are scaled by a^j, packed into M/2 complex
// ones, transformed together, split into their Hermitian halves, divided by
//   sigma_{l,k} = lambda1_l + p_l lam_k + q_l lam_k^2,   l = 0..N_t/2,
// (p_l = pco_l - c_bar for the CH operators), re-packed, transformed back and
// scaled by a^{-j}/N_t.
// LDS in FP64: the tile with one padding row after every 8 (the first FFT
// stage writes rows 8 apart, which would otherwise hit the same banks) and
// the twiddles as products of two short tables (indexed by m / 32 and
// m mod 32), which leaves room for a third block per CU at N_t = 1024 than
// the full table (measured 1.96 -> 1.69 ms at 512^2 x 1024).  In FP32 the
// plain tile and the full table measured fastest.  Both use radix-16 stages
// (16 x 16 x 4 at N_t = 1024: FP32 0.68 -> 0.65 ms, FP64 1.27 -> 1.16 ms).
// Minimum waves per SIMD asked of the compiler: the FP32 tile of 8 modes x
// 1024 levels (40 KB of LDS) fits four 512-thread blocks per CU when the
// kernel holds 64 registers (it takes 69 unconstrained, three blocks; no
// spills at 64): C5 FP32 time solve 642 -> 609 us, mixed 574 -> 550 us.
template <typename T, int NTT, int M>
constexpr int time_solve_min_waves() {
  return (sizeof(T) == 4 && NTT == 1024 && M == 8) ? 8 : 1;
}

template <typename T, int NTT, int M, int NT>
__global__ __launch_bounds__(NT, (time_solve_min_waves<T, NTT, M>())) void k_time_solve(T* __restrict__ S,
                                                                                         TimeArgs<T> ta) {
  if (ta.done && *ta.done) return;
  constexpr int C = M / 2;
  constexpr bool F64 = sizeof(T) == 8;
  constexpr bool SK = F64 && NTT >= 8;
  constexpr int NLO = NTT < 32 ? NTT : 32, NHI = NTT < 32 ? 1 : NTT / 32;
  __shared__ __align__(16) cx<T> z[zrows<SK>(NTT) * C];
  __shared__ cx<T> s_lo[F64 ? NLO : 1];
  __shared__ cx<T> s_hi[F64 ? NHI : 1];
  __shared__ cx<T> s_tw[F64 ? 1 : NTT];
  const int tid = threadIdx.x;
  if constexpr (F64) {
    for (int i = tid; i < NLO + NHI; i += NT) {
      if (i < NLO) s_lo[i] = ta.tw[i];
      else s_hi[i - NLO] = ta.tw[32 * (i - NLO)];
    }
  } else {
    table_to_lds<T, NT, NTT>(s_tw, ta.tw);
  }
  auto twiddles = [&]() {
    if constexpr (F64) return TwSplit<T>{s_hi, s_lo};
    else return TwTable<T>{s_tw};
  };
  const auto tws = twiddles();
  // In a panel wider than the tile, tiles narrower than a 128-byte line
  // share lines with their neighbours.  Workgroups are dealt to the 8 XCDs
  // round-robin; this order gives XCD x the contiguous range of tiles
  // [x B/8, (x+1) B/8) (B tiles), so the tiles sharing a line read it through
  // one L2.  With panels of one tile each tile is a contiguous N_t x M block.
  const int nb = gridDim.x;
  const int tp = 1 << ta.tps;
  const int tile = (tp > M && M * int(sizeof(T)) < 128 && (nb & 7) == 0)
                       ? int(blockIdx.x & 7) * (nb >> 3) + int(blockIdx.x >> 3)
                       : int(blockIdx.x);
  const int col0 = tile * M;
  // level j of this tile's modes starts at Sb + j * tp
  T* const Sb = S + (size_t(col0 >> ta.tps) * NTT << ta.tps) + (col0 & (tp - 1));
  const size_t rs = size_t(tp);
  constexpr int W = NTT * C, IT = cdiv_i(W, NT);
  // FP32: two complex values (16 bytes) per load and store
  constexpr bool V2 = std::is_same<T, float>::value && C % 2 == 0;
  constexpr int W2 = W / 2, IT2 = cdiv_i(W2, NT), C2 = C / 2;
  if constexpr (V2) {
    float4 x[IT2];
#pragma unroll
    for (int i = 0; i < IT2; ++i) {
      const int w = tid + i * NT;
      if (W2 % NT == 0 || w < W2) {
        const int j = w / C2, c = w - (w / C2) * C2;
        x[i] = *reinterpret_cast<const float4*>(Sb + (ta.bcast_in ? 0 : j * rs) + 4 * c);
      }
    }
#pragma unroll
    for (int i = 0; i < IT2; ++i) {
      const int w = tid + i * NT;
      if (W2 % NT == 0 || w < W2) {
        const int j = w / C2, c = w - (w / C2) * C2;
        const T s = ta.aj[j];
        cx<T>* zr = z + zrow<SK>(j) * C + 2 * c;
        zr[0] = scale(mk(T(x[i].x), T(x[i].y)), s);
        zr[1] = scale(mk(T(x[i].z), T(x[i].w)), s);
      }
    }
  } else {
    // issue every load of the tile before using any (latency hiding)
    cx<T> x[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (W % NT == 0 || w < W) {
        const int j = w / C, c = w - (w / C) * C;
        x[i] = *reinterpret_cast<const cx<T>*>(Sb + (ta.bcast_in ? 0 : j * rs) + 2 * c);
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (W % NT == 0 || w < W) {
        const int j = w / C, c = w - (w / C) * C;
        z[zrow<SK>(j) * C + c] = scale(x[i], ta.aj[j]);
      }
    }
  }
  __syncthreads();
  fft_lds_tw<T, NTT, C, C, NT, -1, SK, true>(z, tws);
  constexpr int WD = (NTT / 2 + 1) * C, ITD = cdiv_i(WD, NT);
  static_assert(NT % C == 0, "a thread keeps one mode pair c");
  // the mode pair of every item of this thread (NT is a multiple of C)
  const int c = tid % C;
  const int k1 = col0 + 2 * c, k2 = k1 + 1;
  const T lk1 = ta.lamx[k1 % ta.nx] + ta.lamy[k1 / ta.nx];
  const T lk2 = ta.lamx[k2 % ta.nx] + ta.lamy[k2 / ta.nx];
  const T lk1s = lk1 * lk1, lk2s = lk2 * lk2;
  const double cbd = ta.cbar_mode ? (ta.cbar ? *ta.cbar : ta.cbar_val) : 0.0;
  const T cb = T(cbd);
  // FP64: the level coefficients of every item of this thread, loaded
  // together (their latency was exposed otherwise); FP32 loads them where
  // they are used, which saves registers (C3 256 x 32 tile: 130 -> 99)
  cx<T> l1v[ITD], plv[ITD], qlv[ITD];
#pragma unroll
  for (int i = 0; i < (F64 ? ITD : 0); ++i) {
    const int w = tid + i * NT;
    const int l = w < WD ? w / C : 0;
    l1v[i] = ta.lam1[l];
    plv[i] = ta.pco[l];
    qlv[i] = ta.qco[l];
  }
#pragma unroll
  for (int i = 0; i < ITD; ++i) {
    const int w = tid + i * NT;
    if (w >= WD) continue;
    const int l = w / C;
    const int m = (NTT - l) & (NTT - 1);
    const cx<T> zl = z[zrow<SK>(l) * C + c];
    const cx<T> zm = conj(z[zrow<SK>(m) * C + c]);
    const cx<T> x1 = scale(add(zl, zm), T(0.5));
    const cx<T> x2 = scale(mul_mi(sub(zl, zm)), T(0.5));
    const cx<T> l1 = F64 ? l1v[i] : ta.lam1[l];
    const cx<T> pl0 = F64 ? plv[i] : ta.pco[l];
    const cx<T> ql = F64 ? qlv[i] : ta.qco[l];
    const cx<T> pl = mk(pl0.x - cb, pl0.y);
    const cx<T> s1 = mk(l1.x + pl.x * lk1 + ql.x * lk1s, l1.y + pl.y * lk1 + ql.y * lk1s);
    const cx<T> s2 = mk(l1.x + pl.x * lk2 + ql.x * lk2s, l1.y + pl.y * lk2 + ql.y * lk2s);
    const cx<T> y1 = cdiv_fast(x1, s1);
    const cx<T> y2 = cdiv_fast(x2, s2);
    z[zrow<SK>(l) * C + c] = add(y1, mul_i(y2));
    if (m != l) z[zrow<SK>(m) * C + c] = add(conj(y1), mul_i(conj(y2)));
  }
  __syncthreads();
  fft_lds_tw<T, NTT, C, C, NT, +1, SK, true>(z, tws);
  if constexpr (V2) {
#pragma unroll
    for (int i = 0; i < IT2; ++i) {
      const int w = tid + i * NT;
      if (W2 % NT == 0 || w < W2) {
        const int j = w / C2, c = w - (w / C2) * C2;
        const T s = ta.aij[j];
        const cx<T>* zr = z + zrow<SK>(j) * C + 2 * c;
        const cx<T> a = scale(zr[0], s), b = scale(zr[1], s);
        *reinterpret_cast<float4*>(Sb + j * rs + 4 * c) = make_float4(a.x, a.y, b.x, b.y);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int w = tid + i * NT;
      if (W % NT == 0 || w < W) {
        const int j = w / C, c = w - (w / C) * C;
        *reinterpret_cast<cx<T>*>(Sb + j * rs + 2 * c) = scale(z[zrow<SK>(j) * C + c], ta.aij[j]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// a7.  One workgroup: per level, sum the block partials; then max over levels
//   upd  = max_n ||delta_n||_2,  unrm = max_n ||u_n||_2,  rel = upd / unrm
//   rho  = upd_k / upd_{k-1};  est = rho/(1-rho) * rel
// stop when est <= safety * rtol (k >= 2, rho < 1) and the FP64 residual
// norm max_n ||r_n||_2 has not grown over the last sweep, or rel <= 1e-3 rtol;
// diverged on NaN/Inf or when the update grows 1e3-fold over the first one.
// The scalar averaged Jacobian for the next time solve is mean(3 u^2).
// Control-record fields the stop rule reads, loaded by thread 0 before the
// reduction so that their latency overlaps it.
struct CtrlPrev {
  int iter;
  double upd_prev, upd_first;
};

template <int NT>
__device__ void finalize_levels_grouped(const FinArgs& f, double (&v)[4], int lbeg, int lend);
template <int NT>
__device__ void finalize_control(const FinArgs& f, double* red, double (&v)[4], const CtrlPrev& c0);

template <int NT>
__device__ void finalize_body(const FinArgs& f, double* red) {
  CtrlPrev c0{0, 0.0, 0.0};
  if (threadIdx.x == 0) {
    c0.iter = f.ctrl->iter;
    c0.upd_prev = f.ctrl->upd_prev;
    c0.upd_first = f.ctrl->upd_first;
  }
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // max dsq, max usq, sum u2, max rsq
  if constexpr (NT <= 256) {
    // few partials: one thread per level, its block partials in order
    for (int n = threadIdx.x; n < f.nt; n += NT) {
      double dsq = 0.0, usq = 0.0, u2 = 0.0, rsq = 0.0;
      for (int bb = 0; bb < f.nbl; ++bb) {
        const double* pp = f.part + (size_t(n) * f.nbl + bb) * PART_STRIDE;
        dsq += pp[PART_DSQ];
        usq += pp[PART_USQ];
        u2 += pp[PART_U2];
      }
      for (int bb = 0; bb < f.nbl_f; ++bb) rsq += f.part[(size_t(n) * f.nbl_f + bb) * PART_STRIDE + PART_RSQ];
      v[0] = (dsq != dsq || dsq > v[0]) ? dsq : v[0];
      v[1] = (usq != usq || usq > v[1]) ? usq : v[1];
      v[2] += u2;
      v[3] = (rsq != rsq || rsq > v[3]) ? rsq : v[3];
    }
  } else {
    finalize_levels_grouped<NT>(f, v, 0, f.nt);
  }
  finalize_control<NT>(f, red, v, c0);
}

// Many partials: a group of g lanes (g = the power of two >= the blocks per
// level, at most 64) reads one level's block partials together, several
// levels per wave and FL levels per lane in flight, and combines them with a
// fixed xor-shuffle tree, so every sum is formed in the same order each run.
template <int NT>
__device__ void finalize_levels_grouped(const FinArgs& f, double (&v)[4], int lbeg, int lend) {
  constexpr int NW = NT / 64, FL = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gmax = f.nbl > f.nbl_f ? f.nbl : f.nbl_f;
  int g = 1;
  while (g < gmax && g < 64) g <<= 1;
  const int lpw = 64 / g;  // levels per wave per step
  const int sub = lane / g, j = lane - (lane / g) * g;  // v: group leaders accumulate
  for (int base = lbeg + wave * lpw; base < lend; base += NW * lpw * FL) {
    double s[FL][4];
#pragma unroll
    for (int u = 0; u < FL; ++u) {
      const int n = base + u * NW * lpw + sub;
      s[u][0] = s[u][1] = s[u][2] = s[u][3] = 0.0;
      if (n < lend) {
        for (int bb = j; bb < f.nbl; bb += g) {
          const double* pp = f.part + (size_t(n) * f.nbl + bb) * PART_STRIDE;
          s[u][0] += pp[PART_DSQ];
          s[u][1] += pp[PART_USQ];
          s[u][2] += pp[PART_U2];
        }
        // the forward pass has its own block grid (same slots, its own field)
        for (int bb = j; bb < f.nbl_f; bb += g) s[u][3] += f.part[(size_t(n) * f.nbl_f + bb) * PART_STRIDE + PART_RSQ];
      }
    }
#pragma unroll
    for (int u = 0; u < FL; ++u) {
      for (int off = g >> 1; off > 0; off >>= 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) s[u][q] += __shfl_xor(s[u][q], off, 64);
      const int n = base + u * NW * lpw + sub;
      if (j == 0 && n < lend) {
        v[0] = (s[u][0] != s[u][0] || s[u][0] > v[0]) ? s[u][0] : v[0];
        v[1] = (s[u][1] != s[u][1] || s[u][1] > v[1]) ? s[u][1] : v[1];
        v[2] += s[u][2];
        v[3] = (s[u][3] != s[u][3] || s[u][3] > v[3]) ? s[u][3] : v[3];
      }
    }
  }
}

// Reduction over threads and the stop rule (thread 0).
template <int NT>
__device__ void finalize_control(const FinArgs& f, double* red, double (&v)[4], const CtrlPrev& c0) {
  const bool ismax[4] = {true, true, false, true};
  block_reduce_waves<NT, 4>(red, v, ismax);
  if (threadIdx.x != 0) return;
  Ctrl* c = f.ctrl;
  const double upd = sqrt(v[0]), unrm = sqrt(v[1]), res = sqrt(v[3]);
  const double cbar = v[2] / f.dof;
  const int k = c0.iter;  // 0-based index of the iteration just finished
  const double rel = unrm > 0.0 ? upd / unrm : upd;
  if (k < PINT_HIST_DEV) {
    c->upd_hist[k] = rel;
    c->res_hist[k] = res;
  }
  c->iter = k + 1;
  c->c_bar = cbar;
  StopIn si;
  si.k = k;
  si.upd = upd;
  si.unrm = unrm;
  si.res = res;
  si.cbar = cbar;
  si.upd_prev = c0.upd_prev;
  si.upd_first = c0.upd_first;
  si.res_prev = (k >= 1 && k - 1 < PINT_HIST_DEV) ? c->res_hist[k - 1] : -1.0;
  si.rtol = f.rtol;
  si.safety = f.safety;
  si.stagnate = f.stagnate;
  si.max_iter = f.max_iter;
  const StopOut so = stop_rule(si);
  const double est = so.est;
  c->est = est;
  if (k == 0) c->upd_first = upd;
  c->upd_prev = upd;
  if (so.done) {
    c->status = so.status;
    c->done = 1;
  }
  if (f.host) {
    // status mirror in pinned host memory: read by the host after the stream
    // synchronizes, so no device-to-host copy is needed per check
    Ctrl* h = f.host;
    if (k < PINT_HIST_DEV) {
      h->upd_hist[k] = rel;
      h->res_hist[k] = res;
    }
    h->iter = k + 1;
    h->c_bar = cbar;
    h->est = est;
    h->status = c->status;
    h->done = c->done;
  }
}

// Stand-alone control kernel (one workgroup), used when the update kernel
// does not run it itself.
// One workgroup: 256 threads when the partials are few (its fixed cost is
// lower), 1024 when there are many to stream (N_t x blocks per level large).
template <int NT>
__global__ __launch_bounds__(NT) void k_finalize(FinArgs f) {
  if (f.ctrl->done) return;
  __shared__ double red[4 * (NT / 64)];
  finalize_body<NT>(f, red);
}
constexpr int FIN_WIDE_SLOTS = 16384;

// Many partials: first many workgroups, each reducing the block partials of
// FIN_LEVELS consecutive levels to (max dsq, max usq, sum u2, max rsq) in
// f.fin[group][4]; then one workgroup combines the groups in index order and
// runs the stop rule.  Every sum keeps a fixed order.
constexpr int FIN_LEVELS = 4;
__global__ __launch_bounds__(256) void k_fin_levels(FinArgs f) {
  if (f.ctrl->done) return;
  __shared__ double red[4 * 4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int l0 = blockIdx.x * FIN_LEVELS;
  finalize_levels_grouped<256>(f, v, l0, min(l0 + FIN_LEVELS, f.nt));
  const bool ismax[4] = {true, true, false, true};
  block_reduce_waves<256, 4>(red, v, ismax);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) f.fin[size_t(blockIdx.x) * 4 + q] = v[q];
  }
}

__global__ __launch_bounds__(64) void k_finalize_groups(FinArgs f, int groups) {
  if (f.ctrl->done) return;
  __shared__ double red[4];
  CtrlPrev c0{0, 0.0, 0.0};
  if (threadIdx.x == 0) {
    c0.iter = f.ctrl->iter;
    c0.upd_prev = f.ctrl->upd_prev;
    c0.upd_first = f.ctrl->upd_first;
  }
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < groups; g += 64) {
    const double* p = f.fin + size_t(g) * 4;
    v[0] = (p[0] != p[0] || p[0] > v[0]) ? p[0] : v[0];
    v[1] = (p[1] != p[1] || p[1] > v[1]) ? p[1] : v[1];
    v[2] += p[2];
    v[3] = (p[3] != p[3] || p[3] > v[3]) ? p[3] : v[3];
  }
  finalize_control<64>(f, red, v, c0);
}

// Control record reset and the first iteration's c_bar = mean(3 u^2) of the
// initial guess (CH operators only): k_init_part writes workgroup partial
// sums of 3 u^2 over u0 (broadcast guess) or over U, k_init_ctrl adds them
// in a fixed order.
constexpr int INIT_CHUNK = 4096;  // values per workgroup of k_init_part

__global__ __launch_bounds__(256) void k_init_part(InitArgs a) {
  constexpr int NT = 256, PER = INIT_CHUNK / NT;
  __shared__ double red[NT];
  const double* src = a.broadcast ? a.u0 : a.U;
  const size_t total = a.broadcast ? size_t(a.ns) : size_t(a.ns) * a.nt;
  const size_t base = size_t(blockIdx.x) * INIT_CHUNK;
  double x[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const size_t j = base + threadIdx.x + size_t(i) * NT;
    x[i] = j < total ? src[j] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < PER; ++i) s += 3.0 * x[i] * x[i];
  double v[1] = {s};
  const bool ismax[1] = {false};
  block_reduce<NT, 1>(red, v, ismax);
  if (threadIdx.x == 0) a.part[size_t(blockIdx.x) * PART_STRIDE + PART_U2] = v[0];
}

__global__ __launch_bounds__(256) void k_init_ctrl(Ctrl* c, Ctrl* host, InitArgs a, double dof, int nparts) {
  constexpr int NT = 256;
  __shared__ double red[NT];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) s += a.part[size_t(i) * PART_STRIDE + PART_U2];
  double v[1] = {s};
  const bool ismax[1] = {false};
  block_reduce<NT, 1>(red, v, ismax);
  if (threadIdx.x != 0) return;
  c->iter = 0;
  c->done = 0;
  c->status = PINT_ENOCONV;
  c->c_bar = nparts ? (a.broadcast ? v[0] / a.ns : v[0] / dof) : 0.0;
  c->upd_prev = 0.0;
  c->upd_first = 0.0;
  c->est = 1e300;
  if (host) {
    host->iter = 0;
    host->done = 0;
    host->status = PINT_ENOCONV;
    host->c_bar = c->c_bar;
  }
}

// ------------------------------------------------------------- stage I/O
template <typename TI, typename TO>
__global__ void k_cast(const TI* __restrict__ in, TO* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    out[i] = TO(in[i]);
}

// Per-level mass and Ginzburg-Landau energy (FP64).  One workgroup per level.
__global__ __launch_bounds__(256) void k_diagnostics(DiagArgs a) {
  constexpr int NT = 256;
  __shared__ double red[2 * NT];
  const int n = blockIdx.x;
  const double* u = a.U + size_t(n) * a.ns;
  double m = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < a.ns; i += NT) {
    const int x = i % a.nx, y = i / a.nx;
    const double v = u[i];
    m += v;
    const double w = v * v - 1.0;
    e += 0.25 * w * w;
    double gsq = 0.0;
    if (x + 1 < a.nx) {
      const double dd = u[i + 1] - v;
      gsq += dd * dd;
    }
    if (a.dim == 2 && y + 1 < a.nx) {
      const double dd = u[i + a.nx] - v;
      gsq += dd * dd;
    }
    e += 0.5 * a.eps2 * gsq * a.inv_h2;
  }
  double v[2] = {m, e};
  const bool ismax[2] = {false, false};
  block_reduce<NT, 2>(red, v, ismax);
  if (threadIdx.x == 0) {
    a.mass[n] = v[0] * a.hd;
    a.energy[n] = v[1] * a.hd;
  }
}

// Invariants of a converged solve: block b computes the mass, the energy and
// h^d sum |u| of level b (b = 0: the datum u0, b >= 1: u_b); then one
// workgroup forms max_n |M_n - M_0| / (h^d sum |u_0|) and checks that the
// energy never rises by more than 1e-13 of its previous value.
__global__ __launch_bounds__(256) void k_invariants(DiagArgs a, const double* __restrict__ u0,
                                                     double* __restrict__ out) {
  constexpr int NT = 256;
  __shared__ double red[3 * NT];
  const int lev = blockIdx.x;
  const double* u = lev == 0 ? u0 : a.U + size_t(lev - 1) * a.ns;
  double m = 0.0, e = 0.0, ab = 0.0;
  for (int i = threadIdx.x; i < a.ns; i += NT) {
    const int x = i % a.nx, y = i / a.nx;
    const double v = u[i];
    m += v;
    ab += v < 0 ? -v : v;
    const double w = v * v - 1.0;
    e += 0.25 * w * w;
    double gsq = 0.0;
    if (x + 1 < a.nx) {
      const double dd = u[i + 1] - v;
      gsq += dd * dd;
    }
    if (a.dim == 2 && y + 1 < a.nx) {
      const double dd = u[i + a.nx] - v;
      gsq += dd * dd;
    }
    e += 0.5 * a.eps2 * gsq * a.inv_h2;
  }
  double v[3] = {m, e, ab};
  const bool ismax[3] = {false, false, false};
  block_reduce<NT, 3>(red, v, ismax);
  if (threadIdx.x == 0) {
    out[3 * lev + 0] = v[0] * a.hd;
    out[3 * lev + 1] = v[1] * a.hd;
    out[3 * lev + 2] = v[2] * a.hd;
  }
}

__global__ __launch_bounds__(256) void k_invariants_fin(const double* __restrict__ in, int nt, int energy, Ctrl* c,
                                                         Ctrl* host) {
  constexpr int NT = 256;
  __shared__ double red[2 * NT];
  const double m0 = in[0];
  double drift = 0.0, bad = 0.0;
  for (int n = 1 + int(threadIdx.x); n <= nt; n += NT) {
    const double d = fabs(in[3 * n] - m0);
    drift = (d != d || d > drift) ? d : drift;
    const double ep = in[3 * (n - 1) + 1], en = in[3 * n + 1];
    if (!(en <= ep + 1e-13 * fabs(ep))) bad += 1.0;
  }
  double v[2] = {drift, bad};
  const bool ismax[2] = {true, false};
  block_reduce<NT, 2>(red, v, ismax);
  if (threadIdx.x != 0) return;
  const double scale = in[2];
  const double md = scale > 0.0 ? v[0] / scale : __longlong_as_double(0x7ff8000000000000ll);
  const int ok = energy ? (v[1] == 0.0 ? 1 : 0) : -1;
  c->mass_drift = md;
  c->energy_ok = ok;
  if (host) {
    host->mass_drift = md;
    host->energy_ok = ok;
  }
}

// ------------------------------------------- space-varying averaged Jacobian
// j(x) = (1/N_t) sum_n 3 u_n(x)^2 (eq. approx_jacobian): one thread per point,
// levels summed in order.
__global__ __launch_bounds__(256) void k_jfield(const double* __restrict__ U, double* __restrict__ j, int nt,
                                                 int ns) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ns) return;
  double s = 0.0;
  for (int n = 0; n < nt; ++n) {
    const double u = U[size_t(n) * ns + i];
    s += 3.0 * u * u;
  }
  j[i] = s / nt;
}

__global__ __launch_bounds__(256) void k_axpbypcz(double* __restrict__ out, double a, const double* __restrict__ x,
                                                   double b, const double* __restrict__ y, double c,
                                                   const double* __restrict__ z, size_t n) {
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
    double v = a * x[i] + b * y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

// Fixed-order partial dot products: block b sums i = b*256 + t + k*DOT_BLOCKS*256.
struct DotPtrs {
  const double* x[4];
  const double* y[4];
};
__global__ __launch_bounds__(256) void k_dots(DotPtrs d, int pairs, size_t n, double* __restrict__ partial) {
  __shared__ double red[4 * 4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(DOT_BLOCKS) * 256)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < pairs) v[q] += d.x[q][i] * d.y[q][i];
  const bool ismax[4] = {false, false, false, false};
  block_reduce_waves<256, 4>(red, v, ismax);
  if (threadIdx.x == 0)
    for (int q = 0; q < pairs; ++q) partial[size_t(q) * DOT_BLOCKS + blockIdx.x] = v[q];
}

// U = base + delta for block (level n, share b of nbl); partials as k_rows_inv.
__global__ __launch_bounds__(256) void k_update_plain(double* __restrict__ U, const double* __restrict__ u0,
                                                       const double* __restrict__ delta, double* __restrict__ part,
                                                       int ns, int nbl, int bcast) {
  __shared__ double red[4 * 4];
  const int n = blockIdx.x / nbl, b = blockIdx.x - (blockIdx.x / nbl) * nbl;
  const int chunk = ns / nbl;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = b * chunk + threadIdx.x; i < (b + 1) * chunk; i += 256) {
    const size_t gi = size_t(n) * ns + i;
    const double del = delta[gi];
    const double u = (bcast ? u0[i] : U[gi]) + del;
    U[gi] = u;
    acc[0] += del * del;
    acc[1] += u * u;
    acc[2] += 3.0 * u * u;
    const double ad = del < 0 ? -del : del;
    acc[3] = (ad != ad || ad > acc[3]) ? ad : acc[3];
  }
  const bool ismax[4] = {false, false, false, true};
  block_reduce_waves<256, 4>(red, acc, ismax);
  if (threadIdx.x == 0) {
    double* pp = part + size_t(blockIdx.x) * PART_STRIDE;
    pp[PART_DSQ] = acc[0];
    pp[PART_USQ] = acc[1];
    pp[PART_U2] = acc[2];
    pp[PART_DMAX] = acc[3];
  }
}

// ============================================================== launchers
#define PINT_CHECK_LAUNCH()            \
  do {                                 \
    hipError_t e_ = hipGetLastError(); \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

// Row-pass geometry per grid size: rows per block and threads per block.
template <int DIM, int N>
struct row_cfg {
  static constexpr int RB = DIM == 1 ? 4 : (N >= 512 ? 8 : (N >= 256 ? 16 : (N >= 32 ? 32 : N)));
  // 2D N >= 256: 512 threads (C5 inverse pass 0.944 -> 0.916 ms)
  static constexpr int NT0 = (DIM == 2 && N >= 256) ? 512 : 256;
  static constexpr int NT = RB * N < NT0 ? RB * N : NT0;
  static constexpr int NBL = DIM == 2 ? N / RB : 1;
};
// The forward pass holds v (RB + 4 rows), then g, then the FFT input in one
// LDS buffer (FP64 for v and g): 48 KB for 8 rows of 512, so two blocks fit
// per CU.
template <int DIM, int N, bool WIDE>
struct row_fwd_cfg {
  // 256^2: half the inverse pass's height (8 rows; 16 measured slower); 512^2:
  // the full 8 rows (4 rows: 1171 us per launch at 512^2 x 1024, 8 rows: 1118 us)
  static constexpr int RB = (DIM == 2 && N == 256 && !WIDE) ? row_cfg<DIM, N>::RB / 2 : row_cfg<DIM, N>::RB;
  // 2D N >= 64: 512 threads per block shorten each thread's serial chain;
  // 1024 at N = 512 (C5 mixed / FP64 1.34 / 1.36 -> 1.30 / 1.31 ms, FP32 the same)
  static constexpr int NT0 = (DIM == 2 && N == 512) ? 1024 : ((DIM == 2 && N >= 64) ? 512 : 256);
  static constexpr int NT = RB * N < NT0 ? RB * N : NT0;
  static constexpr int NBL = DIM == 2 ? N / RB : 1;
};
// Column-pass tile width and threads.
// Columns per block: 32, or 16 for FP64 at N >= 256, where 32 columns take
// 72-144 KB of LDS (C5 forward pass: 0.89 -> 0.62 ms); FP32 measured no gain.
template <typename T, int N>
struct col_cfg {
  static constexpr int XB = N < 32 ? N : ((sizeof(T) == 8 && N >= 256) ? 16 : 32);
  // N >= 256: 512 threads, N = 512: 1024 (C5 FP32 inverse pass 0.53 -> 0.49 ms,
  // mixed forward / inverse 0.79 / 0.55 -> 0.74 / 0.50 ms)
  static constexpr int NT0 = N >= 512 ? 1024 : (N >= 256 ? 512 : 256);
  static constexpr int NT = (N * XB / 2) < NT0 ? (N * XB / 2) : NT0;
};

int rows_blocks_per_level(int dim, int n) {
  if (dim == 1) return 1;
  switch (n) {
    case 8: return row_cfg<2, 8>::NBL;
    case 16: return row_cfg<2, 16>::NBL;
    case 32: return row_cfg<2, 32>::NBL;
    case 64: return row_cfg<2, 64>::NBL;
    case 128: return row_cfg<2, 128>::NBL;
    case 256: return row_cfg<2, 256>::NBL;
    case 512: return row_cfg<2, 512>::NBL;
    default: return 0;
  }
}

int rows_fwd_blocks_per_level(int dim, int n) {
  if (dim != 2) return 1;
  switch (n) {
    case 8: return row_fwd_cfg<2, 8, false>::NBL;
    case 16: return row_fwd_cfg<2, 16, false>::NBL;
    case 32: return row_fwd_cfg<2, 32, false>::NBL;
    case 64: return row_fwd_cfg<2, 64, false>::NBL;
    case 128: return row_fwd_cfg<2, 128, false>::NBL;
    case 256: return row_fwd_cfg<2, 256, false>::NBL;
    case 512: return row_fwd_cfg<2, 512, false>::NBL;
    default: return 0;
  }
}

int rows_levels_per_block(int dim, int n) {
  (void)n;
  return dim == 1 ? row_cfg<1, 8>::RB : 1;
}

template <typename T, typename TO, int DIM, int N, bool WIDE, typename RT>
static hipError_t launch_rows_fwd_w(const ResidArgs& a, TO* S, double* rout, const DctTables<T>& dt, int nt,
                                    int mode, hipStream_t st) {
  using C = row_fwd_cfg<DIM, N, WIDE>;
  const int grid = DIM == 2 ? (a.one_level ? 1 : nt) * C::NBL : nt / C::RB;
  if (a.one_level && (DIM != 2 || !a.bcast || a.nt != nt)) return hipErrorInvalidValue;
  if (mode == 0)
    PINT_LAUNCH((k_rows_fwd<T, TO, DIM, N, C::RB, C::NT, 0, RT>), dim3(grid), dim3(C::NT), 0, st, a, S,
                       rout, dt);
  else
    PINT_LAUNCH((k_rows_fwd<T, TO, DIM, N, C::RB, C::NT, 1, RT>), dim3(grid), dim3(C::NT), 0, st, a, S,
                       rout, dt);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename T, typename TO, int DIM, int N, typename RT>
static hipError_t launch_rows_fwd_n(const ResidArgs& a, TO* S, double* rout, const DctTables<T>& dt, int nt,
                                    int mode, hipStream_t st) {
  return launch_rows_fwd_w<T, TO, DIM, N, false, RT>(a, S, rout, dt, nt, mode, st);
}

template <typename T, int DIM, int N>
static hipError_t launch_rows_inv_n(const UpdArgs& a, const T* S, double* dout, const DctTables<T>& dt, int nt,
                                    int mode, hipStream_t st) {
  using C = row_cfg<DIM, N>;
  const int grid = DIM == 2 ? nt * C::NBL : nt / C::RB;
  if (mode == 0)
    PINT_LAUNCH((k_rows_inv<T, DIM, N, C::RB, C::NT, 0>), dim3(grid), dim3(C::NT), 0, st, a, S, dout, dt);
  else
    PINT_LAUNCH((k_rows_inv<T, DIM, N, C::RB, C::NT, 1>), dim3(grid), dim3(C::NT), 0, st, a, S, dout, dt);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename T, int DIM, int N>
static hipError_t launch_rows_dct_n(const T* in, T* out, const DctTables<T>& dt, int nt, bool inv, hipStream_t st) {
  using C = row_cfg<DIM, N>;
  const int grid = DIM == 2 ? nt * C::NBL : nt / C::RB;
  if (!inv)
    PINT_LAUNCH((k_rows_dct<T, DIM, N, C::RB, C::NT, false>), dim3(grid), dim3(C::NT), 0, st, in, out, dt);
  else
    PINT_LAUNCH((k_rows_dct<T, DIM, N, C::RB, C::NT, true>), dim3(grid), dim3(C::NT), 0, st, in, out, dt);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename T, typename TO, int N>
static hipError_t launch_cols_n(const T* Sin, TO* Sout, const int* done, const DctTables<T>& dt, int nt, bool inv,
                                hipStream_t st, int tpi, int tpo, int levels) {
  using C = col_cfg<T, N>;
  // levels: how many levels (from level 0) to transform, of the nt the
  // layouts hold
  if (levels < 0) levels = nt;
  if (levels < 1 || levels > nt) return hipErrorInvalidValue;
  const int grid = levels * (N / C::XB);
  // The plain side is [level][mode]; a panel of the spectral side holds whole
  // pairs of modes and at most one level's modes; in place only when plain.
  constexpr int PLAIN = 2 * ilog2(N);
  const int tps = inv ? tpi : tpo;
  if ((inv ? tpo : tpi) != PLAIN || tps < 1 || tps > PLAIN) return hipErrorInvalidValue;
  if ((void*)Sin == (void*)Sout && tps != PLAIN) return hipErrorInvalidValue;
  if (!inv) {
    if (tps == PLAIN)
      PINT_LAUNCH((k_cols<T, TO, N, C::XB, C::NT, false, false>), dim3(grid), dim3(C::NT), 0, st, Sin, Sout, done,
                  dt, tps, nt);
    else
      PINT_LAUNCH((k_cols<T, TO, N, C::XB, C::NT, false, true>), dim3(grid), dim3(C::NT), 0, st, Sin, Sout, done,
                  dt, tps, nt);
  } else if constexpr (std::is_same<T, TO>::value) {
    if (tps == PLAIN)
      PINT_LAUNCH((k_cols<T, TO, N, C::XB, C::NT, true, false>), dim3(grid), dim3(C::NT), 0, st, Sin, Sout, done,
                  dt, tps, nt);
    else
      PINT_LAUNCH((k_cols<T, TO, N, C::XB, C::NT, true, true>), dim3(grid), dim3(C::NT), 0, st, Sin, Sout, done,
                  dt, tps, nt);
  } else
    return hipErrorInvalidValue;
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

#define PINT_SWITCH_N(CALL)               \
  switch (n) {                            \
    case 8: return CALL(8);               \
    case 16: return CALL(16);             \
    case 32: return CALL(32);             \
    case 64: return CALL(64);             \
    case 128: return CALL(128);           \
    case 256: return CALL(256);           \
    case 512: return CALL(512);           \
    default: return hipErrorInvalidValue; \
  }

template <typename T, typename TO, typename RT>
hipError_t launch_rows_fwd(int dim, int n, const ResidArgs& a, TO* S, double* rout, const DctTables<T>& dt, int nt,
                           int mode, hipStream_t st) {
#define C1_(NN) launch_rows_fwd_n<T, TO, 1, NN, RT>(a, S, rout, dt, nt, mode, st)
#define C2_(NN) launch_rows_fwd_n<T, TO, 2, NN, RT>(a, S, rout, dt, nt, mode, st)
  if (dim == 2) {
    PINT_SWITCH_N(C2_)
  }
  PINT_SWITCH_N(C1_)
#undef C1_
#undef C2_
}

template <typename T>
hipError_t launch_rows_inv(int dim, int n, const UpdArgs& a, const T* S, double* dout, const DctTables<T>& dt,
                           int nt, int mode, hipStream_t st) {
#define C1_(NN) launch_rows_inv_n<T, 1, NN>(a, S, dout, dt, nt, mode, st)
#define C2_(NN) launch_rows_inv_n<T, 2, NN>(a, S, dout, dt, nt, mode, st)
  if (dim == 2) {
    PINT_SWITCH_N(C2_)
  }
  PINT_SWITCH_N(C1_)
#undef C1_
#undef C2_
}

template <typename T, typename TO>
hipError_t launch_cols(int n, const T* Sin, TO* Sout, const int* done, const DctTables<T>& dt, int nt, bool inv,
                       hipStream_t st, int tps_in, int tps_out, int levels) {
#define CC_(NN) launch_cols_n<T, TO, NN>(Sin, Sout, done, dt, nt, inv, st, tps_in, tps_out, levels)
  PINT_SWITCH_N(CC_)
#undef CC_
}

template <typename T, int DIM>
static hipError_t rows_dct_dispatch(int n, const T* in, T* out, const DctTables<T>& dt, int nt, bool inv,
                                    hipStream_t st) {
#define RR_(NN) launch_rows_dct_n<T, DIM, NN>(in, out, dt, nt, inv, st)
  PINT_SWITCH_N(RR_)
#undef RR_
}

// Stage entry: orthonormal DCT-II (or its inverse) of every level; in == out
// allowed.  2D forward = rows then columns; inverse = columns then rows.
template <typename T>
hipError_t launch_dct(int dim, int n, const T* in, T* out, const DctTables<T>& dt, int nt, bool inv,
                      hipStream_t st) {
  if (dim == 1) return rows_dct_dispatch<T, 1>(n, in, out, dt, nt, inv, st);
  hipError_t e;
  if (!inv) {
    e = rows_dct_dispatch<T, 2>(n, in, out, dt, nt, false, st);
    if (e != hipSuccess) return e;
    return launch_cols<T, T>(n, out, out, nullptr, dt, nt, false, st, 2 * ilog2(n), 2 * ilog2(n));
  }
  if (in != out) {
    e = hipMemcpyAsync(out, in, sizeof(T) * size_t(nt) * n * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  e = launch_cols<T, T>(n, out, out, nullptr, dt, nt, true, st, 2 * ilog2(n), 2 * ilog2(n));
  if (e != hipSuccess) return e;
  return rows_dct_dispatch<T, 2>(n, out, out, dt, nt, true, st);
}

// Time solve: tile width M (spatial modes per workgroup) is the largest of
// {8, 16, 32, 64} that divides ns and keeps the LDS tile (N_t x M/2 complex)
// within 64 KB; TimeArgs::tile can cap it.
template <typename T, int NTT>
struct time_cfg {
  static constexpr int BYTES = NTT * int(sizeof(cx<T>));  // one complex column
  // Default tile: the modes whose columns fit in 32 KB of LDS, in [8, 32], so
  // that several blocks share a CU (measured at N_t = 1024: 8 modes 1.5 ms,
  // 16 modes 2.1 ms, 32 modes 3.2 ms per launch); up to 128 KB on request.
  static constexpr int CDEF0 = 32768 / BYTES, CMAX0 = 131072 / BYTES;
  static constexpr int MMAX = 2 * (CMAX0 < 32 ? CMAX0 : 32);
  static constexpr int MDEF0 = 2 * (CDEF0 < 32 ? CDEF0 : 32);
  static constexpr int MDEF = MDEF0 < 8 ? 8 : (MDEF0 < 32 ? MDEF0 : 32);
};

template <typename T, int NTT, int M>
static hipError_t launch_time_m(T* S, const TimeArgs<T>& ta, hipStream_t st) {
  if constexpr (M > time_cfg<T, NTT>::MMAX || M < 2) {
    return hipErrorInvalidValue;
  } else {
    // FP32 at N_t >= 512: 512 threads (C5 0.645 -> 0.629 ms; FP64 slower)
    constexpr int NTS = (sizeof(T) == 4 && NTT >= 512) ? 512 : 256;
    PINT_LAUNCH((k_time_solve<T, NTT, M, NTS>), dim3(ta.ns / M), dim3(NTS), 0, st, S, ta);
    PINT_CHECK_LAUNCH();
    return hipSuccess;
  }
}

template <typename T, int NTT>
static int time_tile_nt(int ns, int tile) {
  int m = time_cfg<T, NTT>::MDEF;
  if (tile > 0) m = tile < time_cfg<T, NTT>::MMAX ? tile : time_cfg<T, NTT>::MMAX;
  while (m > 8 && (m > ns || ns % m != 0)) m /= 2;
  return ns % m == 0 ? m : 0;
}

template <typename T>
static int time_tile_t(int nt, int ns, int tile) {
  switch (nt) {
    case 4: return time_tile_nt<T, 4>(ns, tile);
    case 8: return time_tile_nt<T, 8>(ns, tile);
    case 16: return time_tile_nt<T, 16>(ns, tile);
    case 32: return time_tile_nt<T, 32>(ns, tile);
    case 64: return time_tile_nt<T, 64>(ns, tile);
    case 128: return time_tile_nt<T, 128>(ns, tile);
    case 256: return time_tile_nt<T, 256>(ns, tile);
    case 512: return time_tile_nt<T, 512>(ns, tile);
    case 1024: return time_tile_nt<T, 1024>(ns, tile);
    default: return 0;
  }
}

int time_tile_modes(bool fp64, int nt, int ns, int tile) {
  return fp64 ? time_tile_t<double>(nt, ns, tile) : time_tile_t<float>(nt, ns, tile);
}

template <typename T, int NTT>
static hipError_t launch_time_nt(T* S, const TimeArgs<T>& ta, hipStream_t st) {
  const int m = time_tile_nt<T, NTT>(ta.ns, ta.tile);
  // the panel holds whole tiles and at most one level's modes
  if (m == 0 || ta.tps < 0 || (1 << ta.tps) > ta.ns || (1 << ta.tps) % m != 0) return hipErrorInvalidValue;
  switch (m) {
    case 64: return launch_time_m<T, NTT, 64>(S, ta, st);
    case 32: return launch_time_m<T, NTT, 32>(S, ta, st);
    case 16: return launch_time_m<T, NTT, 16>(S, ta, st);
    case 8: return launch_time_m<T, NTT, 8>(S, ta, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_time(int nt, T* S, const TimeArgs<T>& ta, hipStream_t st) {
  switch (nt) {
    case 4: return launch_time_nt<T, 4>(S, ta, st);
    case 8: return launch_time_nt<T, 8>(S, ta, st);
    case 16: return launch_time_nt<T, 16>(S, ta, st);
    case 32: return launch_time_nt<T, 32>(S, ta, st);
    case 64: return launch_time_nt<T, 64>(S, ta, st);
    case 128: return launch_time_nt<T, 128>(S, ta, st);
    case 256: return launch_time_nt<T, 256>(S, ta, st);
    case 512: return launch_time_nt<T, 512>(S, ta, st);
    case 1024: return launch_time_nt<T, 1024>(S, ta, st);
    default: return hipErrorInvalidValue;
  }
}

int finalize_groups(int nt, int nbl, int nbl_f) {
  const int gmax = nbl > nbl_f ? nbl : nbl_f;
  return size_t(nt) * gmax > size_t(FIN_WIDE_SLOTS) ? (nt + FIN_LEVELS - 1) / FIN_LEVELS : 0;
}

hipError_t launch_finalize(const FinArgs& f, hipStream_t st) {
  const int groups = finalize_groups(f.nt, f.nbl, f.nbl_f);
  if (groups > 0) {
    if (!f.fin) return hipErrorInvalidValue;
    // stage timing: the start event on the first kernel, the stop event on the second
    hipEvent_t e0 = g_launch_ev0, e1 = g_launch_ev1;
    g_launch_ev0 = g_launch_ev1 = nullptr;
    if (e0)
      hipExtLaunchKernelGGL(k_fin_levels, dim3(groups), dim3(256), 0, st, e0, nullptr, 0, f);
    else
      hipLaunchKernelGGL(k_fin_levels, dim3(groups), dim3(256), 0, st, f);
    PINT_CHECK_LAUNCH();
    if (e1)
      hipExtLaunchKernelGGL(k_finalize_groups, dim3(1), dim3(64), 0, st, nullptr, e1, 0, f, groups);
    else
      hipLaunchKernelGGL(k_finalize_groups, dim3(1), dim3(64), 0, st, f, groups);
  } else {
    PINT_LAUNCH(k_finalize<256>, dim3(1), dim3(256), 0, st, f);
  }
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_init(const InitArgs& a, Ctrl* c, Ctrl* host, double dof, bool need_cbar, hipStream_t st) {
  int nparts = 0;
  if (need_cbar) {
    const size_t total = a.broadcast ? size_t(a.ns) : size_t(a.ns) * a.nt;
    nparts = int((total + INIT_CHUNK - 1) / INIT_CHUNK);
    PINT_LAUNCH(k_init_part, dim3(nparts), dim3(256), 0, st, a);
    PINT_CHECK_LAUNCH();
  }
  PINT_LAUNCH(k_init_ctrl, dim3(1), dim3(256), 0, st, c, host, a, dof, nparts);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_jfield(const double* U, double* j, int nt, int ns, hipStream_t st) {
  PINT_LAUNCH(k_jfield, dim3((ns + 255) / 256), dim3(256), 0, st, U, j, nt, ns);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_axpbypcz(double* out, double a, const double* x, double b, const double* y, double c,
                           const double* z, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  PINT_LAUNCH(k_axpbypcz, dim3(unsigned(blocks)), dim3(256), 0, st, out, a, x, b, y, c, z, n);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_dots(const double* const* xs, const double* const* ys, int pairs, size_t n, double* partial,
                       hipStream_t st) {
  if (pairs < 1 || pairs > 4) return hipErrorInvalidValue;
  DotPtrs d{};
  for (int q = 0; q < pairs; ++q) {
    d.x[q] = xs[q];
    d.y[q] = ys[q];
  }
  PINT_LAUNCH(k_dots, dim3(DOT_BLOCKS), dim3(256), 0, st, d, pairs, n, partial);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_update_plain(double* U, const double* u0, const double* delta, double* part, int nt, int ns,
                               int nbl, int bcast, hipStream_t st) {
  if (ns % nbl != 0) return hipErrorInvalidValue;
  PINT_LAUNCH(k_update_plain, dim3(nt * nbl), dim3(256), 0, st, U, u0, delta, part, ns, nbl, bcast);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_invariants(const DiagArgs& a, const double* u0, double* scratch, int nt, bool energy, Ctrl* c,
                             Ctrl* host, hipStream_t st) {
  PINT_LAUNCH(k_invariants, dim3(nt + 1), dim3(256), 0, st, a, u0, scratch);
  PINT_CHECK_LAUNCH();
  PINT_LAUNCH(k_invariants_fin, dim3(1), dim3(256), 0, st, scratch, nt, energy ? 1 : 0, c, host);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename TI, typename TO>
hipError_t launch_cast(const TI* in, TO* out, size_t n, hipStream_t st) {
  PINT_LAUNCH((k_cast<TI, TO>), dim3(1024), dim3(256), 0, st, in, out, n);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_diagnostics(const DiagArgs& a, int nt, hipStream_t st) {
  PINT_LAUNCH(k_diagnostics, dim3(nt), dim3(256), 0, st, a);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template hipError_t launch_rows_fwd<float, float, double>(int, int, const ResidArgs&, float*, double*,
                                                          const DctTables<float>&, int, int, hipStream_t);
template hipError_t launch_rows_fwd<float, float, float>(int, int, const ResidArgs&, float*, double*,
                                                         const DctTables<float>&, int, int, hipStream_t);
template hipError_t launch_rows_fwd<double, double, double>(int, int, const ResidArgs&, double*, double*,
                                                            const DctTables<double>&, int, int, hipStream_t);
template hipError_t launch_rows_fwd<double, float, double>(int, int, const ResidArgs&, float*, double*,
                                                   const DctTables<double>&, int, int, hipStream_t);
template hipError_t launch_rows_inv<float>(int, int, const UpdArgs&, const float*, double*, const DctTables<float>&,
                                           int, int, hipStream_t);
template hipError_t launch_rows_inv<double>(int, int, const UpdArgs&, const double*, double*,
                                            const DctTables<double>&, int, int, hipStream_t);
template hipError_t launch_cols<float, float>(int, const float*, float*, const int*, const DctTables<float>&, int,
                                              bool, hipStream_t, int, int, int);
template hipError_t launch_cols<double, double>(int, const double*, double*, const int*, const DctTables<double>&,
                                                int, bool, hipStream_t, int, int, int);
template hipError_t launch_cols<double, float>(int, const double*, float*, const int*, const DctTables<double>&,
                                               int, bool, hipStream_t, int, int, int);
template hipError_t launch_dct<float>(int, int, const float*, float*, const DctTables<float>&, int, bool,
                                      hipStream_t);
template hipError_t launch_dct<double>(int, int, const double*, double*, const DctTables<double>&, int, bool,
                                       hipStream_t);
template hipError_t launch_time<float>(int, float*, const TimeArgs<float>&, hipStream_t);
template hipError_t launch_time<double>(int, double*, const TimeArgs<double>&, hipStream_t);
template hipError_t launch_cast<double, float>(const double*, float*, size_t, hipStream_t);
template hipError_t launch_cast<double, double>(const double*, double*, size_t, hipStream_t);

}  // namespace pint

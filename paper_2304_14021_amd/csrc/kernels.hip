// HIP kernels (gfx950) of the all-at-once space-time solve, FFT path.
//
// One outer iteration (correction form U <- U + P_alpha^{-1} r(U)) is
//   k_resid_dct   a1 + a2: FP64 residual of one time level (or a pair of 1D
//                 levels), rounded to the working type W, then its orthonormal
//                 DCT-II in LDS  ->  S[n][k]  (W)
//   k_time_solve  a3-a5: per tile of spatial cosine modes, Gamma_alpha scaling,
//                 FFT over time, shifted complex divide, inverse FFT,
//                 Gamma_alpha^{-1} scaling, in place on S (Section 2.1,
//                 eq. pintiter1; Section 4.1, eq. pintiter_CH)
//   k_idct_update a6: DCT-III of one level in LDS, U_n += delta_n in FP64,
//                 per-level partial norms
//   k_finalize    a7: fixed-order reduction of the partials, scalar averaged
//                 Jacobian, stop rule and divergence guard (one workgroup)
// All kernels return at once when the device stop flag is set, so several
// iterations may be enqueued ahead of the host's check.
#include "pint.h"
#include "pint_kernels.hpp"
#include "fft_lds.hpp"

namespace pint {

// ------------------------------------------------------------------ sizing
// Threads per workgroup of the per-slice kernels (2D: one N x N level).
constexpr int slice_threads(int n) { return n >= 128 ? 1024 : (n >= 32 ? 256 : 64); }
// LDS bytes of the per-slice kernels: the FP64 stencil array (N^2 doubles)
// and the DCT array (N^2 + 2N reals of W) share one buffer.
template <typename T, int N, int ROWS>
struct slice_lds {
  static constexpr int a = 8 * N * ROWS;
  static constexpr int b = int(sizeof(T)) * dct_lds_reals<N, ROWS>::value;
  static constexpr int red = 8 * 4 * 1024;
  static constexpr int value0 = a > b ? a : b;
  static constexpr int value = value0 > red ? value0 : red;
};

// Neumann (ghost-reflection) index clamp.
__device__ __forceinline__ int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// ---------------------------------------------------------------- residual
// DIM == 2: ROWS == N rows of one level n = blockIdx.x.
// DIM == 1: ROWS levels n0 .. n0+ROWS-1 (n0 = blockIdx.x * ROWS), one row each.
// The residual of level n is r_n = -(u_n - u_{n-1})/dt + Lap_h g_n with
//   g = c3 v^3 + c1 v + c1p u_{n-1} + c2 Lap_h v,  v = theta u_n + (1-theta) u_{n-1}
// which covers
//   linear theta-method: c3 = 0, c1 = -beta^2, c1p = 0, c2 = -eps^2
//   CH fully implicit  : theta = 1, c3 = 1, c1 = -1, c1p = 0, c2 = -eps^2
//   CH Eyre splitting  : theta = 1, c3 = 1, c1 = 0, c1p = -1, c2 = -eps^2
// (the alpha = 0 rows of eqs. all-at-once1, nonlinear_G and nonlinear_Q).
// MODE 0: write the DCT-II of r (type T) to S.  MODE 1: write r in FP64 to rout.
template <typename T, int DIM, int N, int ROWS, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_resid_dct(ResidArgs a, T* __restrict__ S, double* __restrict__ rout,
                                                   DctTables<T> dt) {
  if (a.done && *a.done) return;
  constexpr int NPT = N * ROWS / NT;
  static_assert(NPT * NT == N * ROWS, "threads must divide the slab");
  __shared__ __align__(16) unsigned char lds[slice_lds<T, N, ROWS>::value];
  double* V = reinterpret_cast<double*>(lds);
  T* A = reinterpret_cast<T*>(lds);
  const int tid = threadIdx.x;
  const int ns = (DIM == 2) ? N * N : N;
  const double th = a.theta, omth = 1.0 - a.theta;

  double d[NPT];
  // Phase 1: v = theta u_n + (1-theta) u_{n-1} -> LDS; d = u_n - u_{n-1} kept.
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int idx = tid + i * NT;                      // [row][x] within the slab
    const int row = idx / N, x = idx - (idx / N) * N;
    const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + row;
    const int off = (DIM == 2) ? idx : x;
    const double un = a.U[(size_t)n * ns + off];
    const double um = (n == 0) ? a.u0[off] : a.U[(size_t)(n - 1) * ns + off];
    d[i] = un - um;
    V[idx] = th * un + omth * um;
  }
  __syncthreads();
  // Phase 2: g (needs Lap_h v from LDS).
  double g[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int idx = tid + i * NT;
    const int row = idx / N, x = idx - (idx / N) * N;
    const double v = V[idx];
    double lap = V[row * N + clampi(x - 1, N)] + V[row * N + clampi(x + 1, N)] - 2.0 * v;
    if (DIM == 2) lap += V[clampi(row - 1, N) * N + x] + V[clampi(row + 1, N) * N + x] - 2.0 * v;
    lap *= a.inv_h2;
    const double um = v - th * d[i];
    g[i] = a.c3 * v * v * v + a.c1 * v + a.c1p * um + a.c2 * lap;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NPT; ++i) V[tid + i * NT] = g[i];
  __syncthreads();
  // Phase 3: r = -d/dt + Lap_h g.
  double rsq[DIM == 2 ? 1 : ROWS];
#pragma unroll
  for (int q = 0; q < (DIM == 2 ? 1 : ROWS); ++q) rsq[q] = 0.0;
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int idx = tid + i * NT;
    const int row = idx / N, x = idx - (idx / N) * N;
    const double gc = V[idx];
    double lap = V[row * N + clampi(x - 1, N)] + V[row * N + clampi(x + 1, N)] - 2.0 * gc;
    if (DIM == 2) lap += V[clampi(row - 1, N) * N + x] + V[clampi(row + 1, N) * N + x] - 2.0 * gc;
    const double r = -d[i] * a.inv_dt + lap * a.inv_h2;
    g[i] = r;
    if (DIM == 2) rsq[0] += r * r;
    else {
#pragma unroll
      for (int q = 0; q < (DIM == 2 ? 1 : ROWS); ++q) rsq[q] += (row == q) ? r * r : 0.0;
    }
  }
  __syncthreads();
  if (MODE == 1) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int idx = tid + i * NT;
      const int row = idx / N, x = idx - (idx / N) * N;
      const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + row;
      const int off = (DIM == 2) ? idx : x;
      rout[(size_t)n * ns + off] = g[i];
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < NPT; ++i) A[tid + i * NT] = T(g[i]);
  __syncthreads();
  dct2_rows<T, N, ROWS, N, NT>(A, dt.tw, dt.wq);
  if (DIM == 2) dct2_cols<T, N, N, NT>(A, dt.tw, dt.wq);
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int idx = tid + i * NT;
    const int row = idx / N, x = idx - (idx / N) * N;
    const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + row;
    const int off = (DIM == 2) ? idx : x;
    S[(size_t)n * ns + off] = A[idx];
  }
  __syncthreads();
  // Per-level partial sum of r^2.
  constexpr int NV = (DIM == 2) ? 1 : ROWS;
  bool ismax[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) ismax[q] = false;
  block_reduce<NT, NV>(reinterpret_cast<double*>(lds), rsq, ismax);
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + q;
      a.part[(size_t)n * PART_STRIDE + PART_RSQ] = rsq[q];
    }
  }
}

// ------------------------------------------------------- inverse + update
// delta = DCT-III of S level(s); U += delta (FP64); partial sums of
// delta^2, U^2, 3U^2 and max|delta| per level.  MODE 1 writes delta in FP64
// to dout instead of updating U.
template <typename T, int DIM, int N, int ROWS, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_idct_update(UpdArgs a, const T* __restrict__ S, double* __restrict__ dout,
                                                     DctTables<T> dt) {
  if (a.done && *a.done) return;
  constexpr int NPT = N * ROWS / NT;
  static_assert(NPT * NT == N * ROWS, "threads must divide the slab");
  __shared__ __align__(16) unsigned char lds[slice_lds<T, N, ROWS>::value];
  T* A = reinterpret_cast<T*>(lds);
  const int tid = threadIdx.x;
  const int ns = (DIM == 2) ? N * N : N;
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int idx = tid + i * NT;
    const int row = idx / N, x = idx - (idx / N) * N;
    const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + row;
    const int off = (DIM == 2) ? idx : x;
    A[idx] = S[(size_t)n * ns + off];
  }
  __syncthreads();
  if (DIM == 2) dct3_cols<T, N, N, NT>(A, dt.tw, dt.wi);
  dct3_rows<T, N, ROWS, N, NT>(A, dt.tw, dt.wi);
  constexpr int NV1 = (DIM == 2) ? 1 : ROWS;
  double acc[4 * NV1];
#pragma unroll
  for (int q = 0; q < 4 * NV1; ++q) acc[q] = 0.0;
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int idx = tid + i * NT;
    const int row = idx / N, x = idx - (idx / N) * N;
    const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + row;
    const int off = (DIM == 2) ? idx : x;
    const double del = double(A[idx]);
    const int q = (DIM == 2) ? 0 : row;
    if (MODE == 1) {
      dout[(size_t)n * ns + off] = del;
      continue;
    }
    const size_t gi = (size_t)n * ns + off;
    const double u = a.U[gi] + del;
    a.U[gi] = u;
#pragma unroll
    for (int qq = 0; qq < NV1; ++qq) {
      if (qq == q) {
        acc[4 * qq + 0] += del * del;
        acc[4 * qq + 1] += u * u;
        acc[4 * qq + 2] += 3.0 * u * u;
        const double ad = del < 0 ? -del : del;
        acc[4 * qq + 3] = (ad != ad || ad > acc[4 * qq + 3]) ? ad : acc[4 * qq + 3];
      }
    }
  }
  if (MODE == 1) return;
  __syncthreads();
  bool ismax[4 * NV1];
#pragma unroll
  for (int q = 0; q < 4 * NV1; ++q) ismax[q] = (q % 4) == 3;
  block_reduce<NT, 4 * NV1>(reinterpret_cast<double*>(lds), acc, ismax);
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV1; ++q) {
      const int n = (DIM == 2) ? blockIdx.x : blockIdx.x * ROWS + q;
      double* pp = a.part + (size_t)n * PART_STRIDE;
      pp[PART_DSQ] = acc[4 * q + 0];
      pp[PART_USQ] = acc[4 * q + 1];
      pp[PART_U2] = acc[4 * q + 2];
      pp[PART_DMAX] = acc[4 * q + 3];
    }
  }
}

// ------------------------------------------------------------- time solve
// One workgroup per tile of M consecutive spatial modes k (M even): the M
// real sequences over time are packed into M/2 complex ones, transformed
// together, split into their Hermitian halves, divided by
//   sigma_{l,k} = lambda1_l + p_l lam_k + q_l lam_k^2,   l = 0..N_t/2,
// (p_l = pco_l - c_bar for the CH operators), re-packed and transformed back.
template <typename T, int NTT, int M, int NT>
__global__ __launch_bounds__(NT) void k_time_solve(T* __restrict__ S, TimeArgs<T> ta) {
  if (ta.done && *ta.done) return;
  constexpr int C = M / 2;
  __shared__ __align__(16) cx<T> z[NTT * C];
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * M;
  const int ns = ta.ns;
  constexpr int W = NTT * C;
  for (int w = tid; w < W; w += NT) {
    const int j = w / C, c = w - (w / C) * C;
    const cx<T> x = *reinterpret_cast<const cx<T>*>(S + (size_t)j * ns + col0 + 2 * c);
    z[w] = scale(x, ta.aj[j]);
  }
  __syncthreads();
  fft_lds<T, NTT, C, C, NT, -1>(z, ta.tw);
  const T cb = ta.cbar_mode ? T(ta.cbar ? *ta.cbar : ta.cbar_val) : T(0);
  constexpr int WD = (NTT / 2 + 1) * C;
  for (int w = tid; w < WD; w += NT) {
    const int l = w / C, c = w - (w / C) * C;
    const int m = (NTT - l) & (NTT - 1);
    const cx<T> zl = z[l * C + c];
    const cx<T> zm = conj(z[m * C + c]);
    const cx<T> x1 = scale(add(zl, zm), T(0.5));
    const cx<T> x2 = scale(mul_mi(sub(zl, zm)), T(0.5));
    const int k1 = col0 + 2 * c, k2 = k1 + 1;
    const T lk1 = ta.lamx[k1 % ta.nx] + ta.lamy[k1 / ta.nx];
    const T lk2 = ta.lamx[k2 % ta.nx] + ta.lamy[k2 / ta.nx];
    const cx<T> l1 = ta.lam1[l];
    const cx<T> pl = mk(ta.pco[l].x - cb, ta.pco[l].y);
    const cx<T> ql = ta.qco[l];
    const cx<T> s1 = mk(l1.x + pl.x * lk1 + ql.x * lk1 * lk1, l1.y + pl.y * lk1 + ql.y * lk1 * lk1);
    const cx<T> s2 = mk(l1.x + pl.x * lk2 + ql.x * lk2 * lk2, l1.y + pl.y * lk2 + ql.y * lk2 * lk2);
    const cx<T> y1 = cdiv(x1, s1);
    const cx<T> y2 = cdiv(x2, s2);
    z[l * C + c] = add(y1, mul_i(y2));
    if (m != l) z[m * C + c] = add(conj(y1), mul_i(conj(y2)));
  }
  __syncthreads();
  fft_lds<T, NTT, C, C, NT, +1>(z, ta.tw);
  for (int w = tid; w < W; w += NT) {
    const int j = w / C, c = w - (w / C) * C;
    *reinterpret_cast<cx<T>*>(S + (size_t)j * ns + col0 + 2 * c) = scale(z[w], ta.aij[j]);
  }
}

// --------------------------------------------------------------- control
// One workgroup: reduce the per-level partials in a fixed order, update the
// scalar averaged Jacobian and apply the stop rule.
//   upd  = max_n ||delta_n||_2,  unrm = max_n ||u_n||_2,  rel = upd / unrm
//   rho  = upd_k / upd_{k-1};  est = rho/(1-rho) * rel
// stop when est <= 0.1 rtol (k >= 2, rho < 1) or rel <= 1e-3 rtol;
// diverged on NaN/Inf or when the update grows 1e3-fold over the first one.
__global__ __launch_bounds__(256) void k_finalize(FinArgs f) {
  if (f.ctrl->done) return;
  constexpr int NT = 256;
  __shared__ double red[4 * NT];
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // max dsq, max usq, sum u2, max rsq
  for (int n = threadIdx.x; n < f.nt; n += NT) {
    const double* pp = f.part + (size_t)n * PART_STRIDE;
    const double dsq = pp[PART_DSQ], usq = pp[PART_USQ], u2 = pp[PART_U2], rsq = pp[PART_RSQ];
    v[0] = (dsq != dsq || dsq > v[0]) ? dsq : v[0];
    v[1] = (usq != usq || usq > v[1]) ? usq : v[1];
    v[2] += u2;
    v[3] = (rsq != rsq || rsq > v[3]) ? rsq : v[3];
  }
  const bool ismax[4] = {true, true, false, true};
  block_reduce<NT, 4>(red, v, ismax);
  if (threadIdx.x != 0) return;
  Ctrl* c = f.ctrl;
  const double upd = sqrt(v[0]), unrm = sqrt(v[1]), res = sqrt(v[3]);
  const double cbar = v[2] / f.dof;
  const int k = c->iter;  // 0-based index of the iteration just finished
  const double rel = unrm > 0.0 ? upd / unrm : upd;
  if (k < PINT_HIST_DEV) {
    c->upd_hist[k] = rel;
    c->res_hist[k] = res;
  }
  c->iter = k + 1;
  c->c_bar = cbar;
  const bool bad = !(upd == upd) || !(unrm == unrm) || !(cbar == cbar) || upd > 1e300 || unrm > 1e300;
  double est = 1e300;
  if (k >= 1 && c->upd_prev > 0.0) {
    const double rho = upd / c->upd_prev;
    if (rho < 1.0) est = rho / (1.0 - rho) * rel;
  }
  if (upd == 0.0) est = 0.0;
  c->est = est;
  if (k == 0) c->upd_first = upd;
  c->upd_prev = upd;
  if (bad || (k >= 2 && upd > 1e3 * c->upd_first)) {
    c->status = PINT_EDIVERGED;
    c->done = 1;
  } else if (est <= 0.1 * f.rtol || rel <= 1e-3 * f.rtol) {
    c->status = PINT_OK;
    c->done = 1;
  } else if (k + 1 >= f.max_iter) {
    c->status = PINT_ENOCONV;
    c->done = 1;
  }
}

// Partial sums of 3 u^2 over the initial guess (the first iteration's c_bar),
// optionally broadcasting u0 into U first.  One workgroup per level.
__global__ __launch_bounds__(256) void k_init(InitArgs a) {
  constexpr int NT = 256;
  __shared__ double red[NT];
  const int n = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < a.ns; i += NT) {
    double u;
    if (a.broadcast) {
      u = a.u0[i];
      a.U[(size_t)n * a.ns + i] = u;
    } else {
      u = a.U[(size_t)n * a.ns + i];
    }
    s += 3.0 * u * u;
  }
  double v[1] = {s};
  const bool ismax[1] = {false};
  block_reduce<NT, 1>(red, v, ismax);
  if (threadIdx.x == 0) a.part[(size_t)n * PART_STRIDE + PART_U2] = v[0];
}

__global__ __launch_bounds__(64) void k_init_ctrl(Ctrl* c, int nt, const double* part, double dof) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int n = 0; n < nt; ++n) s += part[(size_t)n * PART_STRIDE + PART_U2];
  c->iter = 0;
  c->done = 0;
  c->status = PINT_ENOCONV;
  c->c_bar = s / dof;
  c->upd_prev = 0.0;
  c->upd_first = 0.0;
  c->est = 1e300;
}

// ------------------------------------------------------------- stage I/O
template <typename T>
__global__ void k_cast_to(const double* __restrict__ in, T* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = T(in[i]);
}
template <typename T>
__global__ void k_cast_from(const T* __restrict__ in, double* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = double(in[i]);
}

// Stand-alone batched DCT (stage entry point): one level (2D) or ROWS
// levels (1D) per workgroup.
template <typename T, int DIM, int N, int ROWS, int NT, bool INV>
__global__ __launch_bounds__(NT) void k_dct(const T* __restrict__ in, T* __restrict__ out, DctTables<T> dt) {
  constexpr int NPT = N * ROWS / NT;
  __shared__ __align__(16) unsigned char lds[slice_lds<T, N, ROWS>::value];
  T* A = reinterpret_cast<T*>(lds);
  const int tid = threadIdx.x;
  const size_t base = (size_t)blockIdx.x * N * ROWS;
#pragma unroll
  for (int i = 0; i < NPT; ++i) A[tid + i * NT] = in[base + tid + i * NT];
  __syncthreads();
  if (!INV) {
    dct2_rows<T, N, ROWS, N, NT>(A, dt.tw, dt.wq);
    if (DIM == 2) dct2_cols<T, N, N, NT>(A, dt.tw, dt.wq);
  } else {
    if (DIM == 2) dct3_cols<T, N, N, NT>(A, dt.tw, dt.wi);
    dct3_rows<T, N, ROWS, N, NT>(A, dt.tw, dt.wi);
  }
#pragma unroll
  for (int i = 0; i < NPT; ++i) out[base + tid + i * NT] = A[tid + i * NT];
}

// Per-level mass and Ginzburg-Landau energy (FP64).  One workgroup per level.
__global__ __launch_bounds__(256) void k_diagnostics(DiagArgs a) {
  constexpr int NT = 256;
  __shared__ double red[2 * NT];
  const int n = blockIdx.x;
  const double* u = a.U + (size_t)n * a.ns;
  double m = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < a.ns; i += NT) {
    const int x = i % a.nx, y = i / a.nx;
    const double v = u[i];
    m += v;
    const double w = v * v - 1.0;
    e += 0.25 * w * w;
    double gsq = 0.0;
    if (x + 1 < a.nx) {
      const double dd = (u[i + 1] - v);
      gsq += dd * dd;
    }
    if (a.dim == 2 && y + 1 < a.nx) {
      const double dd = (u[i + a.nx] - v);
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

// ------------------------------------------------------------- launchers
#define PINT_CHECK_LAUNCH()                                                \
  do {                                                                     \
    hipError_t e_ = hipGetLastError();                                     \
    if (e_ != hipSuccess) return e_;                                       \
  } while (0)

// Threads per workgroup of the per-level kernels: 2D levels by N; 1D slabs of
// two levels with one thread per point (at least one wavefront of 64).
template <int DIM, int N>
struct slab_cfg {
  static constexpr int ROWS = DIM == 2 ? N : 2;
  static constexpr int NT0 = DIM == 2 ? slice_threads(N) : (N >= 64 ? N : 64);
  static constexpr int NT = N * ROWS < NT0 ? N * ROWS : NT0;
  static_assert((N * ROWS) % NT == 0, "threads must divide the slab");
};

template <typename T, int DIM, int N>
static hipError_t launch_resid_n(const ResidArgs& a, T* S, double* rout, const DctTables<T>& dt, int nt, int mode,
                                 hipStream_t st) {
  using C = slab_cfg<DIM, N>;
  const int grid = DIM == 2 ? nt : nt / C::ROWS;
  if (mode == 0)
    hipLaunchKernelGGL((k_resid_dct<T, DIM, N, C::ROWS, C::NT, 0>), dim3(grid), dim3(C::NT), 0, st, a, S, rout, dt);
  else
    hipLaunchKernelGGL((k_resid_dct<T, DIM, N, C::ROWS, C::NT, 1>), dim3(grid), dim3(C::NT), 0, st, a, S, rout, dt);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename T, int DIM, int N>
static hipError_t launch_upd_n(const UpdArgs& a, const T* S, double* dout, const DctTables<T>& dt, int nt, int mode,
                               hipStream_t st) {
  using C = slab_cfg<DIM, N>;
  const int grid = DIM == 2 ? nt : nt / C::ROWS;
  if (mode == 0)
    hipLaunchKernelGGL((k_idct_update<T, DIM, N, C::ROWS, C::NT, 0>), dim3(grid), dim3(C::NT), 0, st, a, S, dout, dt);
  else
    hipLaunchKernelGGL((k_idct_update<T, DIM, N, C::ROWS, C::NT, 1>), dim3(grid), dim3(C::NT), 0, st, a, S, dout, dt);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename T, int DIM, int N>
static hipError_t launch_dct_n(const T* in, T* out, const DctTables<T>& dt, int nt, bool inv, hipStream_t st) {
  using C = slab_cfg<DIM, N>;
  const int grid = DIM == 2 ? nt : nt / C::ROWS;
  if (!inv)
    hipLaunchKernelGGL((k_dct<T, DIM, N, C::ROWS, C::NT, false>), dim3(grid), dim3(C::NT), 0, st, in, out, dt);
  else
    hipLaunchKernelGGL((k_dct<T, DIM, N, C::ROWS, C::NT, true>), dim3(grid), dim3(C::NT), 0, st, in, out, dt);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

// Sizes of the per-slice path: 2D N in [8, 128]; 1D N in [8, 512].
#define PINT_SWITCH_N(DIM, CALL)                        \
  switch (n) {                                          \
    case 8: return CALL(DIM, 8);                        \
    case 16: return CALL(DIM, 16);                      \
    case 32: return CALL(DIM, 32);                      \
    case 64: return CALL(DIM, 64);                      \
    case 128: return CALL(DIM, 128);                    \
    default: break;                                     \
  }

template <typename T>
hipError_t launch_resid(int dim, int n, const ResidArgs& a, T* S, double* rout, const DctTables<T>& dt, int nt,
                        int mode, hipStream_t st) {
#define C_(D, NN) launch_resid_n<T, D, NN>(a, S, rout, dt, nt, mode, st)
  if (dim == 2) { PINT_SWITCH_N(2, C_) }
  else {
    PINT_SWITCH_N(1, C_)
    if (n == 256) return C_(1, 256);
    if (n == 512) return C_(1, 512);
  }
#undef C_
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_update(int dim, int n, const UpdArgs& a, const T* S, double* dout, const DctTables<T>& dt, int nt,
                         int mode, hipStream_t st) {
#define C_(D, NN) launch_upd_n<T, D, NN>(a, S, dout, dt, nt, mode, st)
  if (dim == 2) { PINT_SWITCH_N(2, C_) }
  else {
    PINT_SWITCH_N(1, C_)
    if (n == 256) return C_(1, 256);
    if (n == 512) return C_(1, 512);
  }
#undef C_
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dct(int dim, int n, const T* in, T* out, const DctTables<T>& dt, int nt, bool inv,
                      hipStream_t st) {
#define C_(D, NN) launch_dct_n<T, D, NN>(in, out, dt, nt, inv, st)
  if (dim == 2) { PINT_SWITCH_N(2, C_) }
  else {
    PINT_SWITCH_N(1, C_)
    if (n == 256) return C_(1, 256);
    if (n == 512) return C_(1, 512);
  }
#undef C_
  return hipErrorInvalidValue;
}

// Time solve: tile width M (spatial modes per workgroup) is the largest of
// {8, 16, 32, 64} that divides ns and keeps the LDS tile (N_t x M/2 complex)
// within 64 KB, so that two workgroups can share a CU.
template <typename T, int NTT>
struct time_cfg {
  static constexpr int BYTES = NTT * int(sizeof(cx<T>));  // one complex column
  static constexpr int CMAX0 = 65536 / BYTES;
  static constexpr int MMAX = 2 * (CMAX0 < 32 ? CMAX0 : 32);
};

template <typename T, int NTT, int M>
static hipError_t launch_time_m(T* S, const TimeArgs<T>& ta, hipStream_t st) {
  if constexpr (M > time_cfg<T, NTT>::MMAX || M < 2) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_time_solve<T, NTT, M, 256>), dim3(ta.ns / M), dim3(256), 0, st, S, ta);
    PINT_CHECK_LAUNCH();
    return hipSuccess;
  }
}

template <typename T, int NTT>
static hipError_t launch_time_nt(T* S, const TimeArgs<T>& ta, hipStream_t st) {
  int m = time_cfg<T, NTT>::MMAX;
  while (m > 8 && (m > ta.ns || ta.ns % m != 0)) m /= 2;
  if (ta.ns % m != 0) return hipErrorInvalidValue;
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

hipError_t launch_finalize(const FinArgs& f, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, f);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_init(const InitArgs& a, Ctrl* c, double dof, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(a.nt), dim3(256), 0, st, a);
  PINT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(64), 0, st, c, a.nt, (const double*)a.part, dof);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template <typename T>
hipError_t launch_cast_to(const double* in, T* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_to<T>, dim3(1024), dim3(256), 0, st, in, out, n);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}
template <typename T>
hipError_t launch_cast_from(const T* in, double* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_from<T>, dim3(1024), dim3(256), 0, st, in, out, n);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_diagnostics(const DiagArgs& a, int nt, hipStream_t st) {
  hipLaunchKernelGGL(k_diagnostics, dim3(nt), dim3(256), 0, st, a);
  PINT_CHECK_LAUNCH();
  return hipSuccess;
}

template hipError_t launch_resid<float>(int, int, const ResidArgs&, float*, double*, const DctTables<float>&, int,
                                        int, hipStream_t);
template hipError_t launch_resid<double>(int, int, const ResidArgs&, double*, double*, const DctTables<double>&, int,
                                         int, hipStream_t);
template hipError_t launch_update<float>(int, int, const UpdArgs&, const float*, double*, const DctTables<float>&,
                                         int, int, hipStream_t);
template hipError_t launch_update<double>(int, int, const UpdArgs&, const double*, double*,
                                          const DctTables<double>&, int, int, hipStream_t);
template hipError_t launch_dct<float>(int, int, const float*, float*, const DctTables<float>&, int, bool,
                                      hipStream_t);
template hipError_t launch_dct<double>(int, int, const double*, double*, const DctTables<double>&, int, bool,
                                       hipStream_t);
template hipError_t launch_time<float>(int, float*, const TimeArgs<float>&, hipStream_t);
template hipError_t launch_time<double>(int, double*, const TimeArgs<double>&, hipStream_t);
template hipError_t launch_cast_to<float>(const double*, float*, size_t, hipStream_t);
template hipError_t launch_cast_to<double>(const double*, double*, size_t, hipStream_t);
template hipError_t launch_cast_from<float>(const float*, double*, size_t, hipStream_t);
template hipError_t launch_cast_from<double>(const double*, double*, size_t, hipStream_t);

}  // namespace pint

// a3-a5 as a dense contraction over the time index on the matrix cores.
//
// For one spatial cosine mode k the time solve of eq. pintiter1 (Steps 1-3;
// CH: eq. pintiter_CH, eq. pintiter_CH_eyre) maps the N_t real values x_n to
//   delta = Gamma^{-1} F^{-1} diag(1/sigma_{l,k}) F Gamma x.
// Because x, Gamma and a are real, F Gamma x is Hermitian and is carried by N_t
// real numbers, row r of y = W_f x:
//   r = 0: Re y_0      r = 1: Re y_{N_t/2}     r = 2l, 2l+1 (1 <= l < N_t/2): Re y_l, Im y_l
// with W_f[r][n] = a^n {1, (-1)^n, cos(2 pi l n/N_t), -sin(2 pi l n/N_t)}.  The
// divide acts on the pairs (rows 2l, 2l+1) as one complex division by sigma_{l,k}
// (rows 0 and 1 are real, divided by the real sigma_{0,k} and sigma_{N_t/2,k}),
// and the inverse is delta = W_b y' with
//   W_b[n][r] = a^{-n}/N_t {1, (-1)^n, 2 cos(2 pi l n/N_t), -2 sin(2 pi l n/N_t)}
// (Hermitian half-spectrum: y'_{N_t-l} = conj(y'_l)).  W_f and W_b are built
// in FP64 on the host.
//
// One workgroup (4 waves) handles NB consecutive modes: the N_t x NB tile is
// staged in LDS, y = W_f X runs on MFMA with FP32 accumulation, the divide is
// applied to the accumulators in registers (each lane holds both rows of a
// pair), y' goes back to LDS and delta = W_b y' runs on MFMA again.
//   DK_F32    v_mfma_f32_32x32x2_f32, operands FP32.
//   DK_BF16   v_mfma_f32_32x32x16_bf16, operands rounded to BF16.
//   DK_BF16X3 the same with a two-term split of both operands
//             (hi = bf16(v), lo = bf16(v - hi)): hi*hi + hi*lo + lo*hi.
// Flops per mode: 2 products of N_t x N_t by N_t -> 4 N_t^2 (x3 for DK_BF16X3).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "pint_kernels.hpp"

namespace pint {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int DPAD = 4;  // LDS row padding (floats)

// columns per workgroup: at least 32 (one MFMA block), and N_t * NB >= 4096 so
// that the 32 x 32 blocks split evenly over the 4 waves
constexpr int dense_nb(int ntt) { return ntt >= 128 ? 32 : 4096 / ntt; }

// acc[q] += A[rows of block q][:] * B[:, cols of block q] over the whole K = NTT.
// A comes from global memory (the W tables; L2-resident), B from the LDS tile
// xs[k][n] (row stride NB + DPAD).
template <int KIND, int NTT, int NB, int BPW>
__device__ __forceinline__ void gemm_tile(f32x16 (&acc)[BPW], const int (&rb)[BPW], const int (&cb)[BPW],
                                          const float* __restrict__ at, const void* ahv, const void* alv,
                                          const float* xs) {
  const __bf16* __restrict__ ah = static_cast<const __bf16*>(ahv);
  const __bf16* __restrict__ al = static_cast<const __bf16*>(alv);
  const int lane = threadIdx.x & 63;
  const int li = lane & 31, hi = lane >> 5;
  constexpr int LD = NB + DPAD;
#pragma unroll
  for (int q = 0; q < BPW; ++q) acc[q] = f32x16{};
  // Operands of chunk c + 1 are loaded while the MFMAs of chunk c run; the
  // chunk shrinks as the blocks per wave grow so the buffers stay small.
  if constexpr (KIND == DK_F32) {
    // A^T is stored [k][m]: a half-wave reads 32 consecutive floats
    constexpr int KS = BPW >= 8 ? 2 : (BPW >= 4 ? 4 : 8);  // MFMA k-steps (of 2) per chunk
    constexpr int NCH = NTT / (2 * KS);
    float ca[KS][BPW], cx_[KS][BPW], na[KS][BPW], nx[KS][BPW];
    auto load = [&](int c, float (&a)[KS][BPW], float (&b)[KS][BPW]) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = c * 2 * KS + 2 * s + hi;
#pragma unroll
        for (int q = 0; q < BPW; ++q) {
          a[s][q] = at[size_t(k) * NTT + rb[q] * 32 + li];
          b[s][q] = xs[k * LD + cb[q] * 32 + li];
        }
      }
    };
    load(0, ca, cx_);
    for (int c = 0; c < NCH; ++c) {
      if (c + 1 < NCH) load(c + 1, na, nx);
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int q = 0; q < BPW; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[s][q], cx_[s][q], acc[q], 0, 0, 0);
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int q = 0; q < BPW; ++q) {
          ca[s][q] = na[s][q];
          cx_[s][q] = nx[s][q];
        }
    }
  } else {
    // A is stored [m][k] in BF16: each lane reads 8 consecutive k (16 bytes)
    constexpr bool X3 = KIND == DK_BF16X3;
    constexpr int KS = BPW >= 4 ? 1 : 2;  // MFMA k-steps (of 16) per chunk
    constexpr int NCH = NTT / (16 * KS);
    bf16x8 ch[KS][BPW], cl[KS][BPW], nh[KS][BPW], nl[KS][BPW];
    auto load = [&](int c, bf16x8 (&h)[KS][BPW], bf16x8 (&l)[KS][BPW]) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int kb = (c * KS + s) * 16 + 8 * hi;
#pragma unroll
        for (int q = 0; q < BPW; ++q) {
          const size_t ao = size_t(rb[q] * 32 + li) * NTT + kb;
          h[s][q] = *reinterpret_cast<const bf16x8*>(ah + ao);
          if constexpr (X3) l[s][q] = *reinterpret_cast<const bf16x8*>(al + ao);
        }
      }
    };
    load(0, ch, cl);
    for (int c = 0; c < NCH; ++c) {
      if (c + 1 < NCH) load(c + 1, nh, nl);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int kb = (c * KS + s) * 16 + 8 * hi;
#pragma unroll
        for (int q = 0; q < BPW; ++q) {
          bf16x8 b_hi, b_lo;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float x = xs[(kb + j) * LD + cb[q] * 32 + li];
            b_hi[j] = __bf16(x);
            if constexpr (X3) b_lo[j] = __bf16(x - float(b_hi[j]));
          }
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch[s][q], b_hi, acc[q], 0, 0, 0);
          if constexpr (X3) {
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch[s][q], b_lo, acc[q], 0, 0, 0);
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cl[s][q], b_hi, acc[q], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int q = 0; q < BPW; ++q) {
          ch[s][q] = nh[s][q];
          if constexpr (X3) cl[s][q] = nl[s][q];
        }
    }
  }
}

// Row (within its 32 x 32 block) of accumulator element i of this lane.
__device__ __forceinline__ int acc_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

template <int KIND, int NTT>
__global__ __launch_bounds__(256) void k_time_dense(float* __restrict__ S, TimeArgs<float> ta, DenseArgs da) {
  if (ta.done && *ta.done) return;
  constexpr int NB = dense_nb(NTT);
  constexpr int LD = NB + DPAD;
  constexpr int NCB = NB / 32, NBLK = (NTT / 32) * NCB, BPW = NBLK / 4;
  static_assert(NBLK % 4 == 0 && BPW >= 1, "block split");
  __shared__ __align__(16) float xs[NTT * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col0 = blockIdx.x * NB;
  const size_t ns = ta.ns;

  // stage the N_t x NB tile (rows of NB consecutive floats), loads issued in
  // batches before they are stored
  {
    constexpr int V = NTT * NB / 4;  // float4 items
    constexpr int PER = V / 256;
    static_assert(V % 256 == 0, "tile split");
    constexpr int BATCH = PER < 8 ? PER : 8;
#pragma unroll
    for (int b0 = 0; b0 < PER; b0 += BATCH) {
      float4 v[BATCH];
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const int w = tid + (b0 + j) * 256;
        const int k = w / (NB / 4), c = (w - k * (NB / 4)) * 4;
        v[j] = *reinterpret_cast<const float4*>(S + size_t(k) * ns + col0 + c);
      }
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const int w = tid + (b0 + j) * 256;
        const int k = w / (NB / 4), c = (w - k * (NB / 4)) * 4;
        *reinterpret_cast<float4*>(xs + k * LD + c) = v[j];
      }
    }
  }
  int rb[BPW], cb[BPW];
#pragma unroll
  for (int q = 0; q < BPW; ++q) {
    const int b = wave * BPW + q;
    rb[q] = b / NCB;
    cb[q] = b - (b / NCB) * NCB;
  }
  __syncthreads();

  f32x16 acc[BPW];
  gemm_tile<KIND, NTT, NB, BPW>(acc, rb, cb, da.wf, da.wf_hi, da.wf_lo, xs);

  // divide the pairs (rows 2l, 2l+1) by sigma_{l,k} in the accumulators
  const float cbar = ta.cbar_mode ? float(ta.cbar ? *ta.cbar : ta.cbar_val) : 0.0f;
  if (da.direct) {
    // direct diagonalization: row j holds eigen-coordinate j, divided by the
    // real d_j + shift_k
#pragma unroll
    for (int q = 0; q < BPW; ++q) {
      const int k = col0 + cb[q] * 32 + (lane & 31);
      const float lk = ta.lamx[k % ta.nx] + ta.lamy[k / ta.nx];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = rb[q] * 32 + acc_row(i, lane);
        acc[q][i] = acc[q][i] / (ta.lam1[r].x + (ta.pco[r].x - cbar) * lk + ta.qco[r].x * lk * lk);
      }
    }
  } else
#pragma unroll
  for (int q = 0; q < BPW; ++q) {
    const int k = col0 + cb[q] * 32 + (lane & 31);
    const float lk = ta.lamx[k % ta.nx] + ta.lamy[k / ta.nx];
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
      const int r = rb[q] * 32 + acc_row(i, lane);  // even
      const int l = r >> 1;
      if (l == 0) {
        // real pair: Re y_0 / sigma_0 and Re y_{N_t/2} / sigma_{N_t/2}
        const float s0 = ta.lam1[0].x + (ta.pco[0].x - cbar) * lk + ta.qco[0].x * lk * lk;
        const int h = NTT / 2;
        const float sh = ta.lam1[h].x + (ta.pco[h].x - cbar) * lk + ta.qco[h].x * lk * lk;
        acc[q][i] = acc[q][i] / s0;
        acc[q][i + 1] = acc[q][i + 1] / sh;
      } else {
        const cx<float> l1 = ta.lam1[l], p = ta.pco[l], qq = ta.qco[l];
        const cx<float> sg = mk(l1.x + (p.x - cbar) * lk + qq.x * lk * lk, l1.y + p.y * lk + qq.y * lk * lk);
        const cx<float> y = cdiv(mk(acc[q][i], acc[q][i + 1]), sg);
        acc[q][i] = y.x;
        acc[q][i + 1] = y.y;
      }
    }
  }
  __syncthreads();  // every wave is done reading the tile
#pragma unroll
  for (int q = 0; q < BPW; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) xs[(rb[q] * 32 + acc_row(i, lane)) * LD + cb[q] * 32 + (lane & 31)] = acc[q][i];
  __syncthreads();

  gemm_tile<KIND, NTT, NB, BPW>(acc, rb, cb, da.wb, da.wb_hi, da.wb_lo, xs);
#pragma unroll
  for (int q = 0; q < BPW; ++q)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int n = rb[q] * 32 + acc_row(i, lane);
      S[size_t(n) * ns + col0 + cb[q] * 32 + (lane & 31)] = acc[q][i];
    }
}

// ---------------------------------------------------------------------------
// BF16 kinds at N_t >= 256: both operand tiles live in LDS as BF16,
// transposed ([column][k], row stride N_t + 8), so that a lane's B operand
// (8 consecutive k of one column) is one 16-byte read, and the FP32 -> BF16
// rounding (and the hi/lo split) is done once per element: when the tile is
// staged, and when y' is written back after the divide.  NW waves and NCB
// column blocks of 32 modes; wave w owns the RPW row blocks from w RPW and
// every column block, so each A fragment (W from global memory) feeds NCB
// MFMAs.
template <int NTT, int NW, int NCB>
struct b16_cfg {
  static constexpr int NB = 32 * NCB, LDK = NTT + 8, NT = 64 * NW, RPW = NTT / 32 / NW;
};

template <int KIND, int NTT, int RPW, int NCB>
__device__ __forceinline__ void gemm_b16(f32x16 (&acc)[RPW][NCB], int rb0, const __bf16* __restrict__ ah,
                                         const __bf16* __restrict__ al, const __bf16* xh, const __bf16* xl) {
  constexpr bool X3 = KIND == DK_BF16X3;
  constexpr int LDK = NTT + 8;
  // MFMA k-steps (of 16) per chunk: the A fragments of two chunks (this one
  // and the next, in flight) stay within the register budget
  constexpr int KS = RPW * NCB * (X3 ? 2 : 1) >= 8 ? 1 : 2;
  constexpr int NCH = NTT / (16 * KS);
  const int lane = threadIdx.x & 63;
  const int li = lane & 31, hi = lane >> 5;
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c] = f32x16{};
  bf16x8 ch[KS][RPW], cl[KS][RPW], nh[KS][RPW], nl[KS][RPW];
  auto load = [&](int c, bf16x8 (&h)[KS][RPW], bf16x8 (&l)[KS][RPW]) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int kb = (c * KS + s) * 16 + 8 * hi;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const size_t ao = size_t((rb0 + r) * 32 + li) * NTT + kb;
        h[s][r] = *reinterpret_cast<const bf16x8*>(ah + ao);
        if constexpr (X3) l[s][r] = *reinterpret_cast<const bf16x8*>(al + ao);
      }
    }
  };
  load(0, ch, cl);
  for (int c = 0; c < NCH; ++c) {
    if (c + 1 < NCH) load(c + 1, nh, nl);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int kb = (c * KS + s) * 16 + 8 * hi;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(xh + (cb * 32 + li) * LDK + kb);
        bf16x8 bl;
        if constexpr (X3) bl = *reinterpret_cast<const bf16x8*>(xl + (cb * 32 + li) * LDK + kb);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          acc[r][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch[s][r], bh, acc[r][cb], 0, 0, 0);
          if constexpr (X3) {
            acc[r][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch[s][r], bl, acc[r][cb], 0, 0, 0);
            acc[r][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cl[s][r], bh, acc[r][cb], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        ch[s][r] = nh[s][r];
        if constexpr (X3) cl[s][r] = nl[s][r];
      }
  }
}

// BF16 hi part (round to nearest even) and, for the split, the BF16 of the
// remainder.
template <bool X3>
__device__ __forceinline__ void split_bf16(float x, __bf16& h, __bf16& l) {
  h = __bf16(x);
  if constexpr (X3) l = __bf16(x - float(h));
}

template <int KIND, int NTT, int NW, int NCB>
__global__ __launch_bounds__(64 * NW) void k_time_dense_b16(float* __restrict__ S, TimeArgs<float> ta,
                                                             DenseArgs da) {
  if (ta.done && *ta.done) return;
  using C = b16_cfg<NTT, NW, NCB>;
  constexpr bool X3 = KIND == DK_BF16X3;
  constexpr int NB = C::NB, LDK = C::LDK, NT = C::NT, RPW = C::RPW;
  static_assert(RPW >= 1 && (NTT / 32) % NW == 0, "row blocks per wave");
  __shared__ __align__(16) __bf16 xh[NB * LDK];
  __shared__ __align__(16) __bf16 xl[X3 ? NB * LDK : 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col0 = blockIdx.x * NB;
  const size_t ns = ta.ns;
  const int rb0 = wave * RPW;

  // stage: item (k8, n) = S[8 k8 .. 8 k8 + 7][col0 + n] -> 16 bytes of row n
  {
    constexpr int ITEMS = (NTT / 8) * NB, PER = ITEMS / NT;
    static_assert(ITEMS % NT == 0, "stage split");
    constexpr int BATCH = PER < 4 ? PER : 4;
    static_assert(PER % BATCH == 0, "stage batches");
#pragma unroll 1
    for (int b0 = 0; b0 < PER; b0 += BATCH) {
      float v[BATCH][8];
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const int w = tid + (b0 + j) * NT;
        const int k8 = w / NB, n = w - (w / NB) * NB;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[j][e] = S[size_t(8 * k8 + e) * ns + col0 + n];
      }
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const int w = tid + (b0 + j) * NT;
        const int k8 = w / NB, n = w - (w / NB) * NB;
        bf16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 he, le;
          split_bf16<X3>(v[j][e], he, le);
          h[e] = he;
          if constexpr (X3) l[e] = le;
        }
        *reinterpret_cast<bf16x8*>(xh + n * LDK + 8 * k8) = h;
        if constexpr (X3) *reinterpret_cast<bf16x8*>(xl + n * LDK + 8 * k8) = l;
      }
    }
  }
  __syncthreads();

  f32x16 acc[RPW][NCB];
  gemm_b16<KIND, NTT, RPW, NCB>(acc, rb0, static_cast<const __bf16*>(da.wf_hi),
                                 static_cast<const __bf16*>(da.wf_lo), xh, xl);

  // divide the pairs (rows 2l, 2l+1) by sigma_{l,k} in the accumulators
  const float cbar = ta.cbar_mode ? float(ta.cbar ? *ta.cbar : ta.cbar_val) : 0.0f;
  float lk[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int k = col0 + cb * 32 + (lane & 31);
    lk[cb] = ta.lamx[k % ta.nx] + ta.lamy[k / ta.nx];
  }
  // one pair of rows at a time: its coefficients serve every column block;
  // the empty asm keeps the compiler from hoisting the coefficient loads of
  // all row blocks at once (registers)
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
      const int row = (rb0 + r) * 32 + acc_row(i, lane);  // even
      const int l = row >> 1;
      // l = 0: the real pair Re y_0 / sigma_0 and Re y_{N_t/2} / sigma_{N_t/2}
      const int l2 = l == 0 ? NTT / 2 : l;
      const cx<float> l1 = ta.lam1[l], p = ta.pco[l], qq = ta.qco[l];
      const cx<float> l1h = ta.lam1[l2], ph = ta.pco[l2], qh = ta.qco[l2];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float x = lk[cb];
        float a0 = acc[r][cb][i], a1 = acc[r][cb][i + 1];
        if (l == 0) {
          a0 = a0 / (l1.x + (p.x - cbar) * x + qq.x * x * x);
          a1 = a1 / (l1h.x + (ph.x - cbar) * x + qh.x * x * x);
        } else {
          const cx<float> sg = mk(l1.x + (p.x - cbar) * x + qq.x * x * x, l1.y + p.y * x + qq.y * x * x);
          const cx<float> y = cdiv(mk(a0, a1), sg);
          a0 = y.x;
          a1 = y.y;
        }
        acc[r][cb][i] = a0;
        acc[r][cb][i + 1] = a1;
      }
    }
  }
  __syncthreads();  // every wave is done reading the staged tile
  // y' back to LDS, transposed: rows acc_row(4g .. 4g+3) are consecutive
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int row = (rb0 + r) * 32 + acc_row(4 * g, lane);
        const int n = cb * 32 + (lane & 31);
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          __bf16 he, le;
          split_bf16<X3>(acc[r][cb][4 * g + e], he, le);
          h[e] = he;
          if constexpr (X3) l[e] = le;
        }
        *reinterpret_cast<bf16x4*>(xh + n * LDK + row) = h;
        if constexpr (X3) *reinterpret_cast<bf16x4*>(xl + n * LDK + row) = l;
      }
  __syncthreads();

  gemm_b16<KIND, NTT, RPW, NCB>(acc, rb0, static_cast<const __bf16*>(da.wb_hi),
                                 static_cast<const __bf16*>(da.wb_lo), xh, xl);
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int n = (rb0 + r) * 32 + acc_row(i, lane);
        S[size_t(n) * ns + col0 + cb * 32 + (lane & 31)] = acc[r][cb][i];
      }
}

template <int KIND, int NTT>
hipError_t launch_dense_nt(float* S, const TimeArgs<float>& ta, const DenseArgs& da, hipStream_t st) {
  if constexpr (KIND != DK_F32 && NTT >= 256) {
    // BF16 kinds: LDS-resident BF16 tiles; 64 columns for the single product,
    // 32 for the split (its hi and lo tiles), 8 waves
    constexpr int NCB = KIND == DK_BF16 ? 2 : 1;
    using C = b16_cfg<NTT, 8, NCB>;
    if (!da.direct && ta.ns % C::NB == 0) {
      PINT_LAUNCH((k_time_dense_b16<KIND, NTT, 8, NCB>), dim3(ta.ns / C::NB), dim3(C::NT), 0, st, S, ta, da);
      return hipGetLastError();
    }
  }
  constexpr int NB = dense_nb(NTT);
  if (ta.ns % NB != 0) return hipErrorInvalidValue;
  PINT_LAUNCH((k_time_dense<KIND, NTT>), dim3(ta.ns / NB), dim3(256), 0, st, S, ta, da);
  return hipGetLastError();
}

template <int KIND>
hipError_t launch_dense_kind(int nt, float* S, const TimeArgs<float>& ta, const DenseArgs& da, hipStream_t st) {
  switch (nt) {
    case 32: return launch_dense_nt<KIND, 32>(S, ta, da, st);
    case 64: return launch_dense_nt<KIND, 64>(S, ta, da, st);
    case 128: return launch_dense_nt<KIND, 128>(S, ta, da, st);
    case 256: return launch_dense_nt<KIND, 256>(S, ta, da, st);
    case 512: return launch_dense_nt<KIND, 512>(S, ta, da, st);
    case 1024: return launch_dense_nt<KIND, 1024>(S, ta, da, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// FP64 eigendecomposition of the time-step pencil (B, C) of the theta-method
// with steps dt_1..dt_{N_t}: B = diag(1/dt_n)(I - S), C = theta I + (1 - theta) S.
// B - d C is lower bidiagonal, so d_j = 1/(theta dt_j) and thread j obtains
//   the right eigenvector by forward substitution (v_n = 0 for n < j, v_j = 1,
//   v_n = v_{n-1} (1/dt_n + d_j (1-theta)) / (1/dt_n - d_j theta) for n > j),
//   the left one by backward substitution (w_m = 0 for m > j, w_j = 1,
//   w_m = w_{m+1} (1/dt_{m+1} + d_j (1-theta)) / (1/dt_m - d_j theta), m < j),
// then scales v to unit 2-norm and w so that w^T C v = 1 (w^T C v = theta w_j
// v_j before scaling, the other terms vanish).  With distinct steps the
// eigenvalues are distinct and (B + mu C)^{-1} = V (D + mu)^{-1} W.
__global__ __launch_bounds__(64) void k_eig_steps(EigArgs a) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= a.nt) return;
  const int nt = a.nt;
  const double th = a.theta, omth = 1.0 - a.theta;
  const double d = 1.0 / (th * a.dts[j]);
  double v = 1.0, nrm2 = 1.0;
  for (int n = j + 1; n < nt; ++n) {
    const double idt = 1.0 / a.dts[n];
    v = v * (idt + d * omth) / (idt - d * th);
    nrm2 += v * v;
  }
  const double s = 1.0 / sqrt(nrm2);
  // second pass: store the scaled right eigenvector
  for (int n = 0; n < j; ++n) a.v64[size_t(n) * nt + j] = 0.0;
  v = s;
  a.v64[size_t(j) * nt + j] = v;
  a.wbT[size_t(j) * nt + j] = float(v);
  for (int n = j + 1; n < nt; ++n) {
    const double idt = 1.0 / a.dts[n];
    v = v * (idt + d * omth) / (idt - d * th);
    a.v64[size_t(n) * nt + j] = v;
    a.wbT[size_t(j) * nt + n] = float(v);
  }
  for (int n = 0; n < j; ++n) a.wbT[size_t(j) * nt + n] = 0.0f;
  // left eigenvector, scaled by 1 / (theta s)
  double w = 1.0 / (th * s);
  a.w64[size_t(j) * nt + j] = w;
  a.wfT[size_t(j) * nt + j] = float(w);
  for (int m = j - 1; m >= 0; --m) {
    w = w * (1.0 / a.dts[m + 1] + d * omth) / (1.0 / a.dts[m] - d * th);
    a.w64[size_t(j) * nt + m] = w;
    a.wfT[size_t(m) * nt + j] = float(w);
  }
  for (int m = j + 1; m < nt; ++m) {
    a.w64[size_t(j) * nt + m] = 0.0;
    a.wfT[size_t(m) * nt + j] = 0.0f;
  }
  a.lam1d[j] = mk(d, 0.0);
  a.lam1f[j] = mk(float(d), 0.0f);
}

// Direct-diagonalization time solve in FP64: per spatial mode k (a column of
// S), y = W x, y_j /= d_j + shift_k, x = V y.  One workgroup takes NB modes;
// the tile and the intermediate stay in LDS; thread (row group g, column c)
// accumulates rows g, g + NG, ... of its column.
template <int NTT>
__global__ __launch_bounds__(256) void k_time_direct64(double* __restrict__ S, TimeArgs<double> ta, DenseArgs da) {
  if (ta.done && *ta.done) return;
  constexpr int NB = NTT >= 512 ? 8 : (NTT >= 256 ? 16 : 32);
  constexpr int NG = 256 / NB, R = NTT / NG;
  __shared__ double xs[NTT * NB];
  const int tid = threadIdx.x, c = tid % NB, g = tid / NB;
  const size_t col0 = size_t(blockIdx.x) * NB;
  const size_t ns = ta.ns;
  for (int w = tid; w < NTT * NB; w += 256) {
    const int n = w / NB, cc = w - (w / NB) * NB;
    xs[w] = S[size_t(n) * ns + col0 + cc];
  }
  __syncthreads();
  const double cbar = ta.cbar_mode ? (ta.cbar ? *ta.cbar : ta.cbar_val) : 0.0;
  const size_t k = col0 + c;
  const double lk = ta.lamx[k % ta.nx] + ta.lamy[k / ta.nx];
  double acc[R];
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = 0.0;
  for (int n = 0; n < NTT; ++n) {
    const double x = xs[n * NB + c];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] += da.w64[size_t(g + i * NG) * NTT + n] * x;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = g + i * NG;
    acc[i] /= ta.lam1[j].x + (ta.pco[j].x - cbar) * lk + ta.qco[j].x * lk * lk;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R; ++i) xs[(g + i * NG) * NB + c] = acc[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = 0.0;
  for (int j = 0; j < NTT; ++j) {
    const double y = xs[j * NB + c];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] += da.v64[size_t(g + i * NG) * NTT + j] * y;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) S[size_t(g + i * NG) * ns + k] = acc[i];
}

template <int NTT>
hipError_t launch_direct64_nt(double* S, const TimeArgs<double>& ta, const DenseArgs& da, hipStream_t st) {
  constexpr int NB = NTT >= 512 ? 8 : (NTT >= 256 ? 16 : 32);
  if (ta.ns % NB != 0) return hipErrorInvalidValue;
  PINT_LAUNCH((k_time_direct64<NTT>), dim3(ta.ns / NB), dim3(256), 0, st, S, ta, da);
  return hipGetLastError();
}

}  // namespace

int dense_cols_per_block(int nt) { return nt >= 32 ? dense_nb(nt) : 0; }

hipError_t launch_eig_steps(const EigArgs& a, hipStream_t st) {
  PINT_LAUNCH(k_eig_steps, dim3((a.nt + 63) / 64), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_time_direct64(int nt, double* S, const TimeArgs<double>& ta, const DenseArgs& da,
                                hipStream_t st) {
  switch (nt) {
    case 32: return launch_direct64_nt<32>(S, ta, da, st);
    case 64: return launch_direct64_nt<64>(S, ta, da, st);
    case 128: return launch_direct64_nt<128>(S, ta, da, st);
    case 256: return launch_direct64_nt<256>(S, ta, da, st);
    case 512: return launch_direct64_nt<512>(S, ta, da, st);
    case 1024: return launch_direct64_nt<1024>(S, ta, da, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_time_dense(int kind, int nt, float* S, const TimeArgs<float>& ta, const DenseArgs& da,
                             hipStream_t st) {
  switch (kind) {
    case DK_F32: return launch_dense_kind<DK_F32>(nt, S, ta, da, st);
    case DK_BF16: return launch_dense_kind<DK_BF16>(nt, S, ta, da, st);
    case DK_BF16X3: return launch_dense_kind<DK_BF16X3>(nt, S, ta, da, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pint

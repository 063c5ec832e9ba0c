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

template <int KIND, int NTT>
hipError_t launch_dense_nt(float* S, const TimeArgs<float>& ta, const DenseArgs& da, hipStream_t st) {
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

}  // namespace

int dense_cols_per_block(int nt) { return nt >= 32 ? dense_nb(nt) : 0; }

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

// Device-side building blocks shared by the solver kernels: a small complex
// type, block-wide reductions through LDS, and compile-time helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pint {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> mulc(cx<T> a, cx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
// i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return mk(-a.y, a.x); }
// -i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return mk(a.y, -a.x); }
// a / b (Smith's algorithm is not needed: |b| is bounded away from 0 and
// from overflow by construction of the shifts)
template <typename T>
__device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = T(1) / (b.x * b.x + b.y * b.y);
  return mk((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// a / b with the hardware reciprocal in FP32 (1 ulp) and an IEEE divide in
// FP64; for the diagonal solves of the preconditioner.
__device__ __forceinline__ float recip_fast(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip_fast(double d) { return 1.0 / d; }
template <typename T>
__device__ __forceinline__ cx<T> cdiv_fast(cx<T> a, cx<T> b) {
  const T d = recip_fast(b.x * b.x + b.y * b.y);
  return mk((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// Offset of mode q of level lev in a spectral array stored as panels of
// 2^tps modes: panel q >> tps holds that range of modes for all nlev levels,
// level-major.  tps = log2(modes per level) gives the plain [level][mode]
// layout.
__device__ __forceinline__ size_t panel_index(int lev, int q, int tps, int nlev) {
  return ((size_t(q >> tps) * size_t(nlev) + size_t(lev)) << tps) + size_t(q & ((1 << tps) - 1));
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int cdiv_i(int a, int b) { return (a + b - 1) / b; }

// Block-wide sum / max of NV doubles per thread, through LDS.  `scratch`
// must hold NT * NV doubles.  Every thread receives the results.  The
// reduction order is fixed (tree over thread index), so results are
// bitwise reproducible run to run.
template <int NT, int NV>
__device__ __forceinline__ void block_reduce(double* scratch, double (&v)[NV], const bool (&is_max)[NV]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NV; ++q) scratch[q * NT + tid] = v[q];
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        double a = scratch[q * NT + tid], b = scratch[q * NT + tid + s];
        // max keeps a NaN from either side so that divergence is detected
        scratch[q * NT + tid] = is_max[q] ? ((a != a || a > b) ? a : b) : a + b;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = scratch[q * NT];
  __syncthreads();
}

// Same contract as block_reduce (fixed combination order, NaN-propagating
// max), in two levels: an xor-shuffle tree inside each wave, then wave 0
// combines the per-wave results from LDS.  One barrier instead of log2(NT).
// The result is valid in thread 0.  scratch: NV * (NT / 64) doubles.
template <int NT, int NV>
__device__ __forceinline__ void block_reduce_waves(double* scratch, double (&v)[NV], const bool (&is_max)[NV]) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double b = __shfl_xor(v[q], off, 64);
      v[q] = is_max[q] ? ((v[q] != v[q] || v[q] > b) ? v[q] : b) : v[q] + b;
    }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) scratch[q * NW + wave] = v[q];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = lane < NW ? scratch[q * NW + lane] : 0.0;  // values are >= 0
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double b = __shfl_xor(v[q], off, 64);
        v[q] = is_max[q] ? ((v[q] != v[q] || v[q] > b) ? v[q] : b) : v[q] + b;
      }
  }
}

}  // namespace pint

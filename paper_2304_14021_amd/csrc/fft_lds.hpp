// Batched transforms on data resident in LDS: Stockham FFT (radix 4, one
// radix-2 stage when log2 N is odd) and the orthonormal DCT-II / DCT-III of
// real sequences computed through one complex FFT per pair of sequences.
//
// Layout of the complex FFT scratch: element m of sequence p lives at
// z[m * ES + p] ("element-major"), ES >= P.  Consecutive threads take
// consecutive p, so every FFT stage reads and writes consecutive LDS words.
// Each stage reads all of its inputs into registers, synchronizes, then
// writes, so the transform runs in place in the same LDS buffer.
//
// Twiddle table `tw` (global, read-only): tw[m] = exp(-2 pi i m / N), m < N,
// computed in FP64 on the host and rounded to T.
#pragma once

#include "device_common.hpp"

namespace pint {

// One Stockham stage of radix R on P sequences of length N (sign SIGN of the
// exponent: -1 forward, +1 inverse, unnormalized).  Ns = product of the radices
// of the previous stages.
template <typename T, int N, int P, int ES, int NT, int R, int SIGN>
__device__ __forceinline__ void fft_stage(cx<T>* z, const cx<T>* __restrict__ tw, int Ns) {
  constexpr int W = (N / R) * P;
  constexpr int IPT = cdiv_i(W, NT);
  const int tid = threadIdx.x;
  cx<T> v[IPT][R];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int w = tid + i * NT;
    if ((W % NT == 0) || w < W) {
      const int t = w / P, p = w - (w / P) * P;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = z[(t + r * (N / R)) * ES + p];
      const int k = t & (Ns - 1);
      const int step = k * (N / (Ns * R));
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w_ = tw[step * r];
        v[i][r] = (SIGN < 0) ? mul(v[i][r], w_) : mulc(v[i][r], w_);
      }
      if constexpr (R == 2) {
        cx<T> a = v[i][0], b = v[i][1];
        v[i][0] = add(a, b);
        v[i][1] = sub(a, b);
      } else {
        cx<T> a = add(v[i][0], v[i][2]), b = sub(v[i][0], v[i][2]);
        cx<T> c = add(v[i][1], v[i][3]), d = sub(v[i][1], v[i][3]);
        v[i][0] = add(a, c);
        v[i][2] = sub(a, c);
        // forward: X1 = b - i d, X3 = b + i d; inverse: signs swapped
        cx<T> id = (SIGN < 0) ? mul_mi(d) : mul_i(d);
        v[i][1] = add(b, id);
        v[i][3] = sub(b, id);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int w = tid + i * NT;
    if ((W % NT == 0) || w < W) {
      const int t = w / P, p = w - (w / P) * P;
      const int k = t & (Ns - 1);
      const int d = (t - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) z[(d + r * Ns) * ES + p] = v[i][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int P, int ES, int NT, int SIGN>
__device__ __forceinline__ void fft_lds(cx<T>* z, const cx<T>* __restrict__ tw) {
  constexpr int L = ilog2(N);
  int Ns = 1;
#pragma unroll
  for (int s = 0; s < L / 2; ++s) {
    fft_stage<T, N, P, ES, NT, 4, SIGN>(z, tw, Ns);
    Ns *= 4;
  }
  if constexpr ((L & 1) != 0) fft_stage<T, N, P, ES, NT, 2, SIGN>(z, tw, Ns);
}

// Source index j of the element that the DCT-via-FFT reordering puts at
// position m: v_m = x_{2m} (m < N/2), v_{N-1-m} = x_{2m+1}.
template <int N>
__device__ __forceinline__ int dct_perm(int m) {
  return (m < N / 2) ? 2 * m : 2 * (N - 1 - m) + 1;
}

// Complex scratch stride (in complex elements) used by the DCT passes: odd,
// so that both the row-major real array and the element-major complex array
// are walked without systematic bank conflicts.
template <int P>
struct dct_es {
  static constexpr int value = P + 1;
};

// LDS reals needed by a DCT pass over NB sequences of length N.
template <int N, int NB>
struct dct_lds_reals {
  static constexpr int value = 2 * N * (NB / 2 + 1);
};

// ---------------------------------------------------------------------------
// Orthonormal DCT-II along x of NB rows (NB even) of a row-major real array
// A (row stride LD >= N) in LDS, in place.  Rows 2p and 2p+1 are packed into
// one complex sequence.  wq[k] = s_k exp(-i pi k / (2N)), s_0 = sqrt(1/N),
// s_k = sqrt(2/N).  A's memory must span at least dct_lds_reals<N,NB> reals.
template <typename T, int N, int NB, int LD, int NT>
__device__ void dct2_rows(T* A, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ wq) {
  constexpr int P = NB / 2, ES = dct_es<P>::value;
  cx<T>* z = reinterpret_cast<cx<T>*>(A);
  const int tid = threadIdx.x;
  {  // pack: m fastest (reads walk a row), z[m*ES + p] = (x_{2p}[j], x_{2p+1}[j])
    constexpr int W = N * P, IPT = cdiv_i(W, NT);
    cx<T> v[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int p = w / N, m = w - (w / N) * N;
        const int j = dct_perm<N>(m);
        v[i] = mk(A[(2 * p) * LD + j], A[(2 * p + 1) * LD + j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int p = w / N, m = w - (w / N) * N;
        z[m * ES + p] = v[i];
      }
    }
    __syncthreads();
  }
  fft_lds<T, N, P, ES, NT, -1>(z, tw);
  {  // post-twiddle and split the two real transforms; k in [0, N/2]
    constexpr int K = N / 2 + 1, W = K * P, IPT = cdiv_i(W, NT);
    T o[IPT][4];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int p = w / K, k = w - (w / K) * K;
        const cx<T> zk = z[k * ES + p];
        const cx<T> zm = conj(z[((N - k) & (N - 1)) * ES + p]);
        const cx<T> v1 = scale(add(zk, zm), T(0.5));
        const cx<T> v2 = scale(mul_mi(sub(zk, zm)), T(0.5));
        const cx<T> wk = wq[k];
        const cx<T> wn = wq[(N - k) & (N - 1)];
        o[i][0] = wk.x * v1.x - wk.y * v1.y;          // Re(wq_k V1_k)
        o[i][1] = wk.x * v2.x - wk.y * v2.y;          // Re(wq_k V2_k)
        o[i][2] = wn.x * v1.x + wn.y * v1.y;          // Re(wq_{N-k} conj(V1_k))
        o[i][3] = wn.x * v2.x + wn.y * v2.y;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int p = w / K, k = w - (w / K) * K;
        A[(2 * p) * LD + k] = o[i][0];
        A[(2 * p + 1) * LD + k] = o[i][1];
        if (k > 0 && k < N / 2) {
          A[(2 * p) * LD + (N - k)] = o[i][2];
          A[(2 * p + 1) * LD + (N - k)] = o[i][3];
        }
      }
    }
    __syncthreads();
  }
}

// Orthonormal DCT-II along y (the columns) of a row-major N x N real array A
// (row stride LD) in LDS, in place.  Columns 2q and 2q+1 are packed into one
// complex sequence; consecutive threads take consecutive column pairs.
template <typename T, int N, int LD, int NT>
__device__ void dct2_cols(T* A, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ wq) {
  constexpr int P = N / 2, ES = dct_es<P>::value;
  cx<T>* z = reinterpret_cast<cx<T>*>(A);
  const int tid = threadIdx.x;
  {
    constexpr int W = N * P, IPT = cdiv_i(W, NT);
    cx<T> v[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int m = w / P, q = w - (w / P) * P;
        const int j = dct_perm<N>(m);
        v[i] = *reinterpret_cast<const cx<T>*>(A + j * LD + 2 * q);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int m = w / P, q = w - (w / P) * P;
        z[m * ES + q] = v[i];
      }
    }
    __syncthreads();
  }
  fft_lds<T, N, P, ES, NT, -1>(z, tw);
  {
    constexpr int K = N / 2 + 1, W = K * P, IPT = cdiv_i(W, NT);
    cx<T> o[IPT][2];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int k = w / P, q = w - (w / P) * P;
        const cx<T> zk = z[k * ES + q];
        const cx<T> zm = conj(z[((N - k) & (N - 1)) * ES + q]);
        const cx<T> v1 = scale(add(zk, zm), T(0.5));
        const cx<T> v2 = scale(mul_mi(sub(zk, zm)), T(0.5));
        const cx<T> wk = wq[k];
        const cx<T> wn = wq[(N - k) & (N - 1)];
        o[i][0] = mk(wk.x * v1.x - wk.y * v1.y, wk.x * v2.x - wk.y * v2.y);
        o[i][1] = mk(wn.x * v1.x + wn.y * v1.y, wn.x * v2.x + wn.y * v2.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int k = w / P, q = w - (w / P) * P;
        *reinterpret_cast<cx<T>*>(A + k * LD + 2 * q) = o[i][0];
        if (k > 0 && k < N / 2) *reinterpret_cast<cx<T>*>(A + (N - k) * LD + 2 * q) = o[i][1];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Inverse (orthonormal DCT-III) along x of NB rows, in place.
// wi[k] = exp(+i pi k / (2N)) / s_k.  Uses V_k = wi_k (X_k - i X_{N-k})
// (X_N = 0), whose inverse FFT is the reordered real sequence.
template <typename T, int N, int NB, int LD, int NT>
__device__ void dct3_rows(T* A, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ wi) {
  constexpr int P = NB / 2, ES = dct_es<P>::value;
  cx<T>* z = reinterpret_cast<cx<T>*>(A);
  const int tid = threadIdx.x;
  {
    constexpr int K = N / 2 + 1, W = K * P, IPT = cdiv_i(W, NT);
    cx<T> o[IPT][2];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int p = w / K, k = w - (w / K) * K;
        const T x1k = A[(2 * p) * LD + k], x2k = A[(2 * p + 1) * LD + k];
        const T x1m = k ? A[(2 * p) * LD + (N - k)] : T(0);
        const T x2m = k ? A[(2 * p + 1) * LD + (N - k)] : T(0);
        const cx<T> wk = wi[k];
        const cx<T> v1 = mul(wk, mk(x1k, -x1m));
        const cx<T> v2 = mul(wk, mk(x2k, -x2m));
        o[i][0] = add(v1, mul_i(v2));               // Z_k = V1_k + i V2_k
        o[i][1] = add(conj(v1), mul_i(conj(v2)));   // Z_{N-k}
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int p = w / K, k = w - (w / K) * K;
        z[k * ES + p] = o[i][0];
        if (k > 0 && k < N / 2) z[(N - k) * ES + p] = o[i][1];
      }
    }
    __syncthreads();
  }
  fft_lds<T, N, P, ES, NT, +1>(z, tw);
  {
    constexpr int W = N * P, IPT = cdiv_i(W, NT);
    cx<T> v[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int p = w / N, m = w - (w / N) * N;
        v[i] = scale(z[m * ES + p], T(1) / T(N));
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int p = w / N, m = w - (w / N) * N;
        const int j = dct_perm<N>(m);
        A[(2 * p) * LD + j] = v[i].x;
        A[(2 * p + 1) * LD + j] = v[i].y;
      }
    }
    __syncthreads();
  }
}

// Inverse (orthonormal DCT-III) along y of a row-major N x N array, in place.
template <typename T, int N, int LD, int NT>
__device__ void dct3_cols(T* A, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ wi) {
  constexpr int P = N / 2, ES = dct_es<P>::value;
  cx<T>* z = reinterpret_cast<cx<T>*>(A);
  const int tid = threadIdx.x;
  {
    constexpr int K = N / 2 + 1, W = K * P, IPT = cdiv_i(W, NT);
    cx<T> o[IPT][2];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int k = w / P, q = w - (w / P) * P;
        const cx<T> xk = *reinterpret_cast<const cx<T>*>(A + k * LD + 2 * q);
        cx<T> xm = mk(T(0), T(0));
        if (k) xm = *reinterpret_cast<const cx<T>*>(A + (N - k) * LD + 2 * q);
        const cx<T> wk = wi[k];
        const cx<T> v1 = mul(wk, mk(xk.x, -xm.x));
        const cx<T> v2 = mul(wk, mk(xk.y, -xm.y));
        o[i][0] = add(v1, mul_i(v2));
        o[i][1] = add(conj(v1), mul_i(conj(v2)));
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if (w < W) {
        const int k = w / P, q = w - (w / P) * P;
        z[k * ES + q] = o[i][0];
        if (k > 0 && k < N / 2) z[(N - k) * ES + q] = o[i][1];
      }
    }
    __syncthreads();
  }
  fft_lds<T, N, P, ES, NT, +1>(z, tw);
  {
    constexpr int W = N * P, IPT = cdiv_i(W, NT);
    cx<T> v[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int m = w / P, q = w - (w / P) * P;
        v[i] = scale(z[m * ES + q], T(1) / T(N));
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int w = tid + i * NT;
      if ((W % NT == 0) || w < W) {
        const int m = w / P, q = w - (w / P) * P;
        const int j = dct_perm<N>(m);
        *reinterpret_cast<cx<T>*>(A + j * LD + 2 * q) = v[i];
      }
    }
    __syncthreads();
  }
}

}  // namespace pint

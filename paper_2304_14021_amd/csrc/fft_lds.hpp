// Batched transforms on data resident in LDS: Stockham FFT (radix-8 stages,
// or radix-16 ones on request, then one radix-4 or radix-2 stage for the
// remaining factor) and the orthonormal DCT-II / DCT-III of real sequences
// computed through one complex FFT per pair of sequences.
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

// Radix-4 DFT of (x0, x1, x2, x3) in place; SIGN -1 forward, +1 inverse.
template <typename T, int SIGN>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
  const cx<T> a = add(x0, x2), b = sub(x0, x2), c = add(x1, x3), d = sub(x1, x3);
  const cx<T> id = (SIGN < 0) ? mul_mi(d) : mul_i(d);
  x0 = add(a, c);
  x2 = sub(a, c);
  x1 = add(b, id);
  x3 = sub(b, id);
}

// Radix-8 DFT in place: two radix-4 DFTs on the even and odd elements
// combined with the eighth roots of unity.
template <typename T, int SIGN>
__device__ __forceinline__ void dft8(cx<T> (&v)[8]) {
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, SIGN>(e0, e1, e2, e3);
  dft4<T, SIGN>(o0, o1, o2, o3);
  const T r = T(0.70710678118654752440);
  // w^k, w = exp(SIGN * 2 pi i / 8)
  const cx<T> w1 = mk(r, T(SIGN) * r);
  const cx<T> w3 = mk(-r, T(SIGN) * r);
  o1 = mul(o1, w1);
  o2 = (SIGN < 0) ? mul_mi(o2) : mul_i(o2);
  o3 = mul(o3, w3);
  v[0] = add(e0, o0);
  v[4] = sub(e0, o0);
  v[1] = add(e1, o1);
  v[5] = sub(e1, o1);
  v[2] = add(e2, o2);
  v[6] = sub(e2, o2);
  v[3] = add(e3, o3);
  v[7] = sub(e3, o3);
}

// Radix-16 DFT in place: with n = n2 + 4 n1 and k = k1 + 4 k2, radix-4 DFTs
// over n1 for each n2, the twiddles w16^(n2 k1), then radix-4 DFTs over n2
// for each k1.
template <typename T, int SIGN>
__device__ __forceinline__ void dft16(cx<T> (&v)[16]) {
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173), r = T(0.70710678118654752440);
  const T sg = T(SIGN);
  cx<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = v[n2];
    y[n2][1] = v[n2 + 4];
    y[n2][2] = v[n2 + 8];
    y[n2][3] = v[n2 + 12];
    dft4<T, SIGN>(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
  }
  // w16^m = exp(SIGN 2 pi i m / 16) for m = n2 k1 in {1, 2, 3, 4, 6, 9}
  y[1][1] = mul(y[1][1], mk(c1, sg * s1));
  y[1][2] = mul(y[1][2], mk(r, sg * r));
  y[1][3] = mul(y[1][3], mk(s1, sg * c1));
  y[2][1] = mul(y[2][1], mk(r, sg * r));
  y[2][2] = (SIGN < 0) ? mul_mi(y[2][2]) : mul_i(y[2][2]);
  y[2][3] = mul(y[2][3], mk(-r, sg * r));
  y[3][1] = mul(y[3][1], mk(s1, sg * c1));
  y[3][2] = mul(y[3][2], mk(-r, sg * r));
  y[3][3] = mul(y[3][3], mk(-c1, -sg * s1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
    dft4<T, SIGN>(a, b, c, d);
    v[k1] = a;
    v[k1 + 4] = b;
    v[k1 + 8] = c;
    v[k1 + 12] = d;
  }
}

// Twiddle accessors: exp(-2 pi i m / N) from a full table (each twiddle of
// a butterfly read), or from two short tables as tw_hi[m / 32] * tw_lo[m % 32]
// with the butterfly's other twiddles formed as powers of its first one
// (a few ulp; fewer LDS reads and a table of 2 sqrt(N) entries).
template <typename T>
struct TwTable {
  static constexpr bool POW = false;
  const cx<T>* t;
  __device__ __forceinline__ cx<T> operator()(int m) const { return t[m]; }
};
template <typename T>
struct TwSplit {
  static constexpr bool POW = true;
  const cx<T>* hi;
  const cx<T>* lo;
  __device__ __forceinline__ cx<T> operator()(int m) const { return mul(hi[m >> 5], lo[m & 31]); }
};

// w[r] = w1^r, r = 1 .. R-1, by products of depth at most 3.
template <typename T, int R>
__device__ __forceinline__ void tw_powers(cx<T> (&w)[R], cx<T> w1) {
  w[1] = w1;
  if constexpr (R > 2) {
    w[2] = mul(w1, w1);
    w[3] = mul(w[2], w1);
  }
  if constexpr (R > 4) {
    w[4] = mul(w[2], w[2]);
    w[5] = mul(w[4], w1);
    w[6] = mul(w[3], w[3]);
    w[7] = mul(w[4], w[3]);
  }
  if constexpr (R > 8) {
#pragma unroll
    for (int r = 8; r < R; ++r) w[r] = mul(w[r - 4], w[4]);
  }
}

// Row of element m in the LDS buffer: with SKEW one padding row follows
// every 8 rows, so that the stride-R row writes of a stage fall in different
// banks when a row is narrow (32 bytes).
template <bool SKEW>
__host__ __device__ constexpr int zrow(int m) { return SKEW ? m + (m >> 3) : m; }
template <bool SKEW>
__host__ __device__ constexpr int zrows(int n) { return SKEW ? n + n / 8 : n; }

// One Stockham stage of radix R (2, 4 or 8) on P sequences of length N
// (SIGN -1 forward, +1 inverse, unnormalized).  Ns = product of the radices
// of the previous stages (the first stage, Ns = 1, has no twiddles).
template <typename T, int N, int P, int ES, int NT, int R, int SIGN, bool SKEW, int Ns, typename TW>
__device__ __forceinline__ void fft_stage_tw(cx<T>* z, const TW& tw) {
  constexpr int W = (N / R) * P;
  constexpr int IPT = cdiv_i(W, NT);
  // Rows t + r N/R and d + r Ns; with SKEW and N/R, Ns multiples of 8 the
  // padding rows split off as constant strides (one address per item).  The
  // first stage writes d = R t, d + r with r < R <= 8 in the same group of 8.
  constexpr int SRC = SKEW ? (N / R) + (N / R) / 8 : N / R;
  constexpr int DST = SKEW ? (Ns >= 8 ? Ns + Ns / 8 : 1) : Ns;
  static_assert(!SKEW || Ns == 1 || Ns % 8 == 0, "stage strides");
  // first stage with padding: d = R t is a multiple of 8, so row d + r sits
  // r + r / 8 rows after row d
  auto dst_off = [](int r) {
    if constexpr (SKEW && Ns == 1) return r + (r >> 3);
    else return r * DST;
  };
  auto src_row = [](int t, int r) {
    if constexpr (!SKEW || (N / R) % 8 == 0) return zrow<SKEW>(t) + r * SRC;
    else return zrow<SKEW>(t + r * (N / R));
  };
  const int tid = threadIdx.x;
  cx<T> v[IPT][R];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int w = tid + i * NT;
    if ((W % NT == 0) || w < W) {
      const int t = w / P, p = w - (w / P) * P;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = z[src_row(t, r) * ES + p];
      if constexpr (Ns > 1) {
        const int k = t & (Ns - 1);
        const int step = k * (N / (Ns * R));
        if constexpr (TW::POW) {
          cx<T> w[R];
          tw_powers<T, R>(w, tw(step));
#pragma unroll
          for (int r = 1; r < R; ++r) v[i][r] = (SIGN < 0) ? mul(v[i][r], w[r]) : mulc(v[i][r], w[r]);
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const cx<T> w_ = tw(step * r);
            v[i][r] = (SIGN < 0) ? mul(v[i][r], w_) : mulc(v[i][r], w_);
          }
        }
      }
      if constexpr (R == 2) {
        const cx<T> a = v[i][0], b = v[i][1];
        v[i][0] = add(a, b);
        v[i][1] = sub(a, b);
      } else if constexpr (R == 4) {
        dft4<T, SIGN>(v[i][0], v[i][1], v[i][2], v[i][3]);
      } else if constexpr (R == 8) {
        dft8<T, SIGN>(v[i]);
      } else {
        dft16<T, SIGN>(v[i]);
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
      for (int r = 0; r < R; ++r) z[(zrow<SKEW>(d) + dst_off(r)) * ES + p] = v[i][r];
    }
  }
  __syncthreads();
}

// Complete FFT: radix-8 stages (radix-16 with R16), then one radix-4 or
// radix-2 stage for the remaining factor.  Input and output in natural order
// (Stockham autosort).
// Callers synchronize before the call (inputs written) and may read the
// result right after it (the last stage ends with a barrier).
template <typename T, int N, int P, int ES, int NT, int SIGN, bool SKEW, int Ns, bool R16, typename TW>
__device__ __forceinline__ void fft_stages_from(cx<T>* z, const TW& tw) {
  if constexpr (R16 && Ns * 16 <= N) {
    fft_stage_tw<T, N, P, ES, NT, 16, SIGN, SKEW, Ns>(z, tw);
    fft_stages_from<T, N, P, ES, NT, SIGN, SKEW, Ns * 16, R16>(z, tw);
  } else if constexpr (Ns * 8 <= N) {
    fft_stage_tw<T, N, P, ES, NT, 8, SIGN, SKEW, Ns>(z, tw);
    fft_stages_from<T, N, P, ES, NT, SIGN, SKEW, Ns * 8, R16>(z, tw);
  } else if constexpr (Ns * 4 == N) {
    fft_stage_tw<T, N, P, ES, NT, 4, SIGN, SKEW, Ns>(z, tw);
  } else if constexpr (Ns * 2 == N) {
    fft_stage_tw<T, N, P, ES, NT, 2, SIGN, SKEW, Ns>(z, tw);
  }
}

template <typename T, int N, int P, int ES, int NT, int SIGN, bool SKEW = false, bool R16 = false, typename TW>
__device__ __forceinline__ void fft_lds_tw(cx<T>* z, const TW& tw) {
  fft_stages_from<T, N, P, ES, NT, SIGN, SKEW, 1, R16>(z, tw);
}

template <typename T, int N, int P, int ES, int NT, int SIGN>
__device__ __forceinline__ void fft_lds(cx<T>* z, const cx<T>* __restrict__ tw) {
  fft_lds_tw<T, N, P, ES, NT, SIGN, false>(z, TwTable<T>{tw});
}

// Source index j of the element that the DCT-via-FFT reordering puts at
// position m: v_m = x_{2m} (m < N/2), v_{N-1-m} = x_{2m+1}.
template <int N>
__device__ __forceinline__ int dct_perm(int m) {
  return (m < N / 2) ? 2 * m : 2 * (N - 1 - m) + 1;
}

// Inverse of dct_perm: position m of source index j.
template <int N>
__device__ __forceinline__ int dct_iperm(int j) {
  return (j & 1) ? (N - 1 - (j >> 1)) : (j >> 1);
}

// After a forward FFT of the packed sequence z = x1 + i x2 (both reordered by
// dct_perm), the orthonormal DCT-II coefficients of x1 and x2 at k and N-k
// (k in [0, N/2]).  zk = Z_k, zn = Z_{N-k mod N}; wk = wq_k, wn = wq_{N-k mod N}
// with wq_k = s_k exp(-i pi k / (2N)).  With V1 = (Z_k + conj Z_{N-k})/2 and
// V2 = (Z_k - conj Z_{N-k})/(2i), X_k = Re(wq_k V_k) and
// X_{N-k} = Re(wq_{N-k} conj(V_k)).
template <typename T>
__device__ __forceinline__ void dct2_split(cx<T> zk, cx<T> zn, cx<T> wk, cx<T> wn, T& x1k, T& x2k, T& x1n,
                                           T& x2n) {
  const cx<T> zc = conj(zn);
  const cx<T> v1 = scale(add(zk, zc), T(0.5));
  const cx<T> v2 = scale(mul_mi(sub(zk, zc)), T(0.5));
  x1k = wk.x * v1.x - wk.y * v1.y;
  x2k = wk.x * v2.x - wk.y * v2.y;
  x1n = wn.x * v1.x + wn.y * v1.y;
  x2n = wn.x * v2.x + wn.y * v2.y;
}

// Before an inverse FFT: the packed spectrum Z_k, Z_{N-k} whose inverse FFT
// is (x1 + i x2) reordered by dct_perm, from the orthonormal DCT-II
// coefficients X1, X2 at k and N-k (X_N = 0).  wi_k = exp(+i pi k / (2N)) / s_k;
// V_k = wi_k (X_k - i X_{N-k}), V_{N-k} = conj(V_k), Z = V1 + i V2.
template <typename T>
__device__ __forceinline__ void dct3_join(T x1k, T x2k, T x1n, T x2n, cx<T> wik, cx<T>& zk, cx<T>& zn) {
  const cx<T> v1 = mul(wik, mk(x1k, -x1n));
  const cx<T> v2 = mul(wik, mk(x2k, -x2n));
  zk = add(v1, mul_i(v2));
  zn = add(conj(v1), mul_i(conj(v2)));
}

}  // namespace pint

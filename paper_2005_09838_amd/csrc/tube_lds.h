// Tube transforms that run in a thread's own LDS row (for the longer even tube lengths).
//
// A real tube of even length N = 2M is handled through the complex sequence
// c[m] = x[2m] + i x[2m+1] of length M (the half-length form of eq. (bar BA-k)), and the
// length-M complex transform is a four-step FFT with M = M1 * M2:
//   step A, for each n1 < M1: a length-M2 DFT over x[n1 + M1 n2], times exp(S 2 pi i n1 k2 / M),
//           stored back at complex position n1 + M1 k2;
//   step C, for each k2 < M2: a length-M1 DFT over those M1 values, result C[k2 + M2 k1]
//           stored at complex position k1 + M1 k2.
// The small DFTs are generated straight-line code (tube_dft_gen.h); the group loops stay
// rolled, so the code is short and needs few registers.
#pragma once
#include "common.h"
#include "tube_dft_gen.h"

template <int N>
struct TubeLds {
  static constexpr int M1 = TubePlan<N>::M1, M2 = TubePlan<N>::M2, M = N / 2;
  static constexpr bool enabled = M1 > 0;
  // complex position of C[k] after the four-step transform
  static __host__ __device__ constexpr int pos(int k) { return (k / M2) + M1 * (k % M2); }
  // float position of x[q] in the row after the inverse transform
  static __host__ __device__ constexpr int xpos(int q) { return 2 * pos(q >> 1) + (q & 1); }
};

// Twiddles for one block: twm[e] = exp(+2 pi i e / M), e < M;  twn[b] = exp(+2 pi i b / N), b <= M.
template <int N>
__device__ __forceinline__ void tube_twiddles(float2* twm, float2* twn) {
  constexpr int M = N / 2;
  for (int e = threadIdx.x; e < M; e += blockDim.x) {
    double s, c;
    sincospi(2.0 * e / M, &s, &c);
    twm[e] = make_float2((float)c, (float)s);
  }
  for (int b = threadIdx.x; b <= M; b += blockDim.x) {
    double s, c;
    sincospi(2.0 * b / N, &s, &c);
    twn[b] = make_float2((float)c, (float)s);
  }
}

template <int M1, int M2, int S>
__device__ __forceinline__ void fft4_lds(float* row, const float2* __restrict__ twm) {
  constexpr int M = M1 * M2;
#pragma unroll 1
  for (int n1 = 0; n1 < M1; ++n1) {
    float re[M2], im[M2];
#pragma unroll
    for (int n2 = 0; n2 < M2; ++n2) {
      re[n2] = row[2 * (n1 + M1 * n2)];
      im[n2] = row[2 * (n1 + M1 * n2) + 1];
    }
    dftc<M2, S>(re, im);
    int e = 0;
#pragma unroll
    for (int k2 = 0; k2 < M2; ++k2) {
      const float2 t = twm[e];
      const float c = t.x, s = S > 0 ? t.y : -t.y;
      row[2 * (n1 + M1 * k2)] = fmaf(re[k2], c, -im[k2] * s);
      row[2 * (n1 + M1 * k2) + 1] = fmaf(re[k2], s, im[k2] * c);
      e += n1;
      if (e >= M) e -= M;
    }
  }
#pragma unroll 1
  for (int k2 = 0; k2 < M2; ++k2) {
    float re[M1], im[M1];
#pragma unroll
    for (int n1 = 0; n1 < M1; ++n1) {
      re[n1] = row[2 * (n1 + M1 * k2)];
      im[n1] = row[2 * (n1 + M1 * k2) + 1];
    }
    dftc<M1, S>(re, im);
#pragma unroll
    for (int k1 = 0; k1 < M1; ++k1) {
      row[2 * (k1 + M1 * k2)] = re[k1];
      row[2 * (k1 + M1 * k2) + 1] = im[k1];
    }
  }
}

// Inverse transform (eq. (barAAk)) of the stored frequencies X[b] = src[b * stride],
// b = 0..M (imaginary parts of X[0] and X[M] taken as 0).  Afterwards M * x[q] sits at
// row[TubeLds<N>::xpos(q)].
//   E[b] = (X[b] + conj X[M-b]) / 2,  O[b] = (X[b] - conj X[M-b]) exp(-2 pi i b / N) / 2,
//   C[b] = E[b] + i O[b],  C[M-b] = conj E[b] + i conj O[b],  c = inverse DFT_M(C).
template <int N>
__device__ __forceinline__ void tube_inv_lds(const float2* __restrict__ src, size_t stride, float* row,
                                             const float2* __restrict__ twm, const float2* __restrict__ twn) {
  using T = TubeLds<N>;
  constexpr int M = T::M;
  float xr[M + 1], xi[M + 1];
#pragma unroll
  for (int b = 0; b <= M; ++b) {
    const float2 v = src[(size_t)b * stride];
    xr[b] = v.x;
    xi[b] = (b == 0 || b == M) ? 0.0f : v.y;
  }
#pragma unroll
  for (int b = 0; b <= M / 2; ++b) {
    const int mb = M - b;
    const float er = 0.5f * (xr[b] + xr[mb]), ei = 0.5f * (xi[b] - xi[mb]);
    const float dr = 0.5f * (xr[b] - xr[mb]), di = 0.5f * (xi[b] + xi[mb]);
    const float2 w = twn[b];
    const float orr = fmaf(dr, w.x, di * w.y), oi = fmaf(di, w.x, -dr * w.y);
    row[2 * b] = er - oi;
    row[2 * b + 1] = ei + orr;
    if (b != 0 && mb != b) {
      row[2 * mb] = er + oi;
      row[2 * mb + 1] = orr - ei;
    }
  }
  fft4_lds<T::M1, T::M2, -1>(row, twm);
}

// Forward transform (eq. (bar BA-k)) of the tube x = row[0..N) (natural order); calls
// store(b, re, im) for b = 0..M.
//   C = DFT_M(c),  E = (C[b] + conj C[M-b]) / 2,  O = (C[b] - conj C[M-b]) / (2i),
//   X[b] = E + exp(2 pi i b / N) O,  X[M-b] = conj(E - exp(2 pi i b / N) O),  X[M] = E[0] - O[0].
template <int N, class Store>
__device__ __forceinline__ void tube_fwd_lds(float* row, const float2* __restrict__ twm,
                                             const float2* __restrict__ twn, Store store) {
  using T = TubeLds<N>;
  constexpr int M = T::M;
  fft4_lds<T::M1, T::M2, +1>(row, twm);
#pragma unroll 2
  for (int b = 0; b <= M / 2; ++b) {
    const int mb = (b == 0) ? 0 : M - b;
    const int pb = 2 * T::pos(b), pm = 2 * T::pos(mb);
    const float cbr = row[pb], cbi = row[pb + 1], cmr = row[pm], cmi = row[pm + 1];
    const float er = 0.5f * (cbr + cmr), ei = 0.5f * (cbi - cmi);
    const float dr = 0.5f * (cbr - cmr), di = 0.5f * (cbi + cmi);
    const float orr = di, oi = -dr;   // D / i
    const float2 w = twn[b];
    const float wr = fmaf(w.x, orr, -w.y * oi), wi = fmaf(w.x, oi, w.y * orr);
    if (b == 0) {
      store(0, er + wr, 0.0f);
      store(M, er - wr, 0.0f);
    } else {
      store(b, er + wr, ei + wi);
      if (mb != b) store(mb, er - wr, wi - ei);
    }
  }
}

// ---------------------------------------------------------------- cooperative stages
// The same transforms with the groups of each stage spread over T threads of a tube
// (thread t takes groups t, t + T, ...); the caller separates the stages with block
// barriers.

// step A of the four-step transform: groups n1 = t, t + T, ...
template <int M1, int M2, int S>
__device__ __forceinline__ void fft4_step_a(float* row, const float2* __restrict__ twm, int t, int T) {
  constexpr int M = M1 * M2;
  for (int n1 = t; n1 < M1; n1 += T) {
    float re[M2], im[M2];
#pragma unroll
    for (int n2 = 0; n2 < M2; ++n2) {
      re[n2] = row[2 * (n1 + M1 * n2)];
      im[n2] = row[2 * (n1 + M1 * n2) + 1];
    }
    dftc<M2, S>(re, im);
    int e = 0;
#pragma unroll
    for (int k2 = 0; k2 < M2; ++k2) {
      const float2 w = twm[e];
      const float c = w.x, s = S > 0 ? w.y : -w.y;
      row[2 * (n1 + M1 * k2)] = fmaf(re[k2], c, -im[k2] * s);
      row[2 * (n1 + M1 * k2) + 1] = fmaf(re[k2], s, im[k2] * c);
      e += n1;
      if (e >= M) e -= M;
    }
  }
}

// step C: groups k2 = t, t + T, ...
template <int M1, int M2, int S>
__device__ __forceinline__ void fft4_step_c(float* row, int t, int T) {
  for (int k2 = t; k2 < M2; k2 += T) {
    float re[M1], im[M1];
#pragma unroll
    for (int n1 = 0; n1 < M1; ++n1) {
      re[n1] = row[2 * (n1 + M1 * k2)];
      im[n1] = row[2 * (n1 + M1 * k2) + 1];
    }
    dftc<M1, S>(re, im);
#pragma unroll
    for (int k1 = 0; k1 < M1; ++k1) {
      row[2 * (k1 + M1 * k2)] = re[k1];
      row[2 * (k1 + M1 * k2) + 1] = im[k1];
    }
  }
}

// pre-step of the inverse for the pairs b = t, t + T, ... <= M/2 (see tube_inv_lds); the
// bins of four pairs are loaded (from clamped addresses, unconditionally) before any of them
// is used, so a thread waits for one load latency per four pairs rather than per pair
template <int N>
__device__ __forceinline__ void tube_inv_pre(const float2* __restrict__ src, size_t stride, float* row,
                                             const float2* __restrict__ twn, int t, int T) {
  constexpr int M = N / 2, B = 8;
  for (int b0 = t; b0 <= M / 2; b0 += B * T) {
    float2 xbv[B], xmv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int b = b0 + u * T;
      const bool ok = b <= M / 2;
      xbv[u] = src[(size_t)(ok ? b : 0) * stride];
      xmv[u] = src[(size_t)(ok ? M - b : 0) * stride];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int b = b0 + u * T;
      if (b > M / 2) break;
      const int mb = M - b;
      const float2 xb = xbv[u], xm = xmv[u];
      const float xbr = xb.x, xbi = (b == 0) ? 0.0f : xb.y;
      const float xmr = xm.x, xmi = (b == 0) ? 0.0f : xm.y;
      const float er = 0.5f * (xbr + xmr), ei = 0.5f * (xbi - xmi);
      const float dr = 0.5f * (xbr - xmr), di = 0.5f * (xbi + xmi);
      const float2 w = twn[b];
      const float orr = fmaf(dr, w.x, di * w.y), oi = fmaf(di, w.x, -dr * w.y);
      row[2 * b] = er - oi;
      row[2 * b + 1] = ei + orr;
      if (b != 0 && mb != b) {
        row[2 * mb] = er + oi;
        row[2 * mb + 1] = orr - ei;
      }
    }
  }
}

// post-step of the forward transform for the pairs b = t, t + T, ... <= M/2 (see tube_fwd_lds)
template <int N, class Store>
__device__ __forceinline__ void tube_fwd_post(const float* row, const float2* __restrict__ twn, int t, int T,
                                              Store store) {
  using TL = TubeLds<N>;
  constexpr int M = N / 2;
  for (int b = t; b <= M / 2; b += T) {
    const int mb = (b == 0) ? 0 : M - b;
    const int pb = 2 * TL::pos(b), pm = 2 * TL::pos(mb);
    const float cbr = row[pb], cbi = row[pb + 1], cmr = row[pm], cmi = row[pm + 1];
    const float er = 0.5f * (cbr + cmr), ei = 0.5f * (cbi - cmi);
    const float dr = 0.5f * (cbr - cmr), di = 0.5f * (cbi + cmi);
    const float orr = di, oi = -dr;
    const float2 w = twn[b];
    const float wr = fmaf(w.x, orr, -w.y * oi), wi = fmaf(w.x, oi, w.y * orr);
    if (b == 0) {
      store(0, er + wr, 0.0f);
      store(M, er - wr, 0.0f);
    } else {
      store(b, er + wr, ei + wi);
      if (mb != b) store(mb, er - wr, wi - ei);
    }
  }
}

// step C with natural output order: the inputs of every group are read first (caller
// puts a block barrier between read and write), then C[k2 + M2 k1] goes to complex
// position k2 + M2 k1.  One group per thread: needs T >= M2.
template <int M1, int M2>
struct Fft4C {
  float re[M1], im[M1];
  __device__ __forceinline__ void read(const float* row, int t) {
    if (t < M2) {
#pragma unroll
      for (int n1 = 0; n1 < M1; ++n1) {
        re[n1] = row[2 * (n1 + M1 * t)];
        im[n1] = row[2 * (n1 + M1 * t) + 1];
      }
    }
  }
  template <int S>
  __device__ __forceinline__ void write(float* row, int t) {
    if (t < M2) {
      dftc<M1, S>(re, im);
#pragma unroll
      for (int k1 = 0; k1 < M1; ++k1) {
        row[2 * (t + M2 * k1)] = re[k1];
        row[2 * (t + M2 * k1) + 1] = im[k1];
      }
    }
  }
};

// Fft4C with the groups t and t + T of each thread (T < M2 <= 2 T).
template <int M1, int M2, int T>
struct Fft4C2 {
  static_assert(T < M2 && M2 <= 2 * T, "two groups per thread");
  float re[2][M1], im[2][M1];
  __device__ __forceinline__ void read(const float* row, int t) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = t + h * T;
      if (g < M2) {
#pragma unroll
        for (int n1 = 0; n1 < M1; ++n1) {
          re[h][n1] = row[2 * (n1 + M1 * g)];
          im[h][n1] = row[2 * (n1 + M1 * g) + 1];
        }
      }
    }
  }
  template <int S>
  __device__ __forceinline__ void write(float* row, int t) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = t + h * T;
      if (g < M2) {
        dftc<M1, S>(re[h], im[h]);
#pragma unroll
        for (int k1 = 0; k1 < M1; ++k1) {
          row[2 * (g + M2 * k1)] = re[h][k1];
          row[2 * (g + M2 * k1) + 1] = im[h][k1];
        }
      }
    }
  }
};

// post-step of the forward transform with C in natural order, pairs b = t, t + T, ...
template <int N, class Store>
__device__ __forceinline__ void tube_fwd_post_nat(const float* row, const float2* __restrict__ twn, int t, int T,
                                                  Store store) {
  constexpr int M = N / 2;
  for (int b = t; b <= M / 2; b += T) {
    const int mb = (b == 0) ? 0 : M - b;
    const float cbr = row[2 * b], cbi = row[2 * b + 1], cmr = row[2 * mb], cmi = row[2 * mb + 1];
    const float er = 0.5f * (cbr + cmr), ei = 0.5f * (cbi - cmi);
    const float dr = 0.5f * (cbr - cmr), di = 0.5f * (cbi + cmi);
    const float orr = di, oi = -dr;
    const float2 w = twn[b];
    const float wr = fmaf(w.x, orr, -w.y * oi), wi = fmaf(w.x, oi, w.y * orr);
    if (b == 0) {
      store(0, er + wr, 0.0f);
      store(M, er - wr, 0.0f);
    } else {
      store(b, er + wr, ei + wi);
      if (mb != b) store(mb, er - wr, wi - ei);
    }
  }
}

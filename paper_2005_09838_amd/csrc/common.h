// Shared device-side definitions of the TCTF2R gfx950 library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TCTF_RMAX 32          // largest tubal rank r supported by the r x r kernels
#define TCTF_N2MAX 1024       // largest n2 (slice kernel: one thread per tube of a slice)
#define TCTF_N1MAX 8192       // largest n1 (tridiagonal H_rho1 solve held in LDS)
#define TCTF_N3MAX 8192       // largest tube length n3
#define TCTF_SLICE_LDS_MAX (150 * 1024)

// Complex numbers: planar pairs in registers, float2 / double2 in memory.
struct cf { float re, im; };
struct cd { double re, im; };

__host__ __device__ __forceinline__ cd cd_make(double r, double i) { cd z; z.re = r; z.im = i; return z; }
__host__ __device__ __forceinline__ cd cd_add(cd a, cd b) { return cd_make(a.re + b.re, a.im + b.im); }
__host__ __device__ __forceinline__ cd cd_sub(cd a, cd b) { return cd_make(a.re - b.re, a.im - b.im); }
__host__ __device__ __forceinline__ cd cd_mul(cd a, cd b) {
  return cd_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
__host__ __device__ __forceinline__ cd cd_mulc(cd a, cd b) {
  return cd_make(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
// conj(a) * b
__host__ __device__ __forceinline__ cd cd_cmul(cd a, cd b) {
  return cd_make(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
__host__ __device__ __forceinline__ cd cd_conj(cd a) { return cd_make(a.re, -a.im); }
__host__ __device__ __forceinline__ cd cd_scale(cd a, double s) { return cd_make(a.re * s, a.im * s); }
// acc += a * b
__host__ __device__ __forceinline__ void cd_fma(cd& acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}

// BF16 with round-to-nearest-even (NaN kept quiet); stored as the upper half of a float.
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__host__ __device__ __forceinline__ float bf16_round(float x) { return bf16_to_f32(f32_to_bf16(x)); }
__host__ __device__ __forceinline__ uint32_t pack_bf16x2(float re, float im) {
  return (uint32_t)f32_to_bf16(re) | ((uint32_t)f32_to_bf16(im) << 16);
}
// MurmurHash3's 32-bit finaliser (Appleby): a bijective mixer, used as a counter-based
// generator of rounding bits.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
// BF16 by stochastic rounding: the 16 dropped bits are compared with 16 uniform random bits
// (added, then truncated), so the result rounds up with probability equal to the dropped
// fraction and its expectation is x.  Unlike round-to-nearest, its error is not the same
// every time a slowly changing value is rounded.  NaN/Inf as round-to-nearest.
__host__ __device__ __forceinline__ uint16_t f32_to_bf16_sr(float x, uint32_t rnd16) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return f32_to_bf16(x);
  return (uint16_t)((u + (rnd16 & 0xffffu)) >> 16);
}
__host__ __device__ __forceinline__ uint32_t pack_bf16x2_sr(float re, float im, uint32_t rnd) {
  return (uint32_t)f32_to_bf16_sr(re, rnd) | ((uint32_t)f32_to_bf16_sr(im, rnd >> 16) << 16);
}
__host__ __device__ __forceinline__ float2 unpack_bf16x2(uint32_t v) {
  return make_float2(bf16_to_f32((uint16_t)(v & 0xffffu)), bf16_to_f32((uint16_t)(v >> 16)));
}

// Unobserved entries of the packed observation tensor are quiet NaNs whose payload holds
// the position t of the entry inside its run of consecutive unobserved entries along
// mode 2 (bits 0..19) and whether that run starts at the first slot of the row (bit 20).
__host__ __device__ __forceinline__ uint32_t pack_unobserved(uint32_t t, uint32_t starts_row) {
  return 0x7fc00000u | (starts_row << 20) | (t & 0xfffffu);
}
__device__ __forceinline__ bool is_unobserved(float g) { return (__float_as_uint(g) & 0x7f800000u) == 0x7f800000u; }
__device__ __forceinline__ uint32_t unobs_pos(float g) { return __float_as_uint(g) & 0xfffffu; }
__device__ __forceinline__ uint32_t unobs_starts_row(float g) { return (__float_as_uint(g) >> 20) & 1u; }

// Weight of stored frequency b in a sum over all n3 frequencies (conjugate pairs).
__host__ __device__ __forceinline__ double bin_weight(int b, int n3) {
  return (b == 0 || (n3 % 2 == 0 && b == n3 / 2)) ? 1.0 : 2.0;
}
__host__ __device__ __forceinline__ bool bin_is_real(int b, int n3) {
  return b == 0 || (n3 % 2 == 0 && b == n3 / 2);
}

// Block-wide FP64 sum of one value per thread (blockDim.x <= 1024); all threads get it.
__device__ __forceinline__ double block_sum_d(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];   // fixed order
  __syncthreads();
  return s;
}
// Three block-wide FP64 sums at once (blockDim.x <= 1024; red holds >= 48 doubles).
__device__ __forceinline__ void block_sum3_d(double& a, double& b, double& c, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
    c += __shfl_xor(c, off);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    red[wid] = a;
    red[16 + wid] = b;
    red[32 + wid] = c;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int w = 0; w < nw; ++w) {   // fixed order
    sa += red[w];
    sb += red[16 + w];
    sc += red[32 + w];
  }
  a = sa;
  b = sb;
  c = sc;
}
__device__ __forceinline__ double block_max_d(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < nw; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// p[i] when ok, else z.  The load itself is unconditional (from p[0] when !ok, which must
// be a valid element) and only its value is selected: a load under a branch is waited for
// at the branch's end, so a batch of guarded loads would otherwise cost one memory latency
// per load instead of one for the batch.
template <typename T>
__device__ __forceinline__ T ld_or(const T* __restrict__ p, size_t i, bool ok, T z) {
  const T v = p[ok ? i : 0];
  return ok ? v : z;
}

// Block-cooperative copy of n elements, dst[e] = load(e) for e < n, in batches of PER
// elements per thread whose loads are all issued before any of their stores (a loop of
// load-then-store would wait out one memory latency per element).  Lanes past n load
// element n - 1 and drop it, so no load sits under a branch.
template <int PER, typename T, typename F>
__device__ __forceinline__ void stage_batched(T* dst, int n, F load) {
  const int nt = blockDim.x;
  for (int e0 = 0; e0 < n; e0 += PER * nt) {
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = e0 + threadIdx.x + u * nt;
      v[u] = load(e < n ? e : n - 1);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = e0 + threadIdx.x + u * nt;
      if (e < n) dst[e] = v[u];
    }
  }
}

// The same with a store functor: store(e, value) for e < n.
template <int PER, typename T, typename L, typename S>
__device__ __forceinline__ void stage_batched_to(int n, L load, S store) {
  const int nt = blockDim.x;
  for (int e0 = 0; e0 < n; e0 += PER * nt) {
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = e0 + threadIdx.x + u * nt;
      v[u] = load(e < n ? e : n - 1);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = e0 + threadIdx.x + u * nt;
      if (e < n) store(e, v[u]);
    }
  }
}

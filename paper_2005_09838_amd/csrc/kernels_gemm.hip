// The three batched complex slice products of one iteration (per stored frequency b):
//   Z~_b = X~_b Y~_b                       (step 3)                   k_zgemm
//   A_b  = W~_b Y~_b^*  and the X right-hand side                      k_agemm
//          R_b = eta A_b G_Y^+ + H_rho1 X~_b (I - eta P_Y)   (step 1, eq. (updataXYW1))
//   X~_b^* W~_b, X~_b^* X~_b, (H X~_b)^*(H X~_b) partial sums over row chunks (step 2)
//                                                                      k_bgemm
// FP32 mode: FP32 operands; the n1 reduction of X~^* W~ accumulates in FP64.
// Mixed mode: W~ is read from BF16 storage and X~, Y~ operands are rounded to BF16;
// products accumulate in FP32.  r x r Grams are always FP64.
#include "kernels.h"

namespace tctf {

__device__ __forceinline__ float2 ld_wt(const void* wt, size_t idx, int mixed) {
  return mixed ? unpack_bf16x2(((const uint32_t*)wt)[idx]) : ((const float2*)wt)[idx];
}
__device__ __forceinline__ cf to_cf(float2 v, int mixed) {
  cf c;
  c.re = mixed ? bf16_round(v.x) : v.x;
  c.im = mixed ? bf16_round(v.y) : v.y;
  return c;
}

// ---------------------------------------------------------------- Z~ = X~ Y~
// Tile: 16 rows (i) x 64 columns (j) of one frequency.
__global__ void __launch_bounds__(256) k_zgemm(const float2* __restrict__ xt, const float2* __restrict__ yt,
                                               float2* __restrict__ zt, int n1, int n2, int r, int nb, int mixed) {
  __shared__ cf xs[16][TCTF_RMAX];
  __shared__ cf ys[TCTF_RMAX][64];
  const int j0 = blockIdx.x * 64, i0 = blockIdx.y * 16, b = blockIdx.z, tid = threadIdx.x;
  for (int e = tid; e < r * 64; e += 256) {
    const int s = e >> 6, jj = e & 63, j = j0 + jj;
    ys[s][jj] = (j < n2) ? to_cf(yt[((size_t)b * r + s) * n2 + j], mixed) : cf{0.f, 0.f};
  }
  for (int e = tid; e < r * 16; e += 256) {
    const int s = e >> 4, il = e & 15, i = i0 + il;
    xs[il][s] = (i < n1) ? to_cf(xt[((size_t)b * r + s) * n1 + i], mixed) : cf{0.f, 0.f};
  }
  __syncthreads();
  const int jl = tid & 63, ig = tid >> 6, j = j0 + jl;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int il = ig + 4 * u, i = i0 + il;
    float ar = 0.f, ai = 0.f;
    for (int s = 0; s < r; ++s) {
      const cf x = xs[il][s], y = ys[s][jl];
      ar = fmaf(x.re, y.re, fmaf(-x.im, y.im, ar));
      ai = fmaf(x.re, y.im, fmaf(x.im, y.re, ai));
    }
    if (i < n1 && j < n2) zt[((size_t)i * nb + b) * n2 + j] = make_float2(ar, ai);
  }
}

void launch_zgemm(const Plan& p) {
  dim3 grid((p.n2 + 63) / 64, (p.n1 + 15) / 16, p.nb);
  k_zgemm<<<grid, 256, 0, p.stream>>>(p.xt, p.yt, p.zt, p.n1, p.n2, p.r, p.nb, p.mixed);
}

// ---------------------------------------------------------------- A = W~ Y~^*, X right-hand side
// Tile: 16 rows of one frequency; thread (il, jl) accumulates A(i, :) over columns
// j = jl (mod 16), then the 16 lanes of a row combine their sums.
__global__ void __launch_bounds__(256) k_agemm(const void* __restrict__ wt, const float2* __restrict__ yt,
                                               const float2* __restrict__ xt, const cd* __restrict__ gyp,
                                               const cd* __restrict__ qy, const int* __restrict__ qy_zero,
                                               const float* __restrict__ htab, float2* __restrict__ rhs,
                                               int n1, int n2, int r, int nb, double eta, double rho1, int mixed,
                                               int raw_a) {
  __shared__ cf ych[TCTF_RMAX][64];
  __shared__ cd gs[TCTF_RMAX * TCTF_RMAX];
  __shared__ cd qs[TCTF_RMAX * TCTF_RMAX];
  __shared__ cf xh[18][TCTF_RMAX];
  const int i0 = blockIdx.x * 16, b = blockIdx.y, tid = threadIdx.x;
  const int il = tid >> 4, jl = tid & 15, i = i0 + il;
  float acc_re[TCTF_RMAX], acc_im[TCTF_RMAX];
#pragma unroll
  for (int s = 0; s < TCTF_RMAX; ++s) { acc_re[s] = 0.f; acc_im[s] = 0.f; }
  for (int j0 = 0; j0 < n2; j0 += 64) {
    __syncthreads();
    for (int e = tid; e < r * 64; e += 256) {
      const int s = e >> 6, jj = e & 63, j = j0 + jj;
      ych[s][jj] = (j < n2) ? to_cf(yt[((size_t)b * r + s) * n2 + j], mixed) : cf{0.f, 0.f};
    }
    __syncthreads();
    if (i < n1) {
      for (int jj = jl; jj < 64 && j0 + jj < n2; jj += 16) {
        const float2 w = ld_wt(wt, ((size_t)i * nb + b) * n2 + j0 + jj, mixed);
#pragma unroll
        for (int s = 0; s < TCTF_RMAX; ++s) {
          if (s < r) {
            const cf y = ych[s][jj];   // w * conj(y)
            acc_re[s] = fmaf(w.x, y.re, fmaf(w.y, y.im, acc_re[s]));
            acc_im[s] = fmaf(w.y, y.re, fmaf(-w.x, y.im, acc_im[s]));
          }
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < TCTF_RMAX; ++s) {
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      acc_re[s] += __shfl_xor(acc_re[s], off);
      acc_im[s] += __shfl_xor(acc_im[s], off);
    }
  }
  const int noqy = qy_zero[b];
  for (int e = tid; e < r * r; e += 256) {
    gs[e] = gyp[(size_t)b * r * r + e];
    qs[e] = qy[(size_t)b * r * r + e];
  }
  for (int e = tid; e < r * 18; e += 256) {
    const int s = e / 18, hl = e % 18, ih = i0 - 1 + hl;
    const float2 v = (ih >= 0 && ih < n1) ? xt[((size_t)b * r + s) * n1 + ih] : make_float2(0.f, 0.f);
    xh[hl][s] = cf{v.x, v.y};
  }
  __syncthreads();
  if (i >= n1) return;
  const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
  const double dii = 1.0 + rho1 * deg;
  if (raw_a) {   // A itself (stationarity measures)
    for (int s = jl; s < r; s += 16) {
      float ar = 0.f, ai = 0.f;
#pragma unroll
      for (int q = 0; q < TCTF_RMAX; ++q)
        if (q == s) { ar = acc_re[q]; ai = acc_im[q]; }
      rhs[((size_t)b * r + s) * n1 + i] = make_float2(ar, ai);
    }
    return;
  }
  for (int s = jl; s < r; s += 16) {
    cd t = cd_make(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < TCTF_RMAX; ++q)
      if (q < r) cd_fma(t, cd_make(acc_re[q], acc_im[q]), gs[q * r + s]);
    t = cd_scale(t, eta);
    if (!noqy) {
      cd u[3];
      for (int h = 0; h < 3; ++h) {
        u[h] = cd_make(0.0, 0.0);
        for (int q = 0; q < r; ++q) cd_fma(u[h], cd_make(xh[il + h][q].re, xh[il + h][q].im), qs[q * r + s]);
      }
      // (H_rho1 U)_i = (1 + rho1 deg_i) U_i - rho1 (U_{i-1} + U_{i+1}); outside rows are 0
      t = cd_add(t, cd_sub(cd_scale(u[1], dii), cd_scale(cd_add(u[0], u[2]), rho1)));
    }
    rhs[((size_t)b * r + s) * n1 + i] = make_float2((float)t.re, (float)t.im);
  }
  (void)htab;
}

void launch_agemm(const Plan& p, int raw_a) {
  dim3 grid((p.n1 + 15) / 16, p.nb);
  k_agemm<<<grid, 256, 0, p.stream>>>(p.wt, p.yt, p.xt, p.gyp, p.qy, p.qy_zero, p.htab, p.rhs, p.n1, p.n2,
                                      p.r, p.nb, p.eta, p.rho1, p.mixed, raw_a);
}

// ---------------------------------------------------------------- X~^* W~ and Gram partials
// Block (j-tile, chunk c, frequency b): rows [c*chunk, min(n1, (c+1)*chunk)).
template <typename Acc>
__global__ void __launch_bounds__(256) k_bgemm(const void* __restrict__ wt, const float2* __restrict__ xt,
                                               float2* __restrict__ bpart, cd* __restrict__ spart,
                                               cd* __restrict__ dpart, int n1, int n2, int r, int nb,
                                               int nchunk, int chunk, int mixed) {
  extern __shared__ cf xc[];   // [chunk + 1][r]
  const int j0 = blockIdx.x * 64, c = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  const int i0 = c * chunk, i1 = min(n1, i0 + chunk);
  const int rows = i1 - i0 + ((i1 < n1) ? 1 : 0);
  for (int e = tid; e < rows * r; e += 256) {
    const int s = e / rows, h = e % rows;
    const float2 v = xt[((size_t)b * r + s) * n1 + i0 + h];
    xc[h * r + s] = cf{v.x, v.y};
  }
  __syncthreads();
  const int jl = tid & 63, sg = tid >> 6, j = j0 + jl;
  constexpr int U = TCTF_RMAX / 4;
  Acc are[U], aim[U];
#pragma unroll
  for (int u = 0; u < U; ++u) { are[u] = 0; aim[u] = 0; }
  if (j < n2) {
    for (int i = i0; i < i1; ++i) {
      const float2 w = ld_wt(wt, ((size_t)i * nb + b) * n2 + j, mixed);
      const Acc wr = w.x, wi = w.y;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int s = sg + 4 * u;
        if (s < r) {
          cf x = xc[(i - i0) * r + s];
          if (mixed) { x.re = bf16_round(x.re); x.im = bf16_round(x.im); }
          const Acc xr = x.re, xi = x.im;   // conj(x) * w
          are[u] = fma(xr, wr, fma(xi, wi, are[u]));
          aim[u] = fma(xr, wi, fma(-xi, wr, aim[u]));
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = sg + 4 * u;
      if (s < r) bpart[(((size_t)b * nchunk + c) * r + s) * n2 + j] = make_float2((float)are[u], (float)aim[u]);
    }
  }
  if (blockIdx.x == 0) {
    for (int e = tid; e < r * r; e += 256) {
      const int s = e / r, t = e % r;
      cd sacc = cd_make(0.0, 0.0), dacc = cd_make(0.0, 0.0);
      for (int i = i0; i < i1; ++i) {
        const cf xs = xc[(i - i0) * r + s], xtt = xc[(i - i0) * r + t];
        cd_fma(sacc, cd_make(xs.re, -xs.im), cd_make(xtt.re, xtt.im));
        if (i + 1 < n1) {
          const cf ys = xc[(i + 1 - i0) * r + s], yt2 = xc[(i + 1 - i0) * r + t];
          const cd ds = cd_make((double)ys.re - xs.re, (double)ys.im - xs.im);
          const cd dt = cd_make((double)yt2.re - xtt.re, (double)yt2.im - xtt.im);
          cd_fma(dacc, cd_conj(ds), dt);
        }
      }
      spart[(((size_t)b * nchunk + c) * r) * r + e] = sacc;
      dpart[(((size_t)b * nchunk + c) * r) * r + e] = dacc;
    }
  }
}

void launch_bgemm(const Plan& p) {
  dim3 grid((p.n2 + 63) / 64, p.nchunk, p.nb);
  const size_t lds = (size_t)(p.chunk + 1) * p.r * sizeof(cf);
  if (p.mixed)
    k_bgemm<float><<<grid, 256, lds, p.stream>>>(p.wt, p.xt, p.bpart, p.spart, p.dpart, p.n1, p.n2, p.r, p.nb,
                                                 p.nchunk, p.chunk, p.mixed);
  else
    k_bgemm<double><<<grid, 256, lds, p.stream>>>(p.wt, p.xt, p.bpart, p.spart, p.dpart, p.n1, p.n2, p.r,
                                                  p.nb, p.nchunk, p.chunk, p.mixed);
}

}  // namespace tctf

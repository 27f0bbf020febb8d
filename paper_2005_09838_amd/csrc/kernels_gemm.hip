// The three batched complex slice products of one iteration (per stored frequency b):
//   Z~_b = X~_b Y~_b                       (step 3)                   k_zgemm
//   A_b  = W~_b Y~_b^*  and the X right-hand side                      k_agemm
//          R_b = eta A_b G_Y^+ + H_rho1 X~_b (I - eta P_Y)   (step 1, eq. (updataXYW1))
//   X~_b^* W~_b, X~_b^* X~_b, (H X~_b)^*(H X~_b) partial sums over row chunks (step 2)
//                                                                      k_bgemm
// FP32 mode: FP32 operands; the n1 reduction of X~^* W~ accumulates in FP64.
// Mixed mode: W~ is read from BF16 storage (the factors stay FP32) and the products
// accumulate in FP32.  r x r Grams are always FP64.
#include "kernels.h"

namespace tctf {

__device__ __forceinline__ float2 ld_wt(const void* wt, size_t idx, int mixed) {
  return mixed ? unpack_bf16x2(((const uint32_t*)wt)[idx]) : ((const float2*)wt)[idx];
}
__device__ __forceinline__ cf to_cf(float2 v, int) {
  cf c;
  c.re = v.x;
  c.im = v.y;
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
// Block: 64 rows of one frequency.  W~ and Y~ are staged through LDS in chunks of 64
// columns (coalesced loads, all issued before use); thread (il, q) = (tid / 4, tid % 4)
// accumulates A(i, s) for s = q, q + 4, ... in FP32.  The epilogue forms, in FP64,
//   R(i, :) = eta A(i, :) G_Y^+ + (H_rho1 U)(i, :),  U = X~ (I - eta P_Y)
// (U only when I - eta P_Y is not exactly 0).
#define AG_ROWS 64
#define AG_COLS 64
__global__ void __launch_bounds__(256) k_agemm(const void* __restrict__ wt, const float2* __restrict__ yt,
                                               const float2* __restrict__ xt, const cd* __restrict__ gyp,
                                               const cd* __restrict__ qy, const int* __restrict__ qy_zero,
                                               float2* __restrict__ rhs, int n1, int n2, int r, int nb,
                                               double eta, double rho1, int mixed, int raw_a) {
  // 49.9 KB of LDS (three blocks per CU): the W~ and Y~ tiles; the epilogue reuses them
  // for A (16 KB), G_Y^+ (16 KB) and Q_Y (16 KB).
  __shared__ __align__(16) float2 smem[(AG_ROWS + TCTF_RMAX) * (AG_COLS + 1)];
  float2 (*wsh)[AG_COLS + 1] = reinterpret_cast<float2 (*)[AG_COLS + 1]>(smem);
  float2 (*ysh)[AG_COLS + 1] = reinterpret_cast<float2 (*)[AG_COLS + 1]>(smem + AG_ROWS * (AG_COLS + 1));
  const int i0 = blockIdx.x * AG_ROWS, b = blockIdx.y, tid = threadIdx.x;
  const int il = tid >> 2, q = tid & 3, i = i0 + il;
  constexpr int SP = TCTF_RMAX / 4;   // outputs per thread at most
  float accr[SP], acci[SP];
#pragma unroll
  for (int u = 0; u < SP; ++u) { accr[u] = 0.f; acci[u] = 0.f; }
  for (int j0 = 0; j0 < n2; j0 += AG_COLS) {
    const int nc = min(AG_COLS, n2 - j0);
    __syncthreads();
    {
      float2 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {   // 64 x 64 tile, 16 elements per thread
        const int e = tid + 256 * u, rr = e >> 6, cc = e & 63;
        const int ii = i0 + rr;
        v[u] = (ii < n1 && cc < nc) ? ld_wt(wt, ((size_t)ii * nb + b) * n2 + j0 + cc, mixed) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u;
        wsh[e >> 6][e & 63] = v[u];
      }
    }
    for (int e = tid; e < r * AG_COLS; e += 256) {
      const int s = e >> 6, cc = e & 63;
      ysh[s][cc] = cc < nc ? yt[((size_t)b * r + s) * n2 + j0 + cc] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 4
    for (int cc = 0; cc < AG_COLS; ++cc) {
      const float2 w = wsh[il][cc];
#pragma unroll
      for (int u = 0; u < SP; ++u) {
        const int s = q + 4 * u;
        if (s < r) {
          const float2 y = ysh[s][cc];   // w * conj(y)
          accr[u] = fmaf(w.x, y.x, fmaf(w.y, y.y, accr[u]));
          acci[u] = fmaf(w.y, y.x, fmaf(-w.x, y.y, acci[u]));
        }
      }
    }
  }
  // epilogue: A rows through LDS (reusing the W~ tile)
  __syncthreads();
  float2* ash = &wsh[0][0];   // [AG_ROWS][r]
#pragma unroll
  for (int u = 0; u < SP; ++u) {
    const int s = q + 4 * u;
    if (s < r) ash[il * r + s] = make_float2(accr[u], acci[u]);
  }
  if (raw_a) {
    __syncthreads();
    for (int e = tid; e < AG_ROWS * r; e += 256) {
      const int s = e / AG_ROWS, rr = e % AG_ROWS;
      if (i0 + rr < n1) rhs[((size_t)b * r + s) * n1 + i0 + rr] = ash[rr * r + s];
    }
    return;
  }
  const int noqy = qy_zero[b];
  cd* gs = reinterpret_cast<cd*>(smem + AG_ROWS * TCTF_RMAX);
  cd* qs = reinterpret_cast<cd*>(smem + AG_ROWS * (AG_COLS + 1));
  static_assert(AG_ROWS * TCTF_RMAX * 2 <= AG_ROWS * (AG_COLS + 1), "A and G_Y^+ fit the W~ tile");
  static_assert(TCTF_RMAX * TCTF_RMAX * 2 <= TCTF_RMAX * (AG_COLS + 1), "Q_Y fits the Y~ tile");
  for (int e = tid; e < r * r; e += 256) {
    gs[e] = gyp[(size_t)b * r * r + e];
    qs[e] = qy[(size_t)b * r * r + e];
  }
  __syncthreads();
  float2 res[SP];
  if (i < n1) {
    const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
    const double dii = 1.0 + rho1 * deg;
#pragma unroll
    for (int us = 0; us < SP; ++us) {
      const int s = q + 4 * us;
      if (s >= r) break;
      cd t = cd_make(0.0, 0.0);
      for (int u = 0; u < r; ++u) {
        const float2 av = ash[il * r + u];
        cd_fma(t, cd_make(av.x, av.y), gs[u * r + s]);
      }
      t = cd_scale(t, eta);
      if (!noqy) {
        cd uu[3];
        for (int h = 0; h < 3; ++h) {
          uu[h] = cd_make(0.0, 0.0);
          const int ih = i - 1 + h;
          if (ih < 0 || ih >= n1) continue;
          for (int v2 = 0; v2 < r; ++v2) {
            const float2 xv = xt[((size_t)b * r + v2) * n1 + ih];
            cd_fma(uu[h], cd_make(xv.x, xv.y), qs[v2 * r + s]);
          }
        }
        // (H_rho1 U)_i = (1 + rho1 deg_i) U_i - rho1 (U_{i-1} + U_{i+1}); outside rows are 0
        t = cd_add(t, cd_sub(cd_scale(uu[1], dii), cd_scale(cd_add(uu[0], uu[2]), rho1)));
      }
      res[us] = make_float2((float)t.re, (float)t.im);
    }
  }
  __syncthreads();   // every thread has read A; its rows now take the results
  if (i < n1) {
#pragma unroll
    for (int us = 0; us < SP; ++us) {
      const int s = q + 4 * us;
      if (s < r) ash[il * r + s] = res[us];
    }
  }
  __syncthreads();
  for (int e = tid; e < AG_ROWS * r; e += 256) {   // coalesced along i
    const int s = e / AG_ROWS, rr = e % AG_ROWS;
    if (i0 + rr < n1) rhs[((size_t)b * r + s) * n1 + i0 + rr] = ash[rr * r + s];
  }
}

void launch_agemm(const Plan& p, int raw_a) {
  dim3 grid((p.n1 + AG_ROWS - 1) / AG_ROWS, p.nb);
  k_agemm<<<grid, 256, 0, p.stream>>>(p.wt, p.yt, p.xt, p.gyp, p.qy, p.qy_zero, p.rhs, p.n1, p.n2, p.r, p.nb,
                                      p.eta, p.rho1, p.mixed, raw_a);
}

// ---------------------------------------------------------------- X~^* W~ and Gram partials
// Block (j-tile of 64, chunk c, frequency b): rows [c*chunk, min(n1, (c+1)*chunk)).  The
// X~ rows of the chunk sit in LDS; W~ is staged 16 rows at a time (coalesced loads).
template <typename Acc>
__global__ void __launch_bounds__(256) k_bgemm(const void* __restrict__ wt, const float2* __restrict__ xt,
                                               float2* __restrict__ bpart, cd* __restrict__ spart,
                                               cd* __restrict__ dpart, int n1, int n2, int r, int nb,
                                               int nchunk, int chunk, int mixed) {
  extern __shared__ cf xc[];   // [chunk + 1][r]
  __shared__ float2 wsh[16][64];
  const int j0 = blockIdx.x * 64, c = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  const int i0 = c * chunk, i1 = min(n1, i0 + chunk);
  const int rows = i1 - i0 + ((i1 < n1) ? 1 : 0);
  for (int e = tid; e < rows * r; e += 256) {
    const int s = e / rows, h = e % rows;
    const float2 v = xt[((size_t)b * r + s) * n1 + i0 + h];
    xc[h * r + s] = cf{v.x, v.y};
  }
  const int jl = tid & 63, sg = tid >> 6, j = j0 + jl;
  constexpr int U = TCTF_RMAX / 4;
  Acc are[U], aim[U];
#pragma unroll
  for (int u = 0; u < U; ++u) { are[u] = 0; aim[u] = 0; }
  for (int ib = i0; ib < i1; ib += 16) {
    const int nr = min(16, i1 - ib);
    __syncthreads();
    {
      float2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {   // 16 x 64 tile, 4 elements per thread
        const int e = tid + 256 * u, rr = e >> 6, cc = e & 63;
        v[u] = (rr < nr && j0 + cc < n2) ? ld_wt(wt, ((size_t)(ib + rr) * nb + b) * n2 + j0 + cc, mixed)
                                         : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u;
        wsh[e >> 6][e & 63] = v[u];
      }
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const float2 w = wsh[rr][jl];
      const Acc wr = w.x, wi = w.y;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int s = sg + 4 * u;
        if (s < r) {
          const cf x = xc[(ib + rr - i0) * r + s];
          const Acc xr = x.re, xi = x.im;   // conj(x) * w
          are[u] = fma(xr, wr, fma(xi, wi, are[u]));
          aim[u] = fma(xr, wi, fma(-xi, wr, aim[u]));
        }
      }
    }
  }
  if (j < n2) {
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

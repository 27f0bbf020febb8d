// The three batched complex slice products of one iteration (per stored frequency b):
//   Z~_b = X~_b Y~_b                       (step 3)                   k_zgemm
//   A_b  = W~_b Y~_b^*  and the X right-hand side                      k_agemm
//          R_b = eta A_b G_Y^+ + H_rho1 X~_b (I - eta P_Y)   (step 1, eq. (updataXYW1))
//   X~_b^* W~_b, X~_b^* X~_b, (H X~_b)^*(H X~_b) partial sums over row chunks (step 2)
//                                                                      k_bgemm
// The complex products run on the matrix cores as real FP32 products (16 x 16 x 4 tiles):
// a complex m x k by k x n product is an m x 2k by 2k x n' real one whose operands are the
// interleaved (re, im) storage itself, with the signs of the complex product placed in the
// operand that is built on the fly.  X~^* W~ is summed in FP64 over blocks of 16 rows;
// r x r Grams and the X right-hand side epilogue are FP64.  Mixed mode reads W~ from its
// BF16 storage and converts to FP32 before the product.
#include "kernels.h"
#include "pinv.h"

namespace tctf {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// D += A B on one 16 x 16 x 4 FP32 tile: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16], and holds D[4 (l / 16) + t][l % 16] in element t.
__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// The FP64 16 x 16 x 4 tile: operands as above; lane l holds D[l / 16 + 4 t][l % 16].
__device__ __forceinline__ v4d mfma4d(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Two consecutive complex entries of W~ (j, j + 1) as four floats; entries past the end read 0.
__device__ __forceinline__ float4 ld_wt2(const void* wt, size_t idx, int valid, int mixed) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (mixed) {
    const uint32_t* w = (const uint32_t*)wt + idx;
    if (valid > 0) { const float2 a = unpack_bf16x2(w[0]); v.x = a.x; v.y = a.y; }
    if (valid > 1) { const float2 a = unpack_bf16x2(w[1]); v.z = a.x; v.w = a.y; }
  } else {
    const float2* w = (const float2*)wt + idx;
    if (valid > 0) { const float2 a = w[0]; v.x = a.x; v.y = a.y; }
    if (valid > 1) { const float2 a = w[1]; v.z = a.x; v.w = a.y; }
  }
  return v;
}

// ---------------------------------------------------------------- Z~ = X~ Y~
// Real form: Z'[i][2j + c] = sum_kk X'[i][kk] Y'[kk][2j + c] with kk = 2s + d,
// X'[i][2s + d] = (re, im)_d X~(i, s) and Y' carrying the signs of the complex product:
// Y'[2s][2j] = Yr, Y'[2s+1][2j] = -Yi, Y'[2s][2j+1] = Yi, Y'[2s+1][2j+1] = Yr.
// Block: 64 rows x one frequency, 4 wavefronts of 16 rows; Y~ staged in LDS by column
// chunks of ZG_COLS; each wavefront sweeps its rows across the chunk in groups of 4
// 16-column tiles.  Output tiles go straight to the interleaved Z~ rows.
// The first npinv blocks instead form G_Y^+ and I - eta P_Y of frequency blockIdx.x for
// the next X-step (pinvy_block): independent work that runs beside the product.
#define ZG_ROWS 64
#define ZG_COLS 128
template <int RM>   // r <= RM: every loop below has a compile-time trip count
__global__ void __launch_bounds__(256) k_zgemm(const float2* __restrict__ xt, const float2* __restrict__ yt,
                                               float2* __restrict__ zt, int n1, int n2, int r, int nb,
                                               int npinv, const cd* __restrict__ gym, cd* __restrict__ gyp,
                                               cd* __restrict__ qy, int* __restrict__ qy_zero, double eta,
                                               int force_eigen) {
  extern __shared__ __align__(16) unsigned char zsm[];
  if ((int)blockIdx.x < npinv) {
    pinvy_block(blockIdx.x, gym, gyp, qy, qy_zero, r, eta, force_eigen, zsm);
    return;
  }
  float2* ysh = (float2*)zsm;   // [s][j] of the column chunk
  const int bid = blockIdx.x - npinv, ntile = (n1 + ZG_ROWS - 1) / ZG_ROWS;
  const int i0 = (bid % ntile) * ZG_ROWS, b = bid / ntile, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  constexpr int KS = RM / 2;   // K steps of 4 over 2r <= 2 RM
  constexpr int YPER = RM * ZG_COLS / 256;
  float2 yv[YPER];   // this thread's share of a Y~ column chunk, loaded ahead of its LDS store
  auto load_y = [&](int j0) {
    const int nc = min(ZG_COLS, n2 - j0);
#pragma unroll
    for (int u = 0; u < YPER; ++u) {
      const int e = tid + 256 * u, s = e / ZG_COLS, jj = e % ZG_COLS;
      yv[u] = (s < r && jj < nc) ? yt[((size_t)b * r + s) * n2 + j0 + jj] : make_float2(0.f, 0.f);
    }
  };
  load_y(0);
  // A operands for every K step: X'[row][4 ks + q] (0 past the ends; loads clamped in range)
  const int row = i0 + 16 * w + m;
  float a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int kk = 4 * ks + q, s = kk >> 1;
    const float2 x = xt[((size_t)b * r + min(s, r - 1)) * n1 + min(row, n1 - 1)];
    a[ks] = (s < r && row < n1) ? ((kk & 1) ? x.y : x.x) : 0.f;
  }
  // this lane's operand pick of Y': component and sign are fixed by (kk & 1, column & 1)
  const int d = q & 1, cpar = m & 1;
  const bool take_im = d != cpar;
  const float sgn = (d == 1 && cpar == 0) ? -1.f : 1.f;
  float* zf = (float*)zt;
  for (int j0 = 0; j0 < n2; j0 += ZG_COLS) {
    const int nc = min(ZG_COLS, n2 - j0);
    if (j0 > 0) {
      __syncthreads();   // every wavefront is done with the previous chunk
      load_y(j0);
    }
#pragma unroll
    for (int u = 0; u < YPER; ++u) ysh[tid + 256 * u] = yv[u];
    __syncthreads();
    const int ntiles = (2 * nc + 15) / 16;
    for (int nt0 = 0; nt0 < ntiles; nt0 += 4) {
      v4f acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int s = min((4 * ks + q) >> 1, r - 1);   // rows past 2r meet a zero A operand
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jj = min((16 * (nt0 + u) + m) >> 1, ZG_COLS - 1);
          const float2 y = ysh[s * ZG_COLS + jj];
          const float bv = sgn * (take_im ? y.y : y.x);
          acc[u] = mfma4(a[ks], bv, acc[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int col = 16 * (nt0 + u) + m;   // index into the chunk's 2 nc floats
        if (col < 2 * nc) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i = i0 + 16 * w + 4 * q + t;
            if (i < n1) zf[(((size_t)i * nb + b) * n2 + j0) * 2 + col] = acc[u][t];
          }
        }
      }
    }
  }
}

void zgemm_set_attr(int r) {
  if (pinvy_lds_bytes(r) > 65536)
    (void)hipFuncSetAttribute((const void*)k_zgemm<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pinvy_lds_bytes(r));
}

void launch_zgemm(const Plan& p, int with_pinv) {
  const int npinv = with_pinv ? p.nb : 0;
  const int grid = npinv + (p.n1 + ZG_ROWS - 1) / ZG_ROWS * p.nb;
  const int rm = p.r <= 8 ? 8 : (p.r <= 16 ? 16 : 32);
  size_t lds = (size_t)rm * ZG_COLS * sizeof(float2);
  if (with_pinv && pinvy_lds_bytes(p.r) > lds) lds = pinvy_lds_bytes(p.r);
#define TCTF_ZGEMM(RM)                                                                                   \
  k_zgemm<RM><<<grid, 256, lds, p.stream>>>(p.xt, p.yt, p.zt, p.n1, p.n2, p.r, p.nb, npinv, p.gym, p.gyp, \
                                           p.qy, p.qy_zero, p.eta, p.force_eigen)
  if (p.r <= 8) TCTF_ZGEMM(8);
  else if (p.r <= 16) TCTF_ZGEMM(16);
  else TCTF_ZGEMM(32);
#undef TCTF_ZGEMM
}

// ---------------------------------------------------------------- A = W~ Y~^*, X right-hand side
// Real form: A'[i][2s + e] = sum_kk W'[i][kk] Y'[kk][2s + e], kk = 2j + c, W' the
// interleaved W~ row and Y'[2j][2s] = Yr, Y'[2j+1][2s] = Yi, Y'[2j][2s+1] = -Yi,
// Y'[2j+1][2s+1] = Yr (Y = Y~(s, j)).  Within a group of 16 K values the K order is
// permuted so that lane (m, q) feeds the four products of the group from the four
// consecutive floats W'[m][16 g + 4 q ..] (two complex entries of W~), and the matching
// Y' values are the same two complex entries of Y~ row s (with the sign pattern).
// Block: 64 rows x one frequency, 4 wavefronts of 16 rows, up to AG_COLS columns of W~ per
// pass with every W~ load of the pass issued before the products.  The epilogue forms, in
// FP64, R(i, :) = eta A(i, :) G_Y^+ + (H_rho1 U)(i, :), U = X~ (I - eta P_Y) (U only when
// I - eta P_Y is not exactly 0).
#define AG_ROWS 64
#define AG_COLS 128
template <int RM>   // r <= RM
__global__ void __launch_bounds__(256) k_agemm(const void* __restrict__ wt, const float2* __restrict__ yt,
                                               const float2* __restrict__ xt, const cd* __restrict__ gyp,
                                               const cd* __restrict__ qy, const int* __restrict__ qy_zero,
                                               float2* __restrict__ rhs, int n1, int n2, int r, int nb,
                                               double eta, double rho1, int mixed, int raw_a) {
  __shared__ __align__(16) float2 ysh[TCTF_RMAX * AG_COLS];   // [s][j] of the column chunk (32 KB)
  __shared__ __align__(16) float2 ash[AG_ROWS * TCTF_RMAX];   // A rows, then the results (16 KB)
  __shared__ __align__(16) cd gs[TCTF_RMAX * TCTF_RMAX];      // G_Y^+ (16 KB)
  const int i0 = blockIdx.x * AG_ROWS, b = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int row = i0 + 16 * w + m;
  constexpr int NNT = RM / 8;          // 16-column tiles of A' (2 RM columns)
  constexpr int YPER = RM * AG_COLS / 256;
  const bool eodd = m & 1;             // this lane's output column 2s + e has e = 1
  v4f acc[NNT];
#pragma unroll
  for (int u = 0; u < NNT; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int j0 = 0; j0 < n2; j0 += AG_COLS) {
    const int nc = min(AG_COLS, n2 - j0), ngroups = (nc + 7) / 8;
    // W~ operands of this pass: group g covers columns j0 + 8 g .. + 7; this lane takes 2
    float4 wa[AG_COLS / 8];
#pragma unroll
    for (int g = 0; g < AG_COLS / 8; ++g) {
      const int jj = 8 * g + 2 * q;
      const int valid = (g < ngroups && row < n1) ? min(2, nc - jj) : 0;
      wa[g] = ld_wt2(wt, ((size_t)row * nb + b) * n2 + j0 + jj, valid, mixed);
    }
    // the Y~ column chunk, loaded while the W~ loads are in flight
    float2 yv[YPER];
#pragma unroll
    for (int u = 0; u < YPER; ++u) {
      const int e = tid + 256 * u, s = e / AG_COLS, jj = e % AG_COLS;
      yv[u] = (s < r && jj < nc) ? yt[((size_t)b * r + s) * n2 + j0 + jj] : make_float2(0.f, 0.f);
    }
    if (j0 > 0) __syncthreads();   // every wavefront is done with the previous chunk
#pragma unroll
    for (int u = 0; u < YPER; ++u) ysh[tid + 256 * u] = yv[u];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < AG_COLS / 8; ++g) {
      if (g < ngroups) {
#pragma unroll
        for (int u = 0; u < NNT; ++u) {
          const int s = min((16 * u + m) >> 1, r - 1);   // columns past 2r are dropped below
          const float4 y2 = *(const float4*)&ysh[s * AG_COLS + 8 * g + 2 * q];   // Y~(s, j), Y~(s, j + 1)
          // e = 0: (Yr, Yi, Yr', Yi');  e = 1: (-Yi, Yr, -Yi', Yr')
          const float b0 = eodd ? -y2.y : y2.x, b1 = eodd ? y2.x : y2.y;
          const float b2 = eodd ? -y2.w : y2.z, b3 = eodd ? y2.z : y2.w;
          acc[u] = mfma4(wa[g].x, b0, acc[u]);
          acc[u] = mfma4(wa[g].y, b1, acc[u]);
          acc[u] = mfma4(wa[g].z, b2, acc[u]);
          acc[u] = mfma4(wa[g].w, b3, acc[u]);
        }
      }
    }
  }
  // A tile to LDS: element t of tile u is A'[16 w + 4 q + t][16 u + m] = (re, im)_e A(i, s)
  float* af = (float*)ash;
#pragma unroll
  for (int u = 0; u < NNT; ++u) {
    const int col = 16 * u + m;
    if (col < 2 * r) {
#pragma unroll
      for (int t = 0; t < 4; ++t) af[(16 * w + 4 * q + t) * 2 * r + col] = acc[u][t];
    }
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
  cd* qs = (cd*)ysh;   // I - eta P_Y reuses the Y~ chunk (16 KB of its 32 KB)
  __syncthreads();     // every wavefront is done with the Y~ chunk
  for (int e = tid; e < r * r; e += 256) {
    gs[e] = gyp[(size_t)b * r * r + e];
    if (!noqy) qs[e] = qy[(size_t)b * r * r + e];
  }
  __syncthreads();
  // thread (il, qq) = (tid / 4, tid % 4) forms R(i0 + il, s) for s = qq, qq + 4, ...
  const int il = tid >> 2, qq = tid & 3, i = i0 + il;
  constexpr int SP = RM / 4;
  float2 res[SP];
  if (i < n1) {
    const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
    const double dii = 1.0 + rho1 * deg;
    // eta A(i, :) G_Y^+ for this thread's SP columns, one independent chain per column
    cd ag[SP];
#pragma unroll
    for (int us = 0; us < SP; ++us) ag[us] = cd_make(0.0, 0.0);
    for (int u = 0; u < r; ++u) {
      const float2 av = ash[il * r + u];
      const cd a = cd_make(av.x, av.y);
#pragma unroll
      for (int us = 0; us < SP; ++us) {
        const int s = min(qq + 4 * us, r - 1);   // columns past r are discarded below
        cd_fma(ag[us], a, gs[u * r + s]);
      }
    }
#pragma unroll
    for (int us = 0; us < SP; ++us) {
      const int s = qq + 4 * us;
      if (s >= r) break;
      cd t = cd_scale(ag[us], eta);
      if (!noqy) {
        // (H_rho1 U)_i = (1 + rho1 deg_i) U_i - rho1 (U_{i-1} + U_{i+1}); outside rows are 0
        cd um = cd_make(0.0, 0.0), u0 = cd_make(0.0, 0.0), up = cd_make(0.0, 0.0);
        for (int v2 = 0; v2 < r; ++v2) {
          const float2* xc = xt + ((size_t)b * r + v2) * n1;
          const cd qv = qs[v2 * r + s];
          const float2 x0 = xc[i];
          cd_fma(u0, cd_make(x0.x, x0.y), qv);
          if (i > 0) {
            const float2 x1 = xc[i - 1];
            cd_fma(um, cd_make(x1.x, x1.y), qv);
          }
          if (i + 1 < n1) {
            const float2 x2 = xc[i + 1];
            cd_fma(up, cd_make(x2.x, x2.y), qv);
          }
        }
        t = cd_add(t, cd_sub(cd_scale(u0, dii), cd_scale(cd_add(um, up), rho1)));
      }
      res[us] = make_float2((float)t.re, (float)t.im);
    }
  }
  __syncthreads();   // every thread has read A; its rows now take the results
  if (i < n1) {
#pragma unroll
    for (int us = 0; us < SP; ++us) {
      const int s = qq + 4 * us;
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
#define TCTF_AGEMM(RM)                                                                                     \
  k_agemm<RM><<<grid, 256, 0, p.stream>>>(p.wt, p.yt, p.xt, p.gyp, p.qy, p.qy_zero, p.rhs, p.n1, p.n2, p.r, \
                                          p.nb, p.eta, p.rho1, p.mixed, raw_a)
  if (p.r <= 8) TCTF_AGEMM(8);
  else if (p.r <= 16) TCTF_AGEMM(16);
  else TCTF_AGEMM(32);
#undef TCTF_AGEMM
}

// ---------------------------------------------------------------- X~^* W~ and Gram partials
// Real form: C'[2s + d][2j + c] = sum_i X'[2s + d][i] W'[i][2j + c] with X'[2s + d][i] =
// (re, im)_d X~(i, s) and W' the interleaved W~ rows; then
// (X~^* W~)(s, j) = (C'[2s][2j] + C'[2s+1][2j+1], C'[2s][2j+1] - C'[2s+1][2j]).
// Block: one chunk of at most 64 rows x one frequency.  The chunk's X~ rows (plus the
// next row, for H X~) and, per pass of BG_COLS columns, its whole W~ slab are staged in
// LDS with every load of a thread issued at once; each wavefront owns a quarter of the
// 16-column tiles of a pass.  After every 16 rows the FP32 tile sums are added into FP64
// accumulators.  The FP64 Gram partials of the chunk are formed from the staged X~ rows.
#define BG_COLS 64                  // complex columns per pass
#define BG_MAXROWS 64               // rows per chunk at most
#define BG_WLD (2 * BG_COLS + 16)   // LDS row stride of the staged W~ slab (floats)
template <int RM>   // r <= RM
__global__ void __launch_bounds__(256) k_bgemm(const void* __restrict__ wt, const float2* __restrict__ xt,
                                               float2* __restrict__ bpart, cd* __restrict__ spart,
                                               cd* __restrict__ dpart, int n1, int n2, int r, int nb,
                                               int nchunk, int chunk, int mixed) {
  extern __shared__ __align__(16) float smb[];
  const int xld = 2 * r + 16;                    // LDS row stride of the staged X~ rows (floats)
  float* xs = smb;                               // [chunk + 1][xld]: (re, im) of X~(i, s) at 2 s
  float* ws = smb + (size_t)(chunk + 1) * xld;   // [chunk rounded up to 4][BG_WLD]
  const int c = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int i0 = c * chunk, i1 = min(n1, i0 + chunk), nrows = i1 - i0;
  const int rows = nrows + ((i1 < n1) ? 1 : 0);
  const int nks = (nrows + 3) / 4;   // K steps of 4 rows
  // W~ slab of one pass: rows i0 .. i1 - 1 (zeros up to a multiple of 4), columns
  // j0 .. j0 + nc - 1; 16 elements per thread, loaded into registers ahead of their use
  constexpr int SLAB_PER = BG_MAXROWS * BG_COLS / 256;
  float2 slab[SLAB_PER];
  auto load_slab = [&](int j0) {
    const int nc = min(BG_COLS, n2 - j0);
#pragma unroll
    for (int u = 0; u < SLAB_PER; ++u) {
      const int e = tid + 256 * u, rr = e / BG_COLS, jj = e % BG_COLS;
      slab[u] = make_float2(0.f, 0.f);
      if (rr < nrows && jj < nc) {
        const size_t idx = ((size_t)(i0 + rr) * nb + b) * n2 + j0 + jj;
        slab[u] = mixed ? unpack_bf16x2(((const uint32_t*)wt)[idx]) : ((const float2*)wt)[idx];
      }
    }
  };
  load_slab(0);
  stage_batched_to<8, float2>(rows * r, [&](int e) {
    const int s = e / rows, h = e % rows;
    return xt[((size_t)b * r + s) * n1 + i0 + h];
  }, [&](int e, float2 v) {
    const int s = e / rows, h = e % rows;
    xs[h * xld + 2 * s] = v.x;
    xs[h * xld + 2 * s + 1] = v.y;
  });
  constexpr int MT = RM / 8;               // 16-row tiles of X' (2 RM rows)
  for (int j0 = 0; j0 < n2; j0 += BG_COLS) {
    const int nc = min(BG_COLS, n2 - j0);
    const int ntiles = (2 * nc + 15) / 16;   // at most 8; wavefront w takes tiles w and w + 4
    __syncthreads();   // the previous pass is done with the slab in LDS
#pragma unroll
    for (int u = 0; u < SLAB_PER; ++u) {
      const int e = tid + 256 * u, rr = e / BG_COLS, jj = e % BG_COLS;
      if (rr < 4 * nks) *(float2*)&ws[rr * BG_WLD + 2 * jj] = slab[u];
    }
    __syncthreads();
    if (j0 + BG_COLS < n2) load_slab(j0 + BG_COLS);   // the next pass's slab, in flight meanwhile
    double dacc[MT][2][4];   // [M tile][own N tile][t]
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) dacc[a][u][t] = 0.0;
    for (int kb = 0; kb < nks; kb += 4) {   // 16 rows per FP32 partial sum
      v4f acc[MT][2];
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[a][u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        const int ks = kb + k4;
        if (ks < nks) {
          const int kr = 4 * ks + q;   // chunk row of this lane's K index
          float av[MT];
#pragma unroll
          for (int a = 0; a < MT; ++a) {
            const int sp = 16 * a + m;   // row 2 s + d of X'
            av[a] = (sp < 2 * r && kr < nrows) ? xs[kr * xld + sp] : 0.f;
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int nt = w + 4 * u;
            if (nt < ntiles) {
              const float bv = ws[kr * BG_WLD + 16 * nt + m];
#pragma unroll
              for (int a = 0; a < MT; ++a) acc[a][u] = mfma4(av[a], bv, acc[a][u]);
            }
          }
        }
      }
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t) dacc[a][u][t] += (double)acc[a][u][t];
    }
    // combine C' into (X~^* W~)(s, j): lanes m and m ^ 1 hold columns 2 j and 2 j + 1
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int nt = w + 4 * u;
          if (nt < ntiles) {
            const int col = 16 * nt + m, j = col >> 1;
#pragma unroll
            for (int tp = 0; tp < 2; ++tp) {
              // rows 2 s (t = 2 tp) and 2 s + 1 (t = 2 tp + 1) of the tile
              const double own = dacc[a][u][2 * tp];
              const double other = __shfl_xor(dacc[a][u][2 * tp + 1], 1);
              const int s = (16 * a + 4 * q + 2 * tp) >> 1;
              const double v = (m & 1) ? own - other : own + other;   // odd lane: imaginary part
              if (s < r && j < nc)
                ((float*)bpart)[((((size_t)b * nchunk + c) * r + s) * n2 + j0 + j) * 2 + (m & 1)] = (float)v;
            }
          }
        }
      }
    }
  }
  // Gram partials of the chunk in FP64 on the matrix cores: C = X'^T X' and the same for the
  // row differences X'(i + 1) - X'(i) (rows whose successor exists), 2r x 2r real tiles of
  // 16 x 16 over K = the chunk's rows; then X~^* X~ (s, t) = (C[2s][2t] + C[2s+1][2t+1],
  // C[2s][2t+1] - C[2s+1][2t]) and the same for (H X~)^*(H X~).
  __syncthreads();   // the W~ slab area is free: the tiles go there
  double* cs = (double*)ws;                 // [2 RM][2 RM]
  double* cdm = cs + 4 * RM * RM;           // [2 RM][2 RM]
  for (int tile = w; tile < MT * MT; tile += 4) {
    const int ta = tile / MT, tb = tile % MT;
    v4d accs = v4d{0.0, 0.0, 0.0, 0.0}, accd = v4d{0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < nks; ++ks) {
      const int kr = 4 * ks + q;              // chunk row of this lane's K index
      const bool in = kr < nrows, hasnext = in && i0 + kr + 1 < n1;
      const int ca = 16 * ta + m, cb = 16 * tb + m;   // columns 2 s + d of X'
      const bool va = ca < 2 * r, vb = cb < 2 * r;
      const float* x0 = xs + (size_t)kr * xld;
      const double a0 = (in && va) ? (double)x0[ca] : 0.0, b0 = (in && vb) ? (double)x0[cb] : 0.0;
      const double a1 = (hasnext && va) ? (double)x0[xld + ca] - a0 : 0.0;
      const double b1 = (hasnext && vb) ? (double)x0[xld + cb] - b0 : 0.0;
      accs = mfma4d(a0, b0, accs);
      accd = mfma4d(a1, b1, accd);
    }
    // element t of the FP64 tile is row 16 ta + q + 4 t, column 16 tb + m
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rw = 16 * ta + q + 4 * t, cl = 16 * tb + m;
      cs[rw * 2 * RM + cl] = accs[t];
      cdm[rw * 2 * RM + cl] = accd[t];
    }
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += 256) {
    const int s = e / r, t = e % r;
    const int r0 = 2 * s * 2 * RM, r1 = (2 * s + 1) * 2 * RM;
    spart[(((size_t)b * nchunk + c) * r) * r + e] =
        cd_make(cs[r0 + 2 * t] + cs[r1 + 2 * t + 1], cs[r0 + 2 * t + 1] - cs[r1 + 2 * t]);
    dpart[(((size_t)b * nchunk + c) * r) * r + e] =
        cd_make(cdm[r0 + 2 * t] + cdm[r1 + 2 * t + 1], cdm[r0 + 2 * t + 1] - cdm[r1 + 2 * t]);
  }
}

size_t bgemm_lds_bytes(int r, int chunk) {
  const int rm = r <= 8 ? 8 : (r <= 16 ? 16 : 32);
  const size_t slab = (size_t)((chunk + 3) / 4 * 4) * BG_WLD * sizeof(float);
  const size_t tiles = 2 * (size_t)(2 * rm) * (2 * rm) * sizeof(double);   // the FP64 Gram tiles
  return (size_t)(chunk + 1) * (2 * r + 16) * sizeof(float) + (slab > tiles ? slab : tiles);
}

void bgemm_set_attr(size_t lds) {
  if (lds > 65536) {
    (void)hipFuncSetAttribute((const void*)k_bgemm<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_bgemm<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_bgemm<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
}

void launch_bgemm(const Plan& p) {
  dim3 grid(p.nchunk, p.nb);
  const size_t lds = bgemm_lds_bytes(p.r, p.chunk);
#define TCTF_BGEMM(RM)                                                                                      \
  k_bgemm<RM><<<grid, 256, lds, p.stream>>>(p.wt, p.xt, p.bpart, p.spart, p.dpart, p.n1, p.n2, p.r, p.nb, \
                                            p.nchunk, p.chunk, p.mixed)
  if (p.r <= 8) TCTF_BGEMM(8);
  else if (p.r <= 16) TCTF_BGEMM(16);
  else TCTF_BGEMM(32);
#undef TCTF_BGEMM
}

}  // namespace tctf

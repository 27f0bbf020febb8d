// The three batched complex slice products of one iteration (per stored frequency b):
//   Z~_b = X~_b Y~_b                       (step 3)                   k_zgemm
//   A_b  = W~_b Y~_b^*  and the X right-hand side                      k_agemm
//          R_b = eta A_b G_Y^+ + H_rho1 X~_b (I - eta P_Y)   (step 1, eq. (updataXYW1))
//   X~_b^* W~_b partial sums over row chunks (step 2), and in extra blocks of the same
//   launch G_X = X~_b^* X~_b + rho1 (H X~_b)^*(H X~_b), G_X^+ and I - eta P_X  k_bgemm
// The complex products run on the matrix cores as real FP32 products (16 x 16 x 4 tiles):
// a complex m x k by k x n product is an m x 2k by 2k x n' real one whose operands are the
// interleaved (re, im) storage itself, with the signs of the complex product placed in the
// operand that is built on the fly.  X~^* W~ runs on the FP64 matrix cores (FP64 partial
// sums over row chunks); r x r Grams and the X right-hand side epilogue are FP64.  Mixed mode reads W~ from its
// BF16 storage (stochastically rounded by the slice kernel) and converts to FP32 before
// the product.
#include <type_traits>
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
                                               int npinv, PinvyArgs pa) {
  extern __shared__ __align__(16) unsigned char zsm[];
  if ((int)blockIdx.x < npinv) {
    pinvy_block(blockIdx.x, pa, zsm);
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
      yv[u] = ld_or(yt, ((size_t)b * r + s) * n2 + j0 + jj, s < r && jj < nc, make_float2(0.f, 0.f));
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
  // Tile u of a group of four covers the group's 64 output floats 4 m + u (lane m's B
  // column), so a lane ends with four consecutive floats of a row: one 16-byte store.  The
  // operand pick of Y' is fixed by (kk & 1, column & 1) = (q & 1, u & 1).
  const int d = q & 1;
  float* zf = (float*)zt;
  const bool vec4 = (n2 & 1) == 0;   // rows start 16-byte aligned
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
          const int cpar = u & 1;
          const int jj = min(8 * nt0 + 2 * m + (u >> 1), ZG_COLS - 1);
          const float2 y = ysh[s * ZG_COLS + jj];
          const float bv = (d == 1 && cpar == 0) ? -y.y : (d != cpar ? y.y : y.x);
          acc[u] = mfma4(a[ks], bv, acc[u]);
        }
      }
      const int col = 16 * nt0 + 4 * m;   // first of this lane's four floats in the chunk's 2 nc
      if (col < 2 * nc) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = i0 + 16 * w + 4 * q + t;
          if (i < n1) {
            float* dst = zf + (((size_t)i * nb + b) * n2 + j0) * 2 + col;
            if (col + 4 <= 2 * nc) {
              if (vec4) {
                *(float4*)dst = make_float4(acc[0][t], acc[1][t], acc[2][t], acc[3][t]);
              } else {
                ((float2*)dst)[0] = make_float2(acc[0][t], acc[1][t]);
                ((float2*)dst)[1] = make_float2(acc[2][t], acc[3][t]);
              }
            } else {   // 2 nc is even: the last two floats of the row
              *(float2*)dst = make_float2(acc[0][t], acc[1][t]);
            }
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
  const PinvyArgs pa = pinvy_args(p);
#define TCTF_ZGEMM(RM) \
  k_zgemm<RM><<<grid, 256, lds, p.stream>>>(p.xt, p.yt, p.zt, p.n1, p.n2, p.r, p.nb, npinv, pa)
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
template <int RM, bool MIXED>   // r <= RM; MIXED: W~ stored as packed bf16 pairs
__global__ void __launch_bounds__(256) k_agemm(const void* wt, const float2* __restrict__ yt,
                                               const float2* __restrict__ xt, const cd* __restrict__ gyp,
                                               const cd* __restrict__ qy, const int* __restrict__ qy_zero,
                                               float2* __restrict__ rhs, int n1, int n2, int r, int nb,
                                               double eta, double rho1, int raw_a, uint32_t* ctr) {
  __shared__ __align__(16) float2 ysh[RM * AG_COLS];   // [s][j] of the column chunk
  __shared__ __align__(16) float2 ash[AG_ROWS * RM];   // A rows, then the results
  __shared__ __align__(16) cd gs[RM * RM];             // G_Y^+
  const int i0 = blockIdx.x * AG_ROWS, b = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int row = i0 + 16 * w + m;
  // one thread of the launch advances the counter of the rounding bits that this
  // iteration's slice kernel (a later launch) uses for the BF16 W~
  if (ctr && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) ctr[0] += 1u;
  constexpr int NNT = RM / 8;          // 16-column tiles of A' (2 RM columns)
  constexpr int YPER = RM * AG_COLS / 256;
  const bool eodd = m & 1;             // this lane's output column 2s + e has e = 1
  v4f acc[NNT];
#pragma unroll
  for (int u = 0; u < NNT; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
  // One pass per AG_COLS columns.  The Y~ chunk is loaded first (its LDS stage must not wait
  // for the W~ loads, the memory counter being in order), then every W~ load of the pass,
  // unconditional from one base (row clamped into range, immediate offsets; the W~ buffer
  // has AG_COLS elements of slack past its end) and kept raw: masks and conversions are
  // applied at the products, so that the products of group g wait only for its own loads.
  for (int j0 = 0; j0 < n2; j0 += AG_COLS) {
    using raw_t = typename std::conditional<MIXED, uint32_t, float2>::type;
    const int nc = min(AG_COLS, n2 - j0), ngroups = (nc + 7) / 8;
    float2 yv[YPER];
#pragma unroll
    for (int u = 0; u < YPER; ++u) {
      const int e = tid + 256 * u, s = e / AG_COLS, jj = e % AG_COLS;
      yv[u] = yt[((size_t)b * r + min(s, r - 1)) * n2 + j0 + min(jj, nc - 1)];
    }
    // group g covers columns j0 + 8 g .. + 7; this lane takes 2 (groups past the last valid
    // one load the last one again: no extra memory traffic, the values are dropped)
    raw_t lo[AG_COLS / 8], hi[AG_COLS / 8];
    const raw_t* wrow = (const raw_t*)wt + ((size_t)min(row, n1 - 1) * nb + b) * n2 + j0 + 2 * q;
#pragma unroll
    for (int g = 0; g < AG_COLS / 8; ++g) {
      const int gc = min(g, ngroups - 1);
      lo[g] = wrow[8 * gc];
      hi[g] = wrow[8 * gc + 1];
    }
    if (j0 > 0) __syncthreads();   // every wavefront is done with the previous chunk
#pragma unroll
    for (int u = 0; u < YPER; ++u) {
      const int e = tid + 256 * u, s = e / AG_COLS, jj = e % AG_COLS;
      ysh[e] = (s < r && jj < nc) ? yv[u] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < AG_COLS / 8; ++g) {
      if (g < ngroups) {
        const int valid = row < n1 ? min(2, nc - (8 * g + 2 * q)) : 0;
        float2 a0, a1;
        if constexpr (MIXED) {
          a0 = unpack_bf16x2(lo[g]);
          a1 = unpack_bf16x2(hi[g]);
        } else {
          a0 = lo[g];
          a1 = hi[g];
        }
        const float2 z = make_float2(0.f, 0.f);
        const float4 wa = make_float4(valid > 0 ? a0.x : z.x, valid > 0 ? a0.y : z.y, valid > 1 ? a1.x : z.x,
                                      valid > 1 ? a1.y : z.y);
#pragma unroll
        for (int u = 0; u < NNT; ++u) {
          const int s = min((16 * u + m) >> 1, r - 1);   // columns past 2r are dropped below
          const float4 y2 = *(const float4*)&ysh[s * AG_COLS + 8 * g + 2 * q];   // Y~(s, j), Y~(s, j + 1)
          // e = 0: (Yr, Yi, Yr', Yi');  e = 1: (-Yi, Yr, -Yi', Yr')
          const float b0 = eodd ? -y2.y : y2.x, b1 = eodd ? y2.x : y2.y;
          const float b2 = eodd ? -y2.w : y2.z, b3 = eodd ? y2.z : y2.w;
          acc[u] = mfma4(wa.x, b0, acc[u]);
          acc[u] = mfma4(wa.y, b1, acc[u]);
          acc[u] = mfma4(wa.z, b2, acc[u]);
          acc[u] = mfma4(wa.w, b3, acc[u]);
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
          const float2 z = make_float2(0.f, 0.f);
          const float2 x0 = xc[i], x1 = ld_or(xc, i - 1, i > 0, z), x2 = ld_or(xc, i + 1, i + 1 < n1, z);
          cd_fma(u0, cd_make(x0.x, x0.y), qv);
          cd_fma(um, cd_make(x1.x, x1.y), qv);
          cd_fma(up, cd_make(x2.x, x2.y), qv);
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

void launch_agemm(const Plan& p, int raw_a, int advance) {
  dim3 grid((p.n1 + AG_ROWS - 1) / AG_ROWS, p.nb);
#define TCTF_AGEMM(RM, MX)                                                                                    \
  k_agemm<RM, MX><<<grid, 256, 0, p.stream>>>(p.wt, p.yt, p.xt, p.gyp, p.qy, p.qy_zero, p.rhs, p.n1, p.n2, p.r, \
                                              p.nb, p.eta, p.rho1, raw_a, advance ? p.ctr : nullptr)
  if (p.mixed) {
    if (p.r <= 8) TCTF_AGEMM(8, true);
    else if (p.r <= 16) TCTF_AGEMM(16, true);
    else TCTF_AGEMM(32, true);
  } else {
    if (p.r <= 8) TCTF_AGEMM(8, false);
    else if (p.r <= 16) TCTF_AGEMM(16, false);
    else TCTF_AGEMM(32, false);
  }
#undef TCTF_AGEMM
}

// Outputs of gramx_block, per frequency b ([nb][r][r] FP64 complex unless noted).
struct GramOut {
  cd* gxm;       // G_X
  cd* dmat;      // (H X~)^*(H X~)
  cd* gxp;       // G_X^+
  cd* qx;        // I - eta G_X^+ G_X (not written when it is exactly 0)
  int* qx_zero;  // [nb] 1 when I - eta P_X = 0
  double rho1, eta;
  int force_eigen;
};

// Rows per staged group of gramx_block (plus the next row): 256, and 64 at r > 16 where the
// two sweeps need the partials beside the staging area.
#define GX_ROWS(RM) ((RM) <= 16 ? 256 : 64)

// LDS bytes of gramx_block at rank r <= RM: the staged rows and the complex Gram partials,
// later G_X with the pseudo-inverse scratch.
static inline size_t gramx_lds_bytes(int r, int rm) {
  const int ks = rm == 8 ? 4 : 1;
  const size_t sb = (size_t)2 * rm * (GX_ROWS(rm) + 4) * sizeof(float);
  const size_t pb = (size_t)ks * 2 * r * r * sizeof(cd);
  const size_t a = rm <= 16 ? (sb > pb ? sb : pb) : sb + pb;
  return a > pinvy_lds_bytes(r) ? a : pinvy_lds_bytes(r);
}

// Frequency b, by a whole block: the FP64 Grams C = X'^T X' and the same for the row
// differences X'(i + 1) - X'(i) over all n1 rows, as 16 x 16 x 4 FP64 matrix-core tiles.
// Rows arrive in groups of GR (plus the next row), staged column by column (X'^T; columns
// past 2r and rows past n1 zero), the next group's loads in flight while the current one is
// multiplied.  Within 16 rows the K order is permuted: lane (m, q) feeds rows 4 q .. 4 q + 3
// of the 16, so one 16-byte LDS read (and one float of the following row) serves four
// steps.  Full groups need no masks; the last group masks the difference at the last row.
// At r <= 8 the four wavefronts share the one tile and split the rows; at r > 16 each
// wavefront takes its four tiles in two sweeps over the rows.  The lanes holding C[2s][2t]
// gather the 2 x 2 real block by shuffles and form X~^* X~ (s, t) = (C[2s][2t] +
// C[2s+1][2t+1], C[2s][2t+1] - C[2s+1][2t]), likewise (H X~)^*(H X~); then
// G_X = X~^* X~ + rho1 (H X~)^*(H X~), its pseudo-inverse (Lemma SVPMPI, pinv_herm) and
// I - eta P_X.
template <int RM>
__device__ inline void gramx_block(int b, const float2* __restrict__ xt, int n1, int r, const GramOut& go,
                                   unsigned char* sm) {
  constexpr int MT = RM / 8, NT = MT * MT;         // 16 x 16 tiles of the real Gram
  constexpr int KS = NT >= 4 ? 1 : 4 / NT;         // wavefronts sharing a tile (row split)
  constexpr int TPW = NT >= 4 ? NT / 4 : 1;        // tiles per wavefront
  constexpr int TPS = TPW < 2 ? TPW : 2;           // tiles per sweep over the rows
  constexpr int NSW = TPW / TPS;                   // sweeps
  constexpr int GR = GX_ROWS(RM);                  // rows per group
  constexpr int LD = GR + 4;                       // LDS stride of a staged column (floats)
  constexpr int PER = ((GR + 1) * RM + 255) / 256; // staged elements per thread (GR + 1 rows)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int rr = r * r, kp = KS > 1 ? w : 0;
  float* xs = (float*)sm;   // [2 RM][LD]: X'^T, column 2 s + d of X' is row 2 s + d here
  // [KS][2][rr]: after the staging area, or in it when one sweep leaves it free
  cd* part = (cd*)(sm + (NSW > 1 ? (size_t)2 * RM * LD * sizeof(float) : 0));
  // element e of a group: column s = e / (GR + 1), row h = e % (GR + 1); past the matrix: zeros
  float2 pf[PER];
  auto load_group = [&](int i0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, s = e / (GR + 1), h = e % (GR + 1);
      pf[u] = ld_or(xt, ((size_t)b * r + s) * n1 + i0 + h, s < r && i0 + h < n1, make_float2(0.f, 0.f));
    }
  };
  load_group(0);
#pragma unroll
  for (int sw = 0; sw < NSW; ++sw) {
    v4d acs[TPS], acd[TPS];
#pragma unroll
    for (int u = 0; u < TPS; ++u) {
      acs[u] = v4d{0.0, 0.0, 0.0, 0.0};
      acd[u] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    for (int i0 = 0; i0 < n1; i0 += GR) {
      const int nrows = min(GR, n1 - i0);
      __syncthreads();   // the previous rows are consumed
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = tid + 256 * u, s = e / (GR + 1), h = e % (GR + 1);
        if (s < RM) {
          xs[(2 * s) * LD + h] = pf[u].x;
          xs[(2 * s + 1) * LD + h] = pf[u].y;
        }
      }
      __syncthreads();
      if (i0 + GR < n1) load_group(i0 + GR);
      else if (sw + 1 < NSW) load_group(0);
      const bool full = i0 + GR < n1;   // GR rows and the next one: no masks
#pragma unroll
      for (int u = 0; u < TPS; ++u) {
        const int tile = KS > 1 ? 0 : w + 4 * (sw * TPS + u);
        const float* pa = xs + (16 * (tile / MT) + m) * LD;   // column 2 s + d of X'
        const float* pb = xs + (16 * (tile % MT) + m) * LD;
        auto step16 = [&](int jb, auto masked) {
          const int h0 = 16 * jb + 4 * q;
          const float4 a4 = *(const float4*)(pa + h0), b4 = *(const float4*)(pb + h0);
          const double av[5] = {a4.x, a4.y, a4.z, a4.w, pa[h0 + 4]};
          const double bv[5] = {b4.x, b4.y, b4.z, b4.w, pb[h0 + 4]};
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            double a1 = av[jj + 1] - av[jj], b1 = bv[jj + 1] - bv[jj];
            if constexpr (decltype(masked)::value) {   // no difference at the last row
              if (i0 + h0 + jj + 1 >= n1) a1 = b1 = 0.0;
            }
            acs[u] = mfma4d(av[jj], bv[jj], acs[u]);
            acd[u] = mfma4d(a1, b1, acd[u]);
          }
        };
        if (full) {
#pragma unroll 2
          for (int jb = kp; jb < GR / 16; jb += KS) step16(jb, std::false_type{});
        } else {
          for (int jb = kp; 16 * jb < nrows; jb += KS) step16(jb, std::true_type{});
        }
      }
    }
    if (NSW == 1) __syncthreads();   // the partials take the staging area
    // element t of a lane: real row 16 ta + q + 4 t, column 16 tb + m; the lanes with q and m
    // even hold C[2s][2t] and read C[2s][2t+1], C[2s+1][2t], C[2s+1][2t+1] from lanes + 1,
    // + 16 and + 17
#pragma unroll
    for (int u = 0; u < TPS; ++u) {
      const int tile = KS > 1 ? 0 : w + 4 * (sw * TPS + u), ta = tile / MT, tb = tile % MT;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double s0 = acs[u][t], s1 = __shfl_down(s0, 1), s16 = __shfl_down(s0, 16),
                     s17 = __shfl_down(s0, 17);
        const double d0 = acd[u][t], d1 = __shfl_down(d0, 1), d16 = __shfl_down(d0, 16),
                     d17 = __shfl_down(d0, 17);
        const int sr = (16 * ta + q + 4 * t) >> 1, sc = (16 * tb + m) >> 1;
        if (!(q & 1) && !(m & 1) && sr < r && sc < r) {
          part[(2 * kp) * rr + sr * r + sc] = cd_make(s0 + s17, s1 - s16);
          part[(2 * kp + 1) * rr + sr * r + sc] = cd_make(d0 + d17, d1 - d16);
        }
      }
    }
  }
  __syncthreads();
  constexpr int GPT = (RM * RM + 255) / 256;   // G_X entries per thread
  cd gv[GPT];
#pragma unroll
  for (int k = 0; k < GPT; ++k) {
    const int e = tid + 256 * k;
    gv[k] = cd_make(0.0, 0.0);
    if (e < rr) {
      cd sv = part[e], dv = part[rr + e];
#pragma unroll
      for (int j = 1; j < KS; ++j) {   // the row parts, in a fixed order
        sv = cd_add(sv, part[2 * j * rr + e]);
        dv = cd_add(dv, part[(2 * j + 1) * rr + e]);
      }
      gv[k] = cd_add(sv, cd_scale(dv, go.rho1));
      go.gxm[(size_t)b * rr + e] = gv[k];
      go.dmat[(size_t)b * rr + e] = dv;
    }
  }
  __syncthreads();   // the partials are read; G_X and the pinv scratch take their place
  cd* gx = (cd*)sm;
  cd* gp = gx + rr;
  PinvScratch ps;
  ps.work = gp + rr;
  ps.vec = ps.work + rr;
  ps.colk = ps.vec + rr;
  ps.rowk = ps.colk + r;
  ps.rot = (double*)(ps.rowk + r);
  ps.red = ps.rot + 96;
#pragma unroll
  for (int k = 0; k < GPT; ++k) {
    const int e = tid + 256 * k;
    if (e < rr) gx[e] = gv[k];
  }
  __syncthreads();
  const int fullr = pinv_herm(gx, gp, r, go.force_eigen, ps);
  const bool qzero = fullr && go.eta == 1.0;
  for (int e = tid; e < rr; e += 256) {
    go.gxp[(size_t)b * rr + e] = gp[e];
    if (!qzero) {   // q = I - eta G_X^+ G_X
      const int s = e / r, t = e % r;
      cd acc = cd_make(0.0, 0.0);
      for (int u = 0; u < r; ++u) cd_fma(acc, gp[s * r + u], gx[u * r + t]);
      go.qx[(size_t)b * rr + e] = cd_make((s == t ? 1.0 : 0.0) - go.eta * acc.re, -go.eta * acc.im);
    }
  }
  if (tid == 0) go.qx_zero[b] = qzero ? 1 : 0;
}

// ---------------------------------------------------------------- X~^* W~, and G_X with its inverse
// Real form: C'[2s + d][2j + c] = sum_i X'[2s + d][i] W'[i][2j + c] with X'[2s + d][i] =
// (re, im)_d X~(i, s) and W' the interleaved W~ rows; then
// (X~^* W~)(s, j) = (C'[2s][2j] + C'[2s+1][2j+1], C'[2s][2j+1] - C'[2s+1][2j]).
// Block: one chunk of at most 64 rows x one frequency.  The chunk's X~ rows and, per pass
// of BG_COLS columns, its whole W~ slab are staged in LDS with every load of a thread
// issued at once; each wavefront owns a quarter of the 16-column tiles of a pass, on the
// FP64 matrix cores.
// At r <= 16 the first nb blocks of the launch instead form, for frequency blockIdx.x, the
// whole Gram G_X = X~^* X~ + rho1 (H X~)^*(H X~) in FP64 on the matrix cores, its
// pseudo-inverse and I - eta P_X (gramx_block), beside the products; at r > 16 k_gramx
// does this work in a launch of its own.
#define BG_COLS 64                  // complex columns per pass
#define BG_MAXROWS 64               // rows per chunk at most
#define BG_WLD (2 * BG_COLS + 16)   // LDS row stride of the staged W~ slab (floats)
template <int RM>   // r <= RM; registers and LDS allow three blocks per compute unit at r <= 16
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RM <= 16 ? 2 : 1)))
k_bgemm(const void* __restrict__ wt, const float2* __restrict__ xt, double2* __restrict__ bpart, GramOut go, int n1,
        int n2, int r, int nb, int nchunk, int chunk, int mixed) {
  extern __shared__ __align__(16) float smb[];
  constexpr bool GRAM = RM <= 16;   // at r > 16 the registers of both paths would not fit twice
  const int ng = GRAM ? nb : 0;   // G_X blocks at the front of the grid
  if constexpr (GRAM) {
    if ((int)blockIdx.x < ng) {
      gramx_block<RM>(blockIdx.x, xt, n1, r, go, (unsigned char*)smb);
      return;
    }
  }
  const int xld = 2 * r + 16;                    // LDS row stride of the staged X~ rows (floats)
  float* xs = smb;                               // [chunk + 1][xld]: (re, im) of X~(i, s) at 2 s
  float* ws = smb + (size_t)(chunk + 1) * xld;   // [chunk rounded up to 4][BG_WLD]
  const int c = ((int)blockIdx.x - ng) % nchunk, b = ((int)blockIdx.x - ng) / nchunk, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int i0 = c * chunk, i1 = min(n1, i0 + chunk), nrows = i1 - i0;
  const int rows = nrows;
  const int nks = (nrows + 3) / 4;   // K steps of 4 rows
  // W~ slab of one pass: rows i0 .. i1 - 1 (zeros up to a multiple of 4), columns
  // j0 .. j0 + nc - 1; 16 elements per thread, loaded into registers ahead of their use
  constexpr int SLAB_PER = BG_MAXROWS * BG_COLS / 256;
  float2 slab[SLAB_PER];
  auto load_slab = [&](int j0) {
    const int nc = min(BG_COLS, n2 - j0);
    // (the storage branch outside the unrolled loops, so that no load waits at a join)
    if (mixed) {
#pragma unroll
      for (int u = 0; u < SLAB_PER; ++u) {
        const int e = tid + 256 * u, rr = e / BG_COLS, jj = e % BG_COLS;
        const size_t idx = ((size_t)(i0 + rr) * nb + b) * n2 + j0 + jj;
        slab[u] = unpack_bf16x2(ld_or((const uint32_t*)wt, idx, rr < nrows && jj < nc, 0u));
      }
    } else {
#pragma unroll
      for (int u = 0; u < SLAB_PER; ++u) {
        const int e = tid + 256 * u, rr = e / BG_COLS, jj = e % BG_COLS;
        const size_t idx = ((size_t)(i0 + rr) * nb + b) * n2 + j0 + jj;
        slab[u] = ld_or((const float2*)wt, idx, rr < nrows && jj < nc, make_float2(0.f, 0.f));
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
    // FP64 matrix-core tiles over every row of the chunk: X~ and W~ are FP32 (or BF16)
    // values, exact in FP64, so the partial sums carry FP64 rounding only (the Y-step's
    // G_X^{-1} amplifies any rounding of X~^* W~)
    v4d acc[MT][2];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int u = 0; u < 2; ++u) acc[a][u] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < nks; ++ks) {
      const int kr = 4 * ks + q;   // chunk row of this lane's K index
      double av[MT];
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int sp = 16 * a + m;   // row 2 s + d of X'
        av[a] = (sp < 2 * r && kr < nrows) ? (double)xs[kr * xld + sp] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int nt = w + 4 * u;
        if (nt < ntiles) {
          const double bv = (double)ws[kr * BG_WLD + 16 * nt + m];
#pragma unroll
          for (int a = 0; a < MT; ++a) acc[a][u] = mfma4d(av[a], bv, acc[a][u]);
        }
      }
    }
    // combine C' into (X~^* W~)(s, j): element t of lane (q, m) holds row 16 a + q + 4 t and
    // column 16 nt + m of its tile, so the lanes with q and m even hold C'[2s][2j] and read
    // C'[2s][2j+1], C'[2s+1][2j] and C'[2s+1][2j+1] from lanes + 1, + 16 and + 17
#pragma unroll
    for (int a = 0; a < MT; ++a) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int nt = w + 4 * u;   // the same in the whole wavefront
        if (nt < ntiles) {
          const int j = (16 * nt + m) >> 1;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double s0 = acc[a][u][t], s1 = __shfl_down(s0, 1), s16 = __shfl_down(s0, 16),
                         s17 = __shfl_down(s0, 17);
            const int s = (16 * a + q + 4 * t) >> 1;
            if (!(q & 1) && !(m & 1) && s < r && j < nc)
              bpart[(((size_t)b * nchunk + c) * r + s) * n2 + j0 + j] = make_double2(s0 + s17, s1 - s16);
          }
        }
      }
    }
  }
}

// G_X alone, one block per frequency (r > 16: beside the products it would cost them
// registers).
template <int RM>
__global__ void __launch_bounds__(256) k_gramx(const float2* __restrict__ xt, GramOut go, int n1, int r) {
  extern __shared__ __align__(16) unsigned char smg[];
  gramx_block<RM>(blockIdx.x, xt, n1, r, go, smg);
}


size_t bgemm_lds_bytes(int r, int chunk) {
  const int rm = r <= 8 ? 8 : (r <= 16 ? 16 : 32);
  const size_t slab = (size_t)((chunk + 3) / 4 * 4) * BG_WLD * sizeof(float);
  const size_t chunkb = (size_t)(chunk + 1) * (2 * r + 16) * sizeof(float) + slab;
  const size_t gram = gramx_lds_bytes(r, rm);
  return chunkb > gram ? chunkb : gram;
}

void bgemm_set_attr(size_t lds) {
  if (lds > 65536) {
    (void)hipFuncSetAttribute((const void*)k_bgemm<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_bgemm<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_bgemm<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_gramx<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
}

void launch_bgemm(const Plan& p) {
  const bool fused = p.r <= 16;
  const int grid = (fused ? p.nb : 0) + p.nchunk * p.nb;   // G_X blocks first, then (chunk, frequency)
  const size_t lds = bgemm_lds_bytes(p.r, p.chunk);
  GramOut go;
  go.gxm = p.gxm;
  go.dmat = p.dmat;
  go.gxp = p.gxp;
  go.qx = p.qx;
  go.qx_zero = p.qx_zero;
  go.rho1 = p.rho1;
  go.eta = p.eta;
  go.force_eigen = p.force_eigen;
#define TCTF_BGEMM(RM)                                                                                  \
  k_bgemm<RM><<<grid, 256, lds, p.stream>>>(p.wt, p.xt, p.bpart, go, p.n1, p.n2, p.r, p.nb, p.nchunk, \
                                            p.chunk, p.mixed)
  if (p.r <= 8) {
    TCTF_BGEMM(8);
  } else if (p.r <= 16) {
    TCTF_BGEMM(16);
  } else {
    k_gramx<32><<<p.nb, 256, lds, p.stream>>>(p.xt, go, p.n1, p.r);
    TCTF_BGEMM(32);
  }
#undef TCTF_BGEMM
}

}  // namespace tctf

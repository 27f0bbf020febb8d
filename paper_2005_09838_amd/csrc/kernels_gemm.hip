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

// Mixed precision: the same product on the BF16 matrix cores (16 x 16 x 16 tiles, FP32
// accumulation).  Each FP32 factor value v is split into v_hi = bf16(v) and v_lo =
// bf16(v - v_hi) (round to nearest), and Z' = X'_hi Y'_hi + X'_hi Y'_lo + X'_lo Y'_hi: three
// BF16 products that keep about 16 bits of each operand, so Z~ carries errors near 2^-17
// relative instead of BF16's 2^-9.  Z~ feeds the W-step directly: BF16-sized noise there,
// new every iteration, made the iterate wander along the weakly determined directions of
// the completion (the RSE drifting by a few percent over thousands of iterations), while the
// split products leave it where the FP32 iteration goes.
// Lane (m, q) supplies A[m][4 q + e] and B[4 q + e][m], e = 0..3, of each 16-deep K chunk:
// in chunk c, K index 16 c + 4 q + e is (s, d) = (8 c + 2 q + e / 2, e % 2), so the lane's A
// values are (re, im) of X~(row, s0) and X~(row, s0 + 1), s0 = 8 c + 2 q, and its B values
// the signed parts of Y~(s0, j) and Y~(s0 + 1, j) (see Y' above).  Output tiles as k_zgemm's.
typedef short v4s __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4f mfma16bf(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// (hi, lo) BF16 parts of x, as the low and high halves of one word
__device__ __forceinline__ uint32_t bf16_split(float x) {
  const uint16_t h = f32_to_bf16(x);
  return (uint32_t)h | ((uint32_t)f32_to_bf16(x - bf16_to_f32(h)) << 16);
}
template <int RM>
__global__ void __launch_bounds__(256) k_zgemm_bf(const float2* __restrict__ xt, const float2* __restrict__ yt,
                                                  float2* __restrict__ zt, int n1, int n2, int r, int nb,
                                                  int npinv, PinvyArgs pa) {
  extern __shared__ __align__(16) unsigned char zsm[];
  if ((int)blockIdx.x < npinv) {
    pinvy_block(blockIdx.x, pa, zsm);
    return;
  }
  uint2* ysh = (uint2*)zsm;   // [s][j] of the column chunk: (re, im) split words
  const int bid = blockIdx.x - npinv, ntile = (n1 + ZG_ROWS - 1) / ZG_ROWS;
  const int i0 = (bid % ntile) * ZG_ROWS, b = bid / ntile, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  constexpr int KC = RM / 8;   // 16-deep K chunks over 2 RM
  constexpr int YPER = RM * ZG_COLS / 256;
  float2 yv[YPER];
  auto load_y = [&](int j0) {
    const int nc = min(ZG_COLS, n2 - j0);
#pragma unroll
    for (int u = 0; u < YPER; ++u) {
      const int e = tid + 256 * u, s = e / ZG_COLS, jj = e % ZG_COLS;
      yv[u] = ld_or(yt, ((size_t)b * r + s) * n2 + j0 + jj, s < r && jj < nc, make_float2(0.f, 0.f));
    }
  };
  load_y(0);
  // A operands: X~(row, s0), X~(row, s0 + 1) of each chunk, split
  const int row = i0 + 16 * w + m;
  v4s ahi[KC], alo[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    uint32_t h[4];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int s = 8 * c + 2 * q + d;
      const float2 xv = xt[((size_t)b * r + min(s, r - 1)) * n1 + min(row, n1 - 1)];   // clamped, unconditional
      const float2 x = (s < r && row < n1) ? xv : make_float2(0.f, 0.f);
      h[2 * d] = bf16_split(x.x);
      h[2 * d + 1] = bf16_split(x.y);
    }
    ahi[c] = v4s{(short)(h[0] & 0xffffu), (short)(h[1] & 0xffffu), (short)(h[2] & 0xffffu), (short)(h[3] & 0xffffu)};
    alo[c] = v4s{(short)(h[0] >> 16), (short)(h[1] >> 16), (short)(h[2] >> 16), (short)(h[3] >> 16)};
  }
  float* zf = (float*)zt;
  const bool vec4 = (n2 & 1) == 0;   // rows start 16-byte aligned
  for (int j0 = 0; j0 < n2; j0 += ZG_COLS) {
    const int nc = min(ZG_COLS, n2 - j0);
    if (j0 > 0) {
      __syncthreads();   // every wavefront is done with the previous chunk
      load_y(j0);
    }
#pragma unroll
    for (int u = 0; u < YPER; ++u) ysh[tid + 256 * u] = make_uint2(bf16_split(yv[u].x), bf16_split(yv[u].y));
    __syncthreads();
    const int ntiles = (2 * nc + 15) / 16;
    for (int nt0 = 0; nt0 < ntiles; nt0 += 4) {
      v4f acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int s0 = 8 * c + 2 * q;   // rows past r are zero in the chunk
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jj = min(8 * nt0 + 2 * m + (u >> 1), ZG_COLS - 1);
          const uint2 y0 = ysh[s0 * ZG_COLS + jj], y1 = ysh[(s0 + 1) * ZG_COLS + jj];   // (re, im) split words
          v4s bh, bl;
          if (u & 1) {   // column 2 j + 1: (Yi, Yr, Yi', Yr')
            bh = v4s{(short)(y0.y & 0xffffu), (short)(y0.x & 0xffffu), (short)(y1.y & 0xffffu), (short)(y1.x & 0xffffu)};
            bl = v4s{(short)(y0.y >> 16), (short)(y0.x >> 16), (short)(y1.y >> 16), (short)(y1.x >> 16)};
          } else {       // column 2 j: (Yr, -Yi, Yr', -Yi')
            bh = v4s{(short)(y0.x & 0xffffu), (short)((y0.y & 0xffffu) ^ 0x8000u), (short)(y1.x & 0xffffu),
                     (short)((y1.y & 0xffffu) ^ 0x8000u)};
            bl = v4s{(short)(y0.x >> 16), (short)((y0.y >> 16) ^ 0x8000u), (short)(y1.x >> 16),
                     (short)((y1.y >> 16) ^ 0x8000u)};
          }
          acc[u] = mfma16bf(alo[c], bh, acc[u]);
          acc[u] = mfma16bf(ahi[c], bl, acc[u]);
          acc[u] = mfma16bf(ahi[c], bh, acc[u]);
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
            } else {
              *(float2*)dst = make_float2(acc[0][t], acc[1][t]);
            }
          }
        }
      }
    }
  }
}

void zgemm_set_attr(int r) {
  if (pinvy_lds_bytes(r) > 65536) {
    (void)hipFuncSetAttribute((const void*)k_zgemm<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pinvy_lds_bytes(r));
    (void)hipFuncSetAttribute((const void*)k_zgemm_bf<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pinvy_lds_bytes(r));
  }
}

void launch_zgemm(const Plan& p, int with_pinv) {
  const int npinv = with_pinv ? p.nb : 0;
  const int grid = npinv + (p.n1 + ZG_ROWS - 1) / ZG_ROWS * p.nb;
  const int rm = p.r <= 8 ? 8 : (p.r <= 16 ? 16 : 32);
  size_t lds = (size_t)rm * ZG_COLS * sizeof(float2);
  if (with_pinv && pinvy_lds_bytes(p.r) > lds) lds = pinvy_lds_bytes(p.r);
  const PinvyArgs pa = pinvy_args(p);
#define TCTF_ZGEMM(RM)                                                                                         \
  do {                                                                                                         \
    if (p.mixed)                                                                                               \
      k_zgemm_bf<RM><<<grid, 256, lds, p.stream>>>(p.xt, p.yt, p.zt, p.n1, p.n2, p.r, p.nb, npinv, pa);        \
    else                                                                                                       \
      k_zgemm<RM><<<grid, 256, lds, p.stream>>>(p.xt, p.yt, p.zt, p.n1, p.n2, p.r, p.nb, npinv, pa);           \
  } while (0)
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
// pass with every W~ load of the pass issued before the products.
// Epilogue, in FP64, with U = X~ (I - eta P_Y) (U = 0 when I - eta P_Y is exactly 0):
// * hk >= 0: the whole X-update.  Since X~_new = H_rho1^{-1} (eta A G_Y^+ + H_rho1 U) =
//   U + eta H_rho1^{-1} V with V = A G_Y^+, and H_rho1^{-1} is the stencil of hinv_stencil,
//   the block forms V on its 64 rows (zero outside the matrix) and writes X~_new on the
//   64 - 2 hk rows whose stencil lies inside them; consecutive blocks overlap by 2 hk rows.
//   U needs X~ on the output rows only, which no other block writes, so X~ is updated in
//   place.  Real bins (b = 0, n3 / 2) keep a zero imaginary part.
// * hk = -1: the right-hand side R = eta A G_Y^+ + H_rho1 U for k_hsolve.
#define AG_ROWS 64
#define AG_COLS 128
struct HStencil {
  int k;                            // half-width, -1: right-hand side only
  double tap[2 * HINV_KMAX + 2];    // c lambda^d
};
template <int RM, bool MIXED>   // r <= RM; MIXED: W~ stored as packed bf16 pairs
__global__ void __launch_bounds__(256) k_agemm(const void* wt, const float2* __restrict__ yt,
                                               const float2* xt, const cd* __restrict__ gyp,   // xt may be xout
                                               const cd* __restrict__ qy, const int* __restrict__ qy_zero,
                                               float2* __restrict__ rhs, int n1, int n2, int r, int nb,
                                               double eta, double rho1, int raw_a, uint32_t* ctr,
                                               float2* xout, int n3, HStencil hs) {
  __shared__ __align__(16) float2 ysh[RM * AG_COLS];   // [s][j] of the column chunk (MIXED: split words)
  __shared__ __align__(16) float2 ash[AG_ROWS * RM];   // A rows, then the results
  __shared__ __align__(16) cd gs[RM * RM];             // G_Y^+
  __shared__ __align__(16) cd vsh[RM <= 16 ? AG_ROWS * RM : 1];   // V = A G_Y^+ [s][row] (stencil only)
  __shared__ double tsh[2 * HINV_KMAX + 2];                        // the stencil's taps
  const int hk = (RM <= 16 && !raw_a) ? hs.k : -1;
#pragma unroll
  for (int d = 0; d < 2 * HINV_KMAX + 2; ++d)   // constant indices: the taps stay in the argument segment
    if ((int)threadIdx.x == d && d <= 2 * hk + 1) tsh[d] = hs.tap[d];   // read after the first barrier
  // with the stencil, block x covers rows x (64 - 2 hk) - hk .. + 63 (some outside the matrix)
  const int i0 = hk >= 0 ? (int)blockIdx.x * (AG_ROWS - 2 * hk) - hk : (int)blockIdx.x * AG_ROWS;
  const int b = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int row = i0 + 16 * w + m;
  const bool row_in = row >= 0 && row < n1;
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
    const raw_t* wrow = (const raw_t*)wt + ((size_t)min(max(row, 0), n1 - 1) * nb + b) * n2 + j0 + 2 * q;
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
      const float2 y = (s < r && jj < nc) ? yv[u] : make_float2(0.f, 0.f);
      if constexpr (MIXED) ((uint2*)ysh)[e] = make_uint2(bf16_split(y.x), bf16_split(y.y));
      else ysh[e] = y;
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < AG_COLS / 8; ++g) {
      if (g < ngroups) {
        const int valid = row_in ? min(2, nc - (8 * g + 2 * q)) : 0;
        if constexpr (MIXED) {
          // BF16 matrix cores: this lane's four K values are the two packed W~ words as they
          // are (exact), Y~ enters split into its hi and lo BF16 parts (two products)
          const uint32_t w0 = valid > 0 ? lo[g] : 0u, w1 = valid > 1 ? hi[g] : 0u;
          const v4s av = v4s{(short)(w0 & 0xffffu), (short)(w0 >> 16), (short)(w1 & 0xffffu), (short)(w1 >> 16)};
#pragma unroll
          for (int u = 0; u < NNT; ++u) {
            const int s = min((16 * u + m) >> 1, r - 1);   // columns past 2r are dropped below
            const uint4 y2 = *(const uint4*)&((const uint2*)ysh)[s * AG_COLS + 8 * g + 2 * q];   // split (re, im) of Y~(s, j), Y~(s, j + 1)
            // e = 0: (Yr, Yi, Yr', Yi');  e = 1: (-Yi, Yr, -Yi', Yr'), per part
            v4s bh, bl;
            if (eodd) {
              bh = v4s{(short)((y2.y & 0xffffu) ^ 0x8000u), (short)(y2.x & 0xffffu), (short)((y2.w & 0xffffu) ^ 0x8000u),
                       (short)(y2.z & 0xffffu)};
              bl = v4s{(short)((y2.y >> 16) ^ 0x8000u), (short)(y2.x >> 16), (short)((y2.w >> 16) ^ 0x8000u),
                       (short)(y2.z >> 16)};
            } else {
              bh = v4s{(short)(y2.x & 0xffffu), (short)(y2.y & 0xffffu), (short)(y2.z & 0xffffu), (short)(y2.w & 0xffffu)};
              bl = v4s{(short)(y2.x >> 16), (short)(y2.y >> 16), (short)(y2.z >> 16), (short)(y2.w >> 16)};
            }
            acc[u] = mfma16bf(av, bl, acc[u]);
            acc[u] = mfma16bf(av, bh, acc[u]);
          }
        } else {
          const float2 a0 = lo[g], a1 = hi[g], z = make_float2(0.f, 0.f);
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
  // thread (il, qq) = (tid / 4, tid % 4) takes row i0 + il, columns s = qq, qq + 4, ...
  const int il = tid >> 2, qq = tid & 3, i = i0 + il;
  constexpr int SP = RM / 4;
  if (hk >= 0) {
    {
      cd ag[SP];   // V(i, :) = A(i, :) G_Y^+, one independent chain per column
#pragma unroll
      for (int us = 0; us < SP; ++us) ag[us] = cd_make(0.0, 0.0);
      if (i >= 0 && i < n1) {
        for (int u = 0; u < r; ++u) {
          const float2 av = ash[il * r + u];
          const cd a = cd_make(av.x, av.y);
#pragma unroll
          for (int us = 0; us < SP; ++us) cd_fma(ag[us], a, gs[u * r + min(qq + 4 * us, r - 1)]);
        }
      }
#pragma unroll
      for (int us = 0; us < SP; ++us)
        if (qq + 4 * us < r) vsh[(qq + 4 * us) * AG_ROWS + il] = ag[us];
    }
    __syncthreads();   // V of every row of the block is in LDS
    // thread (ro, sg) = (tid % 64, tid / 64): row i0 + ro, columns s = sg, sg + 4, ...
    const int ro = tid & 63, sg = tid >> 6, io = i0 + ro;
    const bool out = io >= 0 && io < n1 && ro >= hk && ro < AG_ROWS - hk;
    cd t[SP];
#pragma unroll
    for (int us = 0; us < SP; ++us) t[us] = cd_make(0.0, 0.0);
    if (out) {
      // (H_rho1^{-1} V)(io, s): direct tap c lambda^|io - j| plus the reflections in the two
      // ends, c lambda^(io + j + 1) and c lambda^(2 n1 - 1 - io - j), where within the table
      const int tmax = 2 * hk + 1;
      for (int d = -hk; d <= hk; ++d) {
        const int j = io + d;
        if (j < 0 || j >= n1) continue;
        const int e1 = io + j + 1, e2 = 2 * n1 - 1 - io - j;
        const double wgt = tsh[d < 0 ? -d : d] + (e1 <= tmax ? tsh[min(e1, tmax)] : 0.0) +
                           (e2 <= tmax ? tsh[min(e2, tmax)] : 0.0);
#pragma unroll
        for (int us = 0; us < SP; ++us) {
          const cd v = vsh[min(sg + 4 * us, r - 1) * AG_ROWS + ro + d];
          t[us].re = fma(wgt, v.re, t[us].re);
          t[us].im = fma(wgt, v.im, t[us].im);
        }
      }
#pragma unroll
      for (int us = 0; us < SP; ++us) t[us] = cd_scale(t[us], eta);
      if (!noqy) {
        for (int v2 = 0; v2 < r; ++v2) {
          const float2 x0 = xt[((size_t)b * r + v2) * n1 + io];
          const cd xv = cd_make(x0.x, x0.y);
#pragma unroll
          for (int us = 0; us < SP; ++us) cd_fma(t[us], xv, qs[v2 * r + min(sg + 4 * us, r - 1)]);
        }
      }
    }
    __syncthreads();   // every X~ read of the block is done before X~ is overwritten
    if (out) {
      const bool real_bin = bin_is_real(b, n3);
#pragma unroll
      for (int us = 0; us < SP; ++us) {
        const int s = sg + 4 * us;
        if (s < r) xout[((size_t)b * r + s) * n1 + io] = make_float2((float)t[us].re, real_bin ? 0.0f : (float)t[us].im);
      }
    }
    return;
  }
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

// H_rho1 = I + rho1 D^T D (D: first differences along mode 1) is tridiagonal with
// diagonal 1 + 2 rho1 (1 + rho1 in the end rows) and off-diagonal -rho1.  Away from the
// ends its inverse is c lambda^|i - j|, lambda the root in (0, 1) of
// rho1 lambda^2 - (1 + 2 rho1) lambda + rho1 = 0 and c = lambda / (rho1 (1 - lambda^2));
// an end row is a mirror (the row equation holds with a ghost entry equal to the end
// entry), which adds the image terms c lambda^(i + j + 1) and c lambda^(2 n1 - 1 - i - j).
// The images of images are below lambda^(2 n1), and dropping every tap with |i - j| > k
// changes a result by at most c lambda^(k + 1) / (1 - lambda) times the largest |V| there:
// k is the least with lambda^(k + 1) <= 2^-40: below FP32's rounding unit even where
// neighbouring rows differ in scale by 10^4 (k = 5 at rho1 = 0.01, 11 at rho1 = 0.1).
int hinv_stencil(double rho1, int n1, int r, double* tap) {
  if (r > 16 || !(rho1 >= 0.0)) return -1;
  double lam = 0.0, c = 1.0;
  if (rho1 > 0.0) {
    const double a = 1.0 + 2.0 * rho1;
    lam = 2.0 * rho1 / (a + sqrt(a * a - 4.0 * rho1 * rho1));   // the small root, without cancellation
    c = lam / (rho1 * (1.0 - lam * lam));
  }
  int k = 0;
  double p = lam;   // lambda^(k + 1)
  while (p > 0x1p-40 && k <= HINV_KMAX) {
    p *= lam;
    ++k;
  }
  if (k > HINV_KMAX || n1 < 2 * k + 2) return -1;
  double v = c;
  for (int d = 0; d <= 2 * k + 1; ++d) {
    tap[d] = v;
    v *= lam;
  }
  return k;
}

void launch_agemm(const Plan& p, int raw_a, int advance, int scratch_out) {
  HStencil hs;
  hs.k = raw_a ? -1 : p.hk;
  for (int d = 0; d < 2 * HINV_KMAX + 2; ++d) hs.tap[d] = d <= 2 * hs.k + 1 ? p.htap[d] : 0.0;
  const int rows = hs.k >= 0 ? AG_ROWS - 2 * hs.k : AG_ROWS;
  float2* xout = scratch_out ? p.rhs : p.xt;
  dim3 grid((p.n1 + rows - 1) / rows, p.nb);
#define TCTF_AGEMM(RM, MX)                                                                                    \
  k_agemm<RM, MX><<<grid, 256, 0, p.stream>>>(p.wt, p.yt, p.xt, p.gyp, p.qy, p.qy_zero, p.rhs, p.n1, p.n2, p.r, \
                                              p.nb, p.eta, p.rho1, raw_a, advance ? p.ctr : nullptr, xout, p.n3, hs)
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

// Outputs of the G_X launches, per frequency b ([nb][r][r] FP64 complex unless noted).
struct GramOut {
  cd* gxm;       // G_X
  cd* dmat;      // (H X~)^*(H X~)
  cd* gxp;       // G_X^+
  cd* qx;        // I - eta G_X^+ G_X (not written when it is exactly 0)
  int* qx_zero;  // [nb] 1 when I - eta P_X = 0
  double rho1, eta;
  int force_eigen;
};

// ---------------------------------------------------------------- G_X in two launches
// k_gramx_part: block (row group g, frequency b) forms over its GXR rows i0 .. i0 + GXR - 1
// the FP64 partial Grams S_g = sum_i X~(i, :)^* X~(i, :) and, with the next row staged too,
// D_g = sum_i (X~(i+1, :) - X~(i, :))^* (X~(i+1, :) - X~(i, :)) (no difference past the last
// row), as the real Gram C = X'^T X' of X'[i][2s + d] = (re, im)_d X~(i, s) on the FP64
// matrix cores: the rows are staged column by column (X'^T; zeros past n1 and r), and within
// 16 rows the K order is permuted so that lane (m, q) feeds rows 4q .. 4q + 3, one 16-byte LDS
// read (and one float of the next row) serving four steps.  At r <= 8 the four wavefronts
// share the one tile and split the rows; otherwise each takes its tiles.  The lanes holding
// C[2s][2t] gather the 2 x 2 real block by shuffles: X~^* X~ (s, t) = (C[2s][2t] +
// C[2s+1][2t+1], C[2s][2t+1] - C[2s+1][2t]), likewise D.
// k_gramx_inv: per frequency, the partials summed in a fixed order, G_X = S + rho1 D
// (= X~^* H_rho1 X~), its pseudo-inverse (Lemma SVPMPI, pinv_herm) and I - eta P_X.
#define GXR 64
template <int RM>
__global__ void __launch_bounds__(256) k_gramx_part(const float2* __restrict__ xt, int n1, int r, int ngrp,
                                                    cd* __restrict__ part) {
  constexpr int MT = RM / 8, NT = MT * MT;         // 16 x 16 tiles of the real Gram
  constexpr int KS = NT >= 4 ? 1 : 4 / NT;         // wavefronts sharing a tile (row split)
  constexpr int TPW = NT >= 4 ? NT / 4 : 1;        // tiles per wavefront
  constexpr int LD = GXR + 4;                      // LDS stride of a staged column (floats)
  constexpr int PER = ((GXR + 1) * RM + 255) / 256;
  __shared__ __align__(16) float xs[2 * RM * LD];
  __shared__ cd red[KS > 1 ? 2 * KS * RM * RM : 1];
  const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, w = tid >> 6, m = lane & 15,
            q = lane >> 4;
  const int i0 = g * GXR, rr = r * r, kp = KS > 1 ? w : 0;
  const int nrows = min(GXR, n1 - i0);
  {
    float2 pf[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, s = e / (GXR + 1), h = e % (GXR + 1);
      pf[u] = ld_or(xt, ((size_t)b * r + s) * n1 + i0 + h, s < r && i0 + h < n1, make_float2(0.f, 0.f));
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, s = e / (GXR + 1), h = e % (GXR + 1);
      if (s < RM) {
        xs[(2 * s) * LD + h] = pf[u].x;
        xs[(2 * s + 1) * LD + h] = pf[u].y;
      }
    }
  }
  __syncthreads();
  v4d acs[TPW], acd[TPW];
#pragma unroll
  for (int tu = 0; tu < TPW; ++tu) {
    acs[tu] = v4d{0.0, 0.0, 0.0, 0.0};
    acd[tu] = v4d{0.0, 0.0, 0.0, 0.0};
    const int tile = KS > 1 ? 0 : w + 4 * tu;
    const float* pa = xs + (16 * (tile / MT) + m) * LD;   // column 2 s + d of X'
    const float* pb = xs + (16 * (tile % MT) + m) * LD;
    for (int jb = kp; 16 * jb < nrows; jb += KS) {
      const int h0 = 16 * jb + 4 * q;
      const float4 a4 = *(const float4*)(pa + h0), b4 = *(const float4*)(pb + h0);
      const double av[5] = {a4.x, a4.y, a4.z, a4.w, pa[h0 + 4]};
      const double bv[5] = {b4.x, b4.y, b4.z, b4.w, pb[h0 + 4]};
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const bool dif = i0 + h0 + jj + 1 < n1;   // the row pair (i, i + 1) exists
        const double a1 = dif ? av[jj + 1] - av[jj] : 0.0, b1 = dif ? bv[jj + 1] - bv[jj] : 0.0;
        acs[tu] = mfma4d(av[jj], bv[jj], acs[tu]);
        acd[tu] = mfma4d(a1, b1, acd[tu]);
      }
    }
  }
  // element t of lane (q, m): real row 16 ta + q + 4 t, column 16 tb + m
  cd* out = part + (size_t)(b * ngrp + g) * 2 * rr;
#pragma unroll
  for (int tu = 0; tu < TPW; ++tu) {
    const int tile = KS > 1 ? 0 : w + 4 * tu, ta = tile / MT, tb = tile % MT;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double s0 = acs[tu][t], s1 = __shfl_down(s0, 1), s16 = __shfl_down(s0, 16), s17 = __shfl_down(s0, 17);
      const double d0 = acd[tu][t], d1 = __shfl_down(d0, 1), d16 = __shfl_down(d0, 16), d17 = __shfl_down(d0, 17);
      const int sr = (16 * ta + q + 4 * t) >> 1, sc = (16 * tb + m) >> 1;
      if (!(q & 1) && !(m & 1) && sr < r && sc < r) {
        const cd vs = cd_make(s0 + s17, s1 - s16), vd = cd_make(d0 + d17, d1 - d16);
        if (KS > 1) {
          red[(2 * kp) * rr + sr * r + sc] = vs;
          red[(2 * kp + 1) * rr + sr * r + sc] = vd;
        } else {
          out[sr * r + sc] = vs;
          out[rr + sr * r + sc] = vd;
        }
      }
    }
  }
  if constexpr (KS > 1) {
    __syncthreads();
    for (int e = tid; e < 2 * rr; e += 256) {
      const int which = e / rr, k = e % rr;
      cd v = red[which * rr + k];
      for (int j = 1; j < KS; ++j) v = cd_add(v, red[(2 * j + which) * rr + k]);   // fixed order
      out[e] = v;
    }
  }
}

#define GXI_B 12   // row-group partials loaded at once
__global__ void __launch_bounds__(256) k_gramx_inv(const cd* __restrict__ part, int ngrp, int r, GramOut go) {
  // this small launch runs beside the X~^* W~ product on the same compute units: its
  // wavefronts take issue priority there, since the Y-step waits for the later of the two
  __builtin_amdgcn_s_setprio(3);
  extern __shared__ __align__(16) unsigned char sm[];
  const int b = blockIdx.x, tid = threadIdx.x, rr = r * r;
  cd* gx = (cd*)sm;
  cd* gp = gx + rr;
  PinvScratch ps;
  ps.work = gp + rr;
  ps.vec = ps.work + rr;
  ps.colk = ps.vec + rr;
  ps.rowk = ps.colk + r;
  ps.rot = (double*)(ps.rowk + r);
  ps.red = ps.rot + 96;
  for (int e = tid; e < rr; e += 256) {
    cd sv = cd_make(0.0, 0.0), dv = cd_make(0.0, 0.0);
    const cd* pb = part + (size_t)b * ngrp * 2 * rr + e;
    for (int g0 = 0; g0 < ngrp; g0 += GXI_B) {   // GXI_B groups' loads in flight, summed in group order
      cd vs[GXI_B], vd[GXI_B];
#pragma unroll
      for (int k = 0; k < GXI_B; ++k) {
        const bool ok = g0 + k < ngrp;
        vs[k] = ld_or(pb, (size_t)(g0 + k) * 2 * rr, ok, cd_make(0.0, 0.0));
        vd[k] = ld_or(pb, (size_t)(g0 + k) * 2 * rr + rr, ok, cd_make(0.0, 0.0));
      }
#pragma unroll
      for (int k = 0; k < GXI_B; ++k) {
        if (g0 + k < ngrp) {
          sv = cd_add(sv, vs[k]);
          dv = cd_add(dv, vd[k]);
        }
      }
    }
    const cd gv = cd_add(sv, cd_scale(dv, go.rho1));
    go.gxm[(size_t)b * rr + e] = gv;
    go.dmat[(size_t)b * rr + e] = dv;
    gx[e] = gv;
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

int gramx_groups(int n1) { return (n1 + GXR - 1) / GXR; }

// LDS the inversion launch asks for when the X~^* W~ product beside it leaves compute units
// free: more than a compute unit (160 KB) holds next to one product block, so the inversions
// run on the free units instead of sharing one with the product (FP64 arithmetic beside FP64
// matrix-core work there ran 2.5 times slower)
#define GXI_LDS_ALONE (150 * 1024)
void gramx_set_attr(int r) {
  (void)r;
  (void)hipFuncSetAttribute((const void*)k_gramx_inv, hipFuncAttributeMaxDynamicSharedMemorySize, GXI_LDS_ALONE);
}

void launch_gramx(const Plan& p) {
  GramOut go;
  go.gxm = p.gxm;
  go.dmat = p.dmat;
  go.gxp = p.gxp;
  go.qx = p.qx;
  go.qx_zero = p.qx_zero;
  go.rho1 = p.rho1;
  go.eta = p.eta;
  go.force_eigen = p.force_eigen;
  const int ngrp = gramx_groups(p.n1);
  const dim3 grid(ngrp, p.nb);
  if (p.r <= 8) k_gramx_part<8><<<grid, 256, 0, p.stream>>>(p.xt, p.n1, p.r, ngrp, p.gxpart);
  else if (p.r <= 16) k_gramx_part<16><<<grid, 256, 0, p.stream>>>(p.xt, p.n1, p.r, ngrp, p.gxpart);
  else k_gramx_part<32><<<grid, 256, 0, p.stream>>>(p.xt, p.n1, p.r, ngrp, p.gxpart);
  size_t lds = pinvy_lds_bytes(p.r);
  if ((long)((p.n2 + p.bcg - 1) / p.bcg) * p.nb < p.ncu && lds < GXI_LDS_ALONE) lds = GXI_LDS_ALONE;
  k_gramx_inv<<<p.nb, 256, lds, p.stream>>>(p.gxpart, ngrp, p.r, go);
}

// ---------------------------------------------------------------- X~^* W~
// Real form with the real and imaginary parts in separate tiles: X''[p RM + s][i] =
// (re, im)_p X~(i, s) and W''[i][p CW + c] = (re, im)_p W~(i, j0 + c), C = X''^T W'', so
// (X~^* W~)(s, j0 + c) = (C[s][c] + C[RM + s][CW + c], C[s][CW + c] - C[RM + s][c]) and the
// four terms of one output sit in the same lane and element of four tiles.  Each lane loads
// X~(i, s) and W~(i, j) once per K step and feeds both parts to the FP64 matrix cores.
// Block: one frequency b and CW = 16 WL complex columns, reduced over every row i in the
// block: its BG_W wavefronts take contiguous ranges of 4-row K steps (XL = RM / 16 row
// tiles and WL column tiles of each part), with two groups of loads in flight.  X~ and W~
// are FP32 or BF16 values, exact in FP64, so the sums carry FP64 rounding only (the Y-step's
// G_X^+ amplifies any rounding of X~^* W~).  The wavefronts' complex results are added in a
// fixed tree order through LDS, so the result does not depend on timing.  Block order: the
// column groups of one frequency run on one XCD (blocks are dealt to the eight XCDs in
// turn), so each XCD's L2 holds the X~ rows of its own frequencies only.
#define BG_W 8    // wavefronts per block
template <int XL, int WL>
struct BgShape {
  static constexpr int KG = 16 / (XL + WL);   // K steps per load group (two groups in flight)
};
template <int XL, int WL, bool MX>
__device__ __forceinline__ void bg_load(const void* __restrict__ wt, const float2* __restrict__ xt, int ks, int ks1,
                                        int q, int m, int b, int r, int n1, int n2, int nb, int j0,
                                        float2 (&xv)[BgShape<XL, WL>::KG][XL], float2 (&wv)[BgShape<XL, WL>::KG][WL]) {
  constexpr int KG = BgShape<XL, WL>::KG;
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    const int i = 4 * (ks + k) + q;
    const bool rowok = ks + k < ks1 && i < n1;
#pragma unroll
    for (int a = 0; a < XL; ++a) {
      const int s = 16 * a + m;
      xv[k][a] = ld_or(xt, ((size_t)b * r + s) * n1 + i, rowok && s < r, make_float2(0.f, 0.f));
    }
#pragma unroll
    for (int u = 0; u < WL; ++u) {
      const int j = j0 + 16 * u + m;
      const size_t idx = ((size_t)i * nb + b) * n2 + j;
      if constexpr (MX) wv[k][u] = unpack_bf16x2(ld_or((const uint32_t*)wt, idx, rowok && j < n2, 0u));
      else wv[k][u] = ld_or((const float2*)wt, idx, rowok && j < n2, make_float2(0.f, 0.f));
    }
  }
}

template <int XL, int WL>
__device__ __forceinline__ void bg_mfma(const float2 (&xv)[BgShape<XL, WL>::KG][XL],
                                        const float2 (&wv)[BgShape<XL, WL>::KG][WL], int cnt,
                                        v4d (&acc)[2 * XL][2 * WL]) {
  constexpr int KG = BgShape<XL, WL>::KG;
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    if (k < cnt) {   // the same in the whole wavefront
#pragma unroll
      for (int a = 0; a < 2 * XL; ++a) {
        const double av = (double)(a < XL ? xv[k][a].x : xv[k][a - XL].y);
#pragma unroll
        for (int u = 0; u < 2 * WL; ++u) {
          const double bv = (double)(u < WL ? wv[k][u].x : wv[k][u - WL].y);
          acc[a][u] = mfma4d(av, bv, acc[a][u]);
        }
      }
    }
  }
}

template <int XL, int WL, bool MX>   // r <= 16 XL, 16 WL complex columns per block, MX: W~ in BF16
__global__ void __launch_bounds__(64 * BG_W) __attribute__((amdgpu_waves_per_eu(XL + WL <= 2 ? 4 : 2))) k_bgemm(const void* __restrict__ wt, const float2* __restrict__ xt,
                                                      double2* __restrict__ bout, int n1, int n2, int r, int nb,
                                                      int ncg) {
  constexpr int KG = BgShape<XL, WL>::KG;
  extern __shared__ __align__(16) double2 bred[];   // [BG_W / 2][XL][WL][4][64]
  // XCD-aware order: block id -> (frequency, column group)
  const int nblk = (int)gridDim.x, id = (int)blockIdx.x, x = id & 7, qd = nblk >> 3, rem = nblk & 7;
  const int lid = x * qd + min(x, rem) + (id >> 3);
  const int b = lid / ncg, cg = lid % ncg, j0 = 16 * WL * cg;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, m = lane & 15, q = lane >> 4;
  const int nks = (n1 + 3) >> 2, per = (nks + BG_W - 1) / BG_W;
  const int ks0 = min(nks, w * per), ks1 = min(nks, ks0 + per);
  v4d acc[2 * XL][2 * WL];
#pragma unroll
  for (int a = 0; a < 2 * XL; ++a)
#pragma unroll
    for (int u = 0; u < 2 * WL; ++u) acc[a][u] = v4d{0.0, 0.0, 0.0, 0.0};
  float2 xa[KG][XL], wa[KG][WL], xb[KG][XL], wb[KG][WL];
  bg_load<XL, WL, MX>(wt, xt, ks0, ks1, q, m, b, r, n1, n2, nb, j0, xa, wa);
  for (int ks = ks0; ks < ks1; ks += 2 * KG) {
    if (ks + KG < ks1) bg_load<XL, WL, MX>(wt, xt, ks + KG, ks1, q, m, b, r, n1, n2, nb, j0, xb, wb);
    bg_mfma<XL, WL>(xa, wa, ks1 - ks, acc);
    if (ks + KG >= ks1) break;
    if (ks + 2 * KG < ks1) bg_load<XL, WL, MX>(wt, xt, ks + 2 * KG, ks1, q, m, b, r, n1, n2, nb, j0, xa, wa);
    bg_mfma<XL, WL>(xb, wb, ks1 - ks - KG, acc);
  }
  // complex results of this wavefront: element t of lane (q, m) is row q + 4 t, column m of
  // each tile, i.e. s = 16 a + q + 4 t, j = j0 + 16 u + m
  double2 cz[XL][WL][4];
#pragma unroll
  for (int a = 0; a < XL; ++a)
#pragma unroll
    for (int u = 0; u < WL; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        cz[a][u][t] = make_double2(acc[a][u][t] + acc[XL + a][WL + u][t], acc[a][WL + u][t] - acc[XL + a][u][t]);
  // fixed-order tree over the wavefronts: w += w + h for h = BG_W / 2, ..., 1
#pragma unroll
  for (int h = BG_W / 2; h >= 1; h >>= 1) {
    if (w >= h && w < 2 * h) {
#pragma unroll
      for (int a = 0; a < XL; ++a)
#pragma unroll
        for (int u = 0; u < WL; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t) bred[((((w - h) * XL + a) * WL + u) * 4 + t) * 64 + lane] = cz[a][u][t];
    }
    __syncthreads();
    if (w < h) {
#pragma unroll
      for (int a = 0; a < XL; ++a)
#pragma unroll
        for (int u = 0; u < WL; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double2 o = bred[(((w * XL + a) * WL + u) * 4 + t) * 64 + lane];
            cz[a][u][t].x += o.x;
            cz[a][u][t].y += o.y;
          }
    }
    __syncthreads();
  }
  if (w != 0) return;
#pragma unroll
  for (int a = 0; a < XL; ++a)
#pragma unroll
    for (int u = 0; u < WL; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int s = 16 * a + q + 4 * t, j = j0 + 16 * u + m;
        if (s < r && j < n2) bout[((size_t)b * r + s) * n2 + j] = cz[a][u][t];
      }
}

size_t bgemm_lds_bytes(int r, int bcg) {
  const int xl = r <= 16 ? 1 : 2, wl = bcg / 16;
  return (size_t)(BG_W / 2) * xl * wl * 4 * 64 * sizeof(double2);
}

bool bgemm_cols_valid(int r, int bcg) { return (bcg == 16 || bcg == 32) && r <= 32; }

void bgemm_set_attr() {}   // at most 64 KB of LDS per block

// X~^* W~ -> bpart [nb][r][n2] (G_X: launch_gramx).
void launch_bgemm(const Plan& p) {
  const int ncg = (p.n2 + p.bcg - 1) / p.bcg;
  const int grid = ncg * p.nb;
  const size_t lds = bgemm_lds_bytes(p.r, p.bcg);
#define TCTF_BGEMM(XL, WL)                                                                                       \
  do {                                                                                                           \
    if (p.mixed) k_bgemm<XL, WL, true><<<grid, 64 * BG_W, lds, p.stream>>>(p.wt, p.xt, p.bpart, p.n1, p.n2, p.r, p.nb, ncg);  \
    else k_bgemm<XL, WL, false><<<grid, 64 * BG_W, lds, p.stream>>>(p.wt, p.xt, p.bpart, p.n1, p.n2, p.r, p.nb, ncg); \
  } while (0)
  const bool wide = p.bcg == 32;
  if (p.r <= 16) {
    if (wide) TCTF_BGEMM(1, 2);
    else TCTF_BGEMM(1, 1);
  } else {
    if (wide) TCTF_BGEMM(2, 2);
    else TCTF_BGEMM(2, 1);
  }
#undef TCTF_BGEMM
}

}  // namespace tctf

// Per-frequency solves of one iteration.
//
// k_hsolve: X~_b = H_rho1^{-1} R_b column by column (first line of eq. (updataXYW1) after
//   k_agemm formed R_b = eta A_b G_Y^+ + H_rho1 X~_b (I - eta P_Y)).  H_rho1 = I + rho1 H^T H
//   is a constant SPD tridiagonal matrix (eq. (KKTcondition)); its Thomas coefficients
//   come from the setup table.  One wavefront solves one real column: each lane runs the
//   two first-order recurrences over a contiguous chunk, and the chunks are joined by a
//   log-depth scan of affine maps across the wavefront.
//
// k_ystep: the Y-update (second line of eq. (updataXYW1)) over column blocks of each
//   frequency: Y~ <- (I - eta P_X) Y~ + eta G_X^+ X~^* W~ with P_X = G_X^+ G_X, where
//   G_X = X~^* H_rho1 X~ = X~^* X~ + rho1 (H X~)^*(H X~) and G_X^+ come from the X~^* W~
//   launch; then each block's partial of the Gram of the new Y~.  FP64 arithmetic.
// k_pinvy: G_Y from those partials, the Fourier-domain H term of the objective, the
//   pseudo-inverse of G_Y and I - eta P_Y for the next X-update (the same work rides along
//   the Z~ product in the iteration).
#include "kernels.h"
#include "pinv.h"

namespace tctf {

__global__ void __launch_bounds__(64) k_hsolve(const float2* __restrict__ rhs, const float* __restrict__ htab,
                                               float2* __restrict__ xt, int n1, int r, int n3) {
  extern __shared__ float col[];
  const int part = blockIdx.x & 1, s = (blockIdx.x >> 1) % r, b = (blockIdx.x >> 1) / r;
  const int lane = threadIdx.x;
  float* out = (float*)xt + 2 * ((size_t)b * r + s) * n1 + part;
  if (part == 1 && bin_is_real(b, n3)) {
    for (int i = lane; i < n1; i += 64) out[2 * (size_t)i] = 0.0f;
    return;
  }
  const float* in = (const float*)rhs + 2 * ((size_t)b * r + s) * n1 + part;
  for (int i = lane; i < n1; i += 64) col[i] = in[2 * (size_t)i];
  __syncthreads();
  const float* lf = htab;            // rho1 / alpha_{i-1}
  const float* ia = htab + n1;       // 1 / alpha_i
  const float* bk = htab + 2 * n1;   // rho1 / alpha_i
  const int L = (n1 + 63) / 64, st = min(n1, lane * L), en = min(n1, st + L);
  // forward: y_i = t_i + l_i y_{i-1}
  float a = 1.0f, c = 0.0f;
  for (int i = st; i < en; ++i) {
    c = fmaf(lf[i], c, col[i]);
    a *= lf[i];
    col[i] = c;
  }
  for (int d = 1; d < 64; d <<= 1) {
    const float a2 = __shfl_up(a, d), c2 = __shfl_up(c, d);
    if (lane >= d) { c = fmaf(a, c2, c); a *= a2; }
  }
  float yin = __shfl_up(c, 1);
  if (lane == 0) yin = 0.0f;
  float pr = 1.0f;
  for (int i = st; i < en; ++i) {
    pr *= lf[i];
    col[i] = fmaf(pr, yin, col[i]);
  }
  // backward: x_i = y_i / alpha_i + (rho1 / alpha_i) x_{i+1}
  a = 1.0f;
  c = 0.0f;
  for (int i = en - 1; i >= st; --i) {
    c = fmaf(bk[i], c, ia[i] * col[i]);
    a *= bk[i];
    col[i] = c;
  }
  for (int d = 1; d < 64; d <<= 1) {
    const float a2 = __shfl_down(a, d), c2 = __shfl_down(c, d);
    if (lane + d < 64) { c = fmaf(a, c2, c); a *= a2; }
  }
  float xnext = __shfl_down(c, 1);
  if (lane == 63) xnext = 0.0f;
  pr = 1.0f;
  for (int i = en - 1; i >= st; --i) {
    pr *= bk[i];
    col[i] = fmaf(pr, xnext, col[i]);
  }
  __syncthreads();
  for (int i = lane; i < n1; i += 64) out[2 * (size_t)i] = col[i];
}

// The same solve with one wavefront per complex column (H_rho1 is real, so the real and
// imaginary parts share every coefficient) and everything in registers: lane l holds rows
// [l L, l L + L) of the column and their coefficients, L = ceil(n1 / 64) <= HS_L.  All loads
// of a lane are issued before the recurrences.
#define HS_L 16
__global__ void __launch_bounds__(64) k_hsolve_reg(const float2* __restrict__ rhs, const float* __restrict__ htab,
                                                   float2* __restrict__ xt, int n1, int r, int n3) {
  const int c = blockIdx.x, lane = threadIdx.x;   // complex column c = b r + s
  const int b = c / r;
  const float2* in = rhs + (size_t)c * n1;
  float2* out = xt + (size_t)c * n1;
  const int L = (n1 + 63) / 64, st = min(n1, lane * L), en = min(n1, st + L);
  float2 v[HS_L];
  float lf[HS_L], ia[HS_L], bk[HS_L];
#pragma unroll
  for (int u = 0; u < HS_L; ++u) {
    const int i = st + u;
    const bool ok = i < en;
    v[u] = ok ? in[i] : make_float2(0.f, 0.f);
    lf[u] = ok ? htab[i] : 1.0f;           // rho1 / alpha_{i-1}
    ia[u] = ok ? htab[n1 + i] : 0.0f;      // 1 / alpha_i
    bk[u] = ok ? htab[2 * n1 + i] : 1.0f;  // rho1 / alpha_i
  }
  // forward: y_i = t_i + l_i y_{i-1}
  float a = 1.0f, cr = 0.0f, ci = 0.0f;
#pragma unroll
  for (int u = 0; u < HS_L; ++u) {
    if (st + u < en) {
      cr = fmaf(lf[u], cr, v[u].x);
      ci = fmaf(lf[u], ci, v[u].y);
      a *= lf[u];
      v[u] = make_float2(cr, ci);
    }
  }
  for (int d = 1; d < 64; d <<= 1) {
    const float a2 = __shfl_up(a, d), r2 = __shfl_up(cr, d), i2 = __shfl_up(ci, d);
    if (lane >= d) {
      cr = fmaf(a, r2, cr);
      ci = fmaf(a, i2, ci);
      a *= a2;
    }
  }
  float yr = __shfl_up(cr, 1), yi = __shfl_up(ci, 1);
  if (lane == 0) yr = yi = 0.0f;
  float pr = 1.0f;
#pragma unroll
  for (int u = 0; u < HS_L; ++u) {
    if (st + u < en) {
      pr *= lf[u];
      v[u] = make_float2(fmaf(pr, yr, v[u].x), fmaf(pr, yi, v[u].y));
    }
  }
  // backward: x_i = y_i / alpha_i + (rho1 / alpha_i) x_{i+1}
  a = 1.0f;
  cr = ci = 0.0f;
#pragma unroll
  for (int u = HS_L - 1; u >= 0; --u) {
    if (st + u < en) {
      cr = fmaf(bk[u], cr, ia[u] * v[u].x);
      ci = fmaf(bk[u], ci, ia[u] * v[u].y);
      a *= bk[u];
      v[u] = make_float2(cr, ci);
    }
  }
  for (int d = 1; d < 64; d <<= 1) {
    const float a2 = __shfl_down(a, d), r2 = __shfl_down(cr, d), i2 = __shfl_down(ci, d);
    if (lane + d < 64) {
      cr = fmaf(a, r2, cr);
      ci = fmaf(a, i2, ci);
      a *= a2;
    }
  }
  float xr = __shfl_down(cr, 1), xi = __shfl_down(ci, 1);
  if (lane == 63) xr = xi = 0.0f;
  pr = 1.0f;
  const bool real_bin = bin_is_real(b, n3);
#pragma unroll
  for (int u = HS_L - 1; u >= 0; --u) {
    if (st + u < en) {
      pr *= bk[u];
      out[st + u] = make_float2(fmaf(pr, xr, v[u].x), real_bin ? 0.0f : fmaf(pr, xi, v[u].y));
    }
  }
}

void launch_hsolve(const Plan& p) {
  if (p.n1 <= 64 * HS_L) {
    k_hsolve_reg<<<p.nb * p.r, 64, 0, p.stream>>>(p.rhs, p.htab, p.xt, p.n1, p.r, p.n3);
    return;
  }
  const size_t lds = (size_t)p.n1 * sizeof(float);
  k_hsolve<<<p.nb * p.r * 2, 64, lds, p.stream>>>(p.rhs, p.htab, p.xt, p.n1, p.r, p.n3);
}

// Dynamic LDS layout of k_ystep: G_X^+ and q = I - eta P_X (r x r FP64 complex), then the
// column block of cw columns with an odd row stride cw | 1, so that the rows of one column
// fall in different LDS banks.
struct YLayout {
  size_t gp, q, bsum, yold, ynew, total;
};
__host__ __device__ inline YLayout ystep_layout(int r, int cw) {
  YLayout L;
  const size_t m = (size_t)r * r * sizeof(cd), ld = (size_t)(cw | 1);
  size_t o = 0;
  L.gp = o; o += m;
  L.q = o; o += m;
  L.bsum = o; o += (size_t)r * ld * sizeof(cd);       // columns of X~^* W~ (FP64)
  L.yold = o; o += (size_t)r * ld * sizeof(float2);   // the same columns of the old Y~
  L.ynew = o; o += (size_t)r * ld * sizeof(float2);   // and of the new (stored) Y~
  L.total = o;
  return L;
}

// Column blocks of the Y-step: enough blocks to cover the compute units, a multiple of 8
// columns each (at least 8), at most 512 / r (two elements per thread).
void ystep_split(int n2, int r, int nb, int* ny, int* cw) {
  const int want = (256 + nb - 1) / nb;
  int c = (n2 + want - 1) / want;
  c &= ~7;   // so that every block starts on a 64-byte boundary of a row of Y~
  if (c < 8) c = 8;
  if (c > 512 / r) c = 512 / r;
  if (c > n2) c = n2;
  *cw = c;
  *ny = (n2 + c - 1) / c;
}

// Block (column block jb, frequency b), 256 threads, r <= RM; G_X^+ and I - eta P_X come
// from the G_X launch (k_gramx_inv), X~^* W~ from k_bgemm.  Every load of the block is
// issued before any use: G_X^+ and q, the old columns and X~^* W~ on the block's columns.
// Then Y~ <- (I - eta P_X) Y~ + eta G_X^+ X~^* W~ (eq. (updataXYW1)) is formed on the
// block's columns in FP64 and stored in FP32, and the block's FP64 partial of G_Y = Y~ Y~^*
// from the stored values.  init: only the partial of G_Y.
template <int RM>
__global__ void __launch_bounds__(256) k_ystep(float2* __restrict__ yt, const double2* __restrict__ bpart,
                                               const cd* __restrict__ gxp, const cd* __restrict__ qx,
                                               const int* __restrict__ qx_zero, cd* __restrict__ gyq, int n2,
                                               int r, int n3, int cw, int ny, double eta, int init) {
  constexpr int GPT = (RM * RM + 255) / 256;   // r x r entries per thread
  extern __shared__ __align__(16) unsigned char sm[];
  const YLayout L = ystep_layout(r, cw);
  const int jb = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, rr = r * r;
  cd* gp = (cd*)(sm + L.gp);
  cd* q = (cd*)(sm + L.q);
  cd* bsum = (cd*)(sm + L.bsum);
  float2* yold = (float2*)(sm + L.yold);
  float2* ynew = (float2*)(sm + L.ynew);
  const int j0 = jb * cw, nj = min(cw, n2 - j0), nel = r * nj, ld = cw | 1;
  const bool real_bin = bin_is_real(b, n3);
  const bool qzero = init || qx_zero[b] != 0;
  const float2 z2 = make_float2(0.f, 0.f);
  const cd zc = cd_make(0.0, 0.0);

  cd g4[GPT], q4[GPT];
#pragma unroll
  for (int k = 0; k < GPT; ++k) {
    const int e = tid + 256 * k;
    g4[k] = ld_or(gxp, (size_t)b * rr + e, !init && e < rr, zc);
    q4[k] = ld_or(qx, (size_t)b * rr + e, !qzero && e < rr, zc);
  }
  const double2 zd = make_double2(0.0, 0.0);
  float2 y[2];
  cd acc[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + 256 * u, t = e / nj, jj = e % nj;
    const size_t at = ((size_t)b * r + t) * n2 + j0 + jj;
    y[u] = ld_or(yt, at, e < nel, z2);
    const double2 v = ld_or(bpart, at, !init && e < nel, zd);
    acc[u] = cd_make(v.x, v.y);
  }
#pragma unroll
  for (int k = 0; k < GPT; ++k) {
    const int e = tid + 256 * k;
    if (e < rr) {
      gp[e] = g4[k];
      q[e] = q4[k];
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + 256 * u;
    if (e < nel) {
      const int t = e / nj, jj = e % nj;
      yold[t * ld + jj] = y[u];
      bsum[t * ld + jj] = acc[u];
    }
  }
  __syncthreads();
  if (!init) {
    for (int e = tid; e < nel; e += 256) {
      const int s = e / nj, jj = e % nj;
      cd a1 = zc, a2 = zc;
#pragma unroll 4
      for (int t = 0; t < r; ++t) cd_fma(a2, gp[s * r + t], bsum[t * ld + jj]);
      if (!qzero) {
#pragma unroll 4
        for (int t = 0; t < r; ++t) {
          const float2 yv = yold[t * ld + jj];
          cd_fma(a1, q[s * r + t], cd_make(yv.x, yv.y));
        }
      }
      a1 = cd_add(a1, cd_scale(a2, eta));
      const float2 o = make_float2((float)a1.re, real_bin ? 0.0f : (float)a1.im);
      ynew[s * ld + jj] = o;
      yt[((size_t)b * r + s) * n2 + j0 + jj] = o;
    }
    __syncthreads();
  }
  // partial G_Y(s, t) = sum over the block's columns of Y~(s, j) conj(Y~(t, j)), stored values
  const float2* yb = init ? yold : ynew;
  for (int e = tid; e < rr; e += 256) {
    const int s = e / r, t = e % r;
    cd g = zc;
#pragma unroll 4
    for (int jj = 0; jj < nj; ++jj) {
      const float2 a = yb[s * ld + jj], c = yb[t * ld + jj];
      cd_fma(g, cd_make(a.x, a.y), cd_make(c.x, -c.y));
    }
    gyq[((size_t)b * ny + jb) * rr + e] = g;
  }
}

// Per frequency: G_Y^+ and I - eta P_Y (pinvy_block).  In the iteration this work rides
// along the Z~ product (k_zgemm); this kernel serves create and stage timing.
__global__ void __launch_bounds__(256) k_pinvy(PinvyArgs pa) {
  extern __shared__ __align__(16) unsigned char psm[];
  pinvy_block(blockIdx.x, pa, psm);
}

void pinvy_set_attr(int r) {
  if (pinvy_lds_bytes(r) > 65536)
    (void)hipFuncSetAttribute((const void*)k_pinvy, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pinvy_lds_bytes(r));
}

void launch_pinvy(const Plan& p, hipStream_t stream) {
  k_pinvy<<<p.nb, 256, pinvy_lds_bytes(p.r), stream>>>(pinvy_args(p));
}

size_t ystep_lds_bytes(int r, int cw) { return ystep_layout(r, cw).total; }

void ystep_set_attr(size_t lds) {
  if (lds > 65536) {
    (void)hipFuncSetAttribute((const void*)k_ystep<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_ystep<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_ystep<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
}

void launch_ystep(const Plan& p, int init) {
  const size_t lds = ystep_layout(p.r, p.ycw).total;
  const dim3 grid(p.ny, p.nb);
#define TCTF_YSTEP(RM)                                                                                       \
  k_ystep<RM><<<grid, 256, lds, p.stream>>>(p.yt, p.bpart, p.gxp, p.qx, p.qx_zero, p.gym, p.n2, p.r, p.n3,    \
                                            p.ycw, p.ny, p.eta, init)
  if (p.r <= 8) TCTF_YSTEP(8);
  else if (p.r <= 16) TCTF_YSTEP(16);
  else TCTF_YSTEP(32);
#undef TCTF_YSTEP
}

}  // namespace tctf

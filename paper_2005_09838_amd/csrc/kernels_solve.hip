// Per-frequency solves of one iteration.
//
// k_hsolve: X~_b = H_rho1^{-1} R_b column by column (first line of eq. (updataXYW1) after
//   k_agemm formed R_b = eta A_b G_Y^+ + H_rho1 X~_b (I - eta P_Y)).  H_rho1 = I + rho1 H^T H
//   is a constant SPD tridiagonal matrix (eq. (KKTcondition)); its Thomas coefficients
//   come from the setup table.  One wavefront solves one real column: each lane runs the
//   two first-order recurrences over a contiguous chunk, and the chunks are joined by a
//   log-depth scan of affine maps across the wavefront.
//
// k_ystep: per frequency, the Y-update (second line of eq. (updataXYW1)):
//   G_X = X~^* H_rho1 X~ = X~^* X~ + rho1 (H X~)^*(H X~),  Y~ <- (I - eta P_X) Y~ + eta G_X^+ X~^* W~,
//   with P_X = G_X^+ G_X; then the Gram of the new Y~ and the Fourier-domain H term of the
//   objective.  FP64 throughout.
// k_pinvy: the pseudo-inverse of that Gram and I - eta P_Y for the next X-update.
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

// Dynamic LDS layout of k_ystep (r x r FP64 complex matrices unless noted); jb columns of
// Y~ are handled per block step.
#define YS_THREADS 512
#define YS_LDS_BUDGET (150 * 1024)
struct YLayout {
  size_t gx, dm, gp, q, gy, gpart, work, vec, colk, rowk, rot, red, bsum, yold, ynew, total;
};
__host__ __device__ inline YLayout ystep_layout(int r, int jb) {
  YLayout L;
  const size_t m = (size_t)r * r * sizeof(cd);
  const size_t npart = (size_t)(r * r < YS_THREADS ? YS_THREADS : r * r);
  size_t o = 0;
  L.gx = o; o += m;
  L.dm = o; o += m;
  L.gp = o; o += m;
  L.q = o; o += m;
  L.gy = o; o += m;
  L.gpart = o; o += npart * sizeof(cd);                 // partial Gram sums of one block step
  L.work = o; o += m;
  L.vec = o; o += m;
  L.colk = o; o += r * sizeof(cd);
  L.rowk = o; o += r * sizeof(cd);
  L.rot = o; o += 96 * sizeof(double);
  L.red = o; o += 16 * sizeof(double);
  // the column blocks below have a row stride of (jb | 1): odd, so the rows of one column
  // fall in different LDS banks
  const size_t ld = (size_t)(jb | 1);
  L.bsum = o; o += (size_t)r * ld * sizeof(cd);         // columns of X~^* W~ (FP64)
  L.yold = o; o += (size_t)r * ld * sizeof(float2);     // the same columns of the old Y~
  L.ynew = o; o += (size_t)r * ld * sizeof(float2);     // and of the new (stored) Y~
  L.total = o;
  return L;
}

// Columns per block step: all of n2 when they fit the LDS budget, else as many as fit.
static int ystep_jb(int r, int n2) {
  const size_t fixed = ystep_layout(r, 0).total;
  const size_t per = (size_t)r * (sizeof(cd) + 2 * sizeof(float2));
  int jb = (int)((YS_LDS_BUDGET - fixed) / per) - 1;
  if (jb > n2) jb = n2;
  if (jb < 1) jb = 1;
  return jb;
}

// One block per frequency.  Y~ is visited in blocks of jb columns: the chunk partials of
// X~^* W~ and the old columns are loaded together (independent loads, summed in a fixed
// order), the new columns are formed in FP64 and stored in FP32, and their FP64 Gram is
// accumulated from the stored values, so Y~ is read once and written once.  When a
// pseudo-inverse keeps every eigenvalue and eta = 1, I - eta P is exactly 0 and is not
// formed.
__global__ void __launch_bounds__(YS_THREADS) k_ystep(float2* __restrict__ yt, const float2* __restrict__ bpart,
                                                      const cd* __restrict__ spart, const cd* __restrict__ dpart,
                                                      cd* __restrict__ gy_out, double* __restrict__ bin_obj,
                                                      int n2, int r, int n3, int nchunk, int jb, double eta,
                                                      double rho1, int force_eigen, int init) {
  extern __shared__ __align__(16) unsigned char sm[];
  const YLayout L = ystep_layout(r, jb);
  cd* gx = (cd*)(sm + L.gx);
  cd* dm = (cd*)(sm + L.dm);
  cd* gp = (cd*)(sm + L.gp);
  cd* q = (cd*)(sm + L.q);
  cd* gy = (cd*)(sm + L.gy);
  cd* gpart = (cd*)(sm + L.gpart);
  PinvScratch ps;
  ps.work = (cd*)(sm + L.work);
  ps.vec = (cd*)(sm + L.vec);
  ps.colk = (cd*)(sm + L.colk);
  ps.rowk = (cd*)(sm + L.rowk);
  ps.rot = (double*)(sm + L.rot);
  ps.red = (double*)(sm + L.red);
  cd* bsum = (cd*)(sm + L.bsum);
  float2* yold = (float2*)(sm + L.yold);
  float2* ynew = (float2*)(sm + L.ynew);
  const int b = blockIdx.x, tid = threadIdx.x, rr = r * r, nt = YS_THREADS;
  const bool real_bin = bin_is_real(b, n3);
  const int ld = jb | 1;

  // One batch of column-block elements per thread (four in flight): the old Y~ entries and
  // the sums of the X~^* W~ chunk partials (fixed order).
  float2 y[4];
  cd acc[4];
  auto load_batch = [&](int j0, int nj, int e0) {
    const int nel = r * nj;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + tid + u * nt;
      y[u] = make_float2(0.f, 0.f);
      acc[u] = cd_make(0.0, 0.0);
      if (e < nel) {
        const int t = e / nj, jj = e % nj;
        y[u] = yt[((size_t)b * r + t) * n2 + j0 + jj];
        if (!init) {
          const float2* bp = bpart + ((size_t)b * nchunk * r + t) * n2 + j0 + jj;
#pragma unroll 8
          for (int c = 0; c < nchunk; ++c) {
            const float2 v = bp[(size_t)c * r * n2];
            acc[u].re += v.x;
            acc[u].im += v.y;
          }
        }
      }
    }
  };
  auto store_batch = [&](int nj, int e0) {
    const int nel = r * nj;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + tid + u * nt;
      if (e < nel) {
        const int t = e / nj, jj = e % nj;
        yold[t * ld + jj] = y[u];
        bsum[t * ld + jj] = acc[u];
      }
    }
  };
  // when the first column block is one batch, its loads are issued before the G_X work
  const int nj0 = min(jb, n2);
  const bool early = r * nj0 <= 4 * nt;
  if (early) load_batch(0, nj0, 0);

  // G_X = S + rho1 D from the chunk partials (fixed order)
  for (int e = tid; e < rr; e += nt) {
    cd sacc = cd_make(0.0, 0.0), dacc = cd_make(0.0, 0.0);
#pragma unroll 4
    for (int c = 0; c < nchunk; ++c) {
      sacc = cd_add(sacc, spart[((size_t)b * nchunk + c) * rr + e]);
      dacc = cd_add(dacc, dpart[((size_t)b * nchunk + c) * rr + e]);
    }
    dm[e] = dacc;
    gx[e] = cd_add(sacc, cd_scale(dacc, rho1));
    gy[e] = cd_make(0.0, 0.0);
  }
  __syncthreads();

  bool qzero = true;
  if (!init) {
    const int full = pinv_herm(gx, gp, r, force_eigen, ps);
    qzero = full && eta == 1.0;
    if (!qzero) {   // q = I - eta G_X^+ G_X
      for (int e = tid; e < rr; e += nt) {
        const int s = e / r, t = e % r;
        cd acc = cd_make(0.0, 0.0);
        for (int u = 0; u < r; ++u) cd_fma(acc, gp[s * r + u], gx[u * r + t]);
        q[e] = cd_make((s == t ? 1.0 : 0.0) - eta * acc.re, -eta * acc.im);
      }
      __syncthreads();
    }
  }
  const int np = rr < nt ? nt / rr : 1;   // partial sums per Gram entry
  for (int j0 = 0; j0 < n2; j0 += jb) {
    const int nj = min(jb, n2 - j0), nel = r * nj;
    for (int e0 = 0; e0 < nel; e0 += 4 * nt) {
      if (!(early && j0 == 0)) load_batch(j0, nj, e0);
      store_batch(nj, e0);
    }
    __syncthreads();
    if (!init) {
      // Y~ <- q Y~ + eta G_X^+ B on these columns
      for (int e = tid; e < nel; e += nt) {
        const int s = e / nj, jj = e % nj;
        cd acc = cd_make(0.0, 0.0), acc2 = cd_make(0.0, 0.0);
#pragma unroll 4
        for (int t = 0; t < r; ++t) cd_fma(acc2, gp[s * r + t], bsum[t * ld + jj]);
        if (!qzero) {
#pragma unroll 4
          for (int t = 0; t < r; ++t) {
            const float2 y = yold[t * ld + jj];
            cd_fma(acc, q[s * r + t], cd_make(y.x, y.y));
          }
        }
        acc = cd_add(acc, cd_scale(acc2, eta));
        const float2 v = make_float2((float)acc.re, real_bin ? 0.0f : (float)acc.im);
        ynew[s * ld + jj] = v;
        yt[((size_t)b * r + s) * n2 + j0 + jj] = v;
      }
      __syncthreads();
    }
    // G_Y += (stored columns) (stored columns)^*, np interleaved partial sums per entry
    const float2* yb = init ? yold : ynew;
    for (int e2 = tid; e2 < rr * np; e2 += nt) {
      const int e = e2 % rr, part = e2 / rr, s = e / r, t = e % r;
      cd acc = cd_make(0.0, 0.0);
#pragma unroll 4
      for (int jj = part; jj < nj; jj += np) {
        const float2 u = yb[s * ld + jj], v = yb[t * ld + jj];
        cd_fma(acc, cd_make(u.x, u.y), cd_make(v.x, -v.y));
      }
      gpart[e2] = acc;
    }
    __syncthreads();
    for (int e = tid; e < rr; e += nt) {
      cd acc = gy[e];
      for (int part = 0; part < np; ++part) acc = cd_add(acc, gpart[part * rr + e]);
      gy[e] = acc;
    }
    __syncthreads();
  }

  // G_Y for k_pinvy, and c_b tr(D G_Y): the rho1 term of eq. (fun-XYW) for this frequency
  double tr = 0.0;
  for (int e = tid; e < rr; e += nt) {
    const int s = e / r, t = e % r;
    gy_out[(size_t)b * rr + e] = gy[e];
    const cd d = dm[s * r + t], g = gy[t * r + s];
    tr += d.re * g.re - d.im * g.im;
  }
  tr = block_sum_d(tr, ps.red);
  if (tid == 0) bin_obj[b] = bin_weight(b, n3) * tr;
}

// Per frequency: G_Y^+ and I - eta P_Y (pinvy_block).  In the iteration this work rides
// along the Z~ product (k_zgemm); this kernel serves create and stage timing.
__global__ void __launch_bounds__(256) k_pinvy(const cd* __restrict__ gy_in, cd* __restrict__ gyp_out,
                                               cd* __restrict__ qy_out, int* __restrict__ qy_zero, int r,
                                               double eta, int force_eigen) {
  extern __shared__ __align__(16) unsigned char psm[];
  pinvy_block(blockIdx.x, gy_in, gyp_out, qy_out, qy_zero, r, eta, force_eigen, psm);
}

void pinvy_set_attr(int r) {
  if (pinvy_lds_bytes(r) > 65536)
    (void)hipFuncSetAttribute((const void*)k_pinvy, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pinvy_lds_bytes(r));
}

void launch_pinvy(const Plan& p, hipStream_t stream) {
  k_pinvy<<<p.nb, 256, pinvy_lds_bytes(p.r), stream>>>(p.gym, p.gyp, p.qy, p.qy_zero, p.r, p.eta, p.force_eigen);
}

size_t ystep_lds_bytes(int r, int n2) { return ystep_layout(r, ystep_jb(r, n2)).total; }

void ystep_set_attr(size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_ystep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

void launch_ystep(const Plan& p, int init) {
  const int jb = ystep_jb(p.r, p.n2);
  const size_t lds = ystep_layout(p.r, jb).total;
  k_ystep<<<p.nb, YS_THREADS, lds, p.stream>>>(p.yt, p.bpart, p.spart, p.dpart, p.gym, p.bin_obj, p.n2, p.r,
                                               p.n3, p.nchunk, jb, p.eta, p.rho1, p.force_eigen, init);
}

}  // namespace tctf

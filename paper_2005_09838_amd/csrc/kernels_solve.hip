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
//   with P_X = G_X^+ G_X; then the Gram of the new Y~, its pseudo-inverse and I - eta P_Y
//   for the next X-update, and the Fourier-domain H term of the objective.  FP64 throughout.
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

void launch_hsolve(const Plan& p) {
  const size_t lds = (size_t)p.n1 * sizeof(float);
  k_hsolve<<<p.nb * p.r * 2, 64, lds, p.stream>>>(p.rhs, p.htab, p.xt, p.n1, p.r, p.n3);
}

// Dynamic LDS layout of k_ystep (r x r FP64 complex matrices unless noted).
struct YLayout {
  size_t gx, dm, gp, q, work, vec, colk, rowk, rot, red, blk, yb, total;
};
__host__ __device__ inline YLayout ystep_layout(int r) {
  YLayout L;
  const size_t m = (size_t)r * r * sizeof(cd);
  size_t o = 0;
  L.gx = o; o += m;
  L.dm = o; o += m;
  L.gp = o; o += m;
  L.q = o; o += m;
  L.work = o; o += m;
  L.vec = o; o += m;
  L.colk = o; o += r * sizeof(cd);
  L.rowk = o; o += r * sizeof(cd);
  L.rot = o; o += 96 * sizeof(double);
  L.red = o; o += 16 * sizeof(double);
  L.blk = o; o += (size_t)r * 32 * sizeof(cd);   // column block of X~^* W~ (FP64)
  L.yb = o; o += (size_t)r * 32 * sizeof(cd);    // column block of the old Y~
  L.total = o;
  return L;
}

__global__ void __launch_bounds__(256) k_ystep(float2* __restrict__ yt, const float2* __restrict__ bpart,
                                               const cd* __restrict__ spart, const cd* __restrict__ dpart,
                                               cd* __restrict__ gyp_out, cd* __restrict__ qy_out,
                                               int* __restrict__ qy_zero, double* __restrict__ bin_obj,
                                               int n2, int r, int n3, int nchunk, double eta, double rho1,
                                               int force_eigen, int init) {
  extern __shared__ __align__(16) unsigned char sm[];
  const YLayout L = ystep_layout(r);
  cd* gx = (cd*)(sm + L.gx);
  cd* dm = (cd*)(sm + L.dm);
  cd* gp = (cd*)(sm + L.gp);
  cd* q = (cd*)(sm + L.q);
  PinvScratch ps;
  ps.work = (cd*)(sm + L.work);
  ps.vec = (cd*)(sm + L.vec);
  ps.colk = (cd*)(sm + L.colk);
  ps.rowk = (cd*)(sm + L.rowk);
  ps.rot = (double*)(sm + L.rot);
  ps.red = (double*)(sm + L.red);
  cd* blk = (cd*)(sm + L.blk);
  cd* yb = (cd*)(sm + L.yb);
  const int b = blockIdx.x, tid = threadIdx.x, rr = r * r;
  const bool real_bin = bin_is_real(b, n3);

  // G_X = S + rho1 D from the chunk partials (fixed order)
  for (int e = tid; e < rr; e += 256) {
    cd sacc = cd_make(0.0, 0.0), dacc = cd_make(0.0, 0.0);
    for (int c = 0; c < nchunk; ++c) {
      sacc = cd_add(sacc, spart[((size_t)b * nchunk + c) * rr + e]);
      dacc = cd_add(dacc, dpart[((size_t)b * nchunk + c) * rr + e]);
    }
    dm[e] = dacc;
    gx[e] = cd_add(sacc, cd_scale(dacc, rho1));
  }
  __syncthreads();

  if (!init) {
    const int full = pinv_herm(gx, gp, r, force_eigen, ps);
    const bool qzero = full && eta == 1.0;
    // q = I - eta G_X^+ G_X
    for (int e = tid; e < rr; e += 256) {
      const int s = e / r, t = e % r;
      cd acc = cd_make(0.0, 0.0);
      for (int u = 0; u < r; ++u) cd_fma(acc, gp[s * r + u], gx[u * r + t]);
      q[e] = cd_make((s == t ? 1.0 : 0.0) - eta * acc.re, -eta * acc.im);
    }
    __syncthreads();
    // Y~ <- q Y~ + eta G_X^+ B, 32 columns at a time
    for (int j0 = 0; j0 < n2; j0 += 32) {
      const int nj = min(32, n2 - j0);
      for (int e = tid; e < r * 32; e += 256) {
        const int t = e >> 5, jj = e & 31;
        if (jj < nj) {
          cd acc = cd_make(0.0, 0.0);
          for (int c = 0; c < nchunk; ++c) {
            const float2 v = bpart[(((size_t)b * nchunk + c) * r + t) * n2 + j0 + jj];
            acc.re += v.x;
            acc.im += v.y;
          }
          blk[t * 32 + jj] = acc;
          const float2 y = yt[((size_t)b * r + t) * n2 + j0 + jj];
          yb[t * 32 + jj] = cd_make(y.x, y.y);
        }
      }
      __syncthreads();
      for (int e = tid; e < r * 32; e += 256) {
        const int s = e >> 5, jj = e & 31;
        if (jj < nj) {
          cd acc = cd_make(0.0, 0.0), acc2 = cd_make(0.0, 0.0);
          for (int t = 0; t < r; ++t) cd_fma(acc2, gp[s * r + t], blk[t * 32 + jj]);
          if (!qzero)
            for (int t = 0; t < r; ++t) cd_fma(acc, q[s * r + t], yb[t * 32 + jj]);
          acc = cd_add(acc, cd_scale(acc2, eta));
          yt[((size_t)b * r + s) * n2 + j0 + jj] = make_float2((float)acc.re, real_bin ? 0.0f : (float)acc.im);
        }
      }
      __syncthreads();
    }
  }

  // G_Y = Y~ Y~^* of the stored (FP32) Y~, its pseudo-inverse and q = I - eta G_Y G_Y^+
  for (int e = tid; e < rr; e += 256) {
    const int s = e / r, t = e % r;
    const float2* ys = yt + ((size_t)b * r + s) * n2;
    const float2* ytt = yt + ((size_t)b * r + t) * n2;
    cd acc = cd_make(0.0, 0.0);
    for (int j = 0; j < n2; ++j) {
      const float2 u = ys[j], v = ytt[j];
      cd_fma(acc, cd_make(u.x, u.y), cd_make(v.x, -v.y));
    }
    gx[e] = acc;
  }
  __syncthreads();
  const int fully = pinv_herm(gx, gp, r, force_eigen, ps);
  const bool qyz = fully && eta == 1.0;
  for (int e = tid; e < rr; e += 256) {
    const int s = e / r, t = e % r;
    cd acc = cd_make(0.0, 0.0);
    for (int u = 0; u < r; ++u) cd_fma(acc, gx[s * r + u], gp[u * r + t]);
    q[e] = cd_make((s == t ? 1.0 : 0.0) - eta * acc.re, -eta * acc.im);
    gyp_out[(size_t)b * rr + e] = gp[e];
  }
  __syncthreads();
  for (int e = tid; e < rr; e += 256) qy_out[(size_t)b * rr + e] = q[e];
  // c_b tr(D G_Y): the rho1 term of eq. (fun-XYW) for this frequency
  double tr = 0.0;
  for (int e = tid; e < rr; e += 256) {
    const int s = e / r, t = e % r;
    const cd d = dm[s * r + t], g = gx[t * r + s];
    tr += d.re * g.re - d.im * g.im;
  }
  tr = block_sum_d(tr, ps.red);
  if (tid == 0) {
    qy_zero[b] = qyz ? 1 : 0;
    bin_obj[b] = bin_weight(b, n3) * tr;
  }
}

size_t ystep_lds_bytes(int r) { return ystep_layout(r).total; }

void ystep_set_attr(size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_ystep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

void launch_ystep(const Plan& p, int init) {
  const size_t lds = ystep_lds_bytes(p.r);
  k_ystep<<<p.nb, 256, lds, p.stream>>>(p.yt, p.bpart, p.spart, p.dpart, p.gyp, p.qy, p.qy_zero, p.bin_obj,
                                        p.n2, p.r, p.n3, p.nchunk, p.eta, p.rho1, p.force_eigen, init);
}

}  // namespace tctf

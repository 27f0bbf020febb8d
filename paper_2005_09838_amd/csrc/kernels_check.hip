// Stationarity measures of Theorem ThKKT / eq. (AKKTstar) at the current iterate.
//   factor: sqrt(sum_k ||grad_X h_k||^2 + ||grad_Y h_k||^2) / (||W~|| (||X~|| + ||Y~||)),
//           with the gradients of eq. (hkXYDer) rewritten as
//           grad_X = H_rho1 X~ G_Y - W~ Y~^*,  grad_Y = G_X Y~ - X~^* W~   (G_Y = Y~Y~^*,
//           G_X = X~^* H_rho1 X~), summed over all n3 frequencies through the weights c_b;
//   w_kkt:  max over unobserved entries of |(W_k K_{mu rho2} - Z_k)_ij| / ||Z||_inf;
//   w_obs:  max over observed entries of |W - G|.
#include "kernels.h"

namespace tctf {

__global__ void __launch_bounds__(256) k_stat_bin(const float2* __restrict__ xt, const float2* __restrict__ yt,
                                                  const void* __restrict__ wt, const float2* __restrict__ a,
                                                  const double2* __restrict__ bpart, const cd* __restrict__ gxm,
                                                  double* __restrict__ out, int n1, int n2, int n3, int r,
                                                  int nb, double rho1, int mixed) {
  __shared__ cd gy[TCTF_RMAX * TCTF_RMAX];
  __shared__ cd gx[TCTF_RMAX * TCTF_RMAX];
  __shared__ double red[16];
  const int b = blockIdx.x, tid = threadIdx.x, rr = r * r;
  const float2* X = xt + (size_t)b * r * n1;
  const float2* Y = yt + (size_t)b * r * n2;
  for (int e = tid; e < rr; e += 256) {
    const int s = e / r, t = e % r;
    cd acc = cd_make(0.0, 0.0);
    for (int j = 0; j < n2; ++j) {
      const float2 u = Y[(size_t)s * n2 + j], v = Y[(size_t)t * n2 + j];
      cd_fma(acc, cd_make(u.x, u.y), cd_make(v.x, -v.y));
    }
    gy[e] = acc;
    gx[e] = gxm[(size_t)b * rr + e];
  }
  __syncthreads();
  double gyn = 0.0, gxn = 0.0, xn = 0.0, yn = 0.0, wn = 0.0;
  for (int e = tid; e < r * n2; e += 256) {   // grad_Y(s, j)
    const int s = e / n2, j = e % n2;
    cd v = cd_make(0.0, 0.0);
    for (int t = 0; t < r; ++t) {
      const float2 y = Y[(size_t)t * n2 + j];
      cd_fma(v, gx[s * r + t], cd_make(y.x, y.y));
    }
    const double2 bb = bpart[((size_t)b * r + s) * n2 + j];
    v.re -= bb.x;
    v.im -= bb.y;
    gyn += v.re * v.re + v.im * v.im;
    const float2 y = Y[(size_t)s * n2 + j];
    yn += (double)y.x * y.x + (double)y.y * y.y;
  }
  for (int e = tid; e < n1 * r; e += 256) {   // grad_X(i, s)
    const int s = e / n1, i = e % n1;
    const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
    cd v = cd_make(0.0, 0.0);
    for (int t = 0; t < r; ++t) {
      const float2 x0 = X[(size_t)t * n1 + i];
      cd hx = cd_scale(cd_make(x0.x, x0.y), 1.0 + rho1 * deg);
      if (i > 0) { const float2 xm = X[(size_t)t * n1 + i - 1]; hx = cd_sub(hx, cd_scale(cd_make(xm.x, xm.y), rho1)); }
      if (i + 1 < n1) { const float2 xp = X[(size_t)t * n1 + i + 1]; hx = cd_sub(hx, cd_scale(cd_make(xp.x, xp.y), rho1)); }
      cd_fma(v, hx, gy[t * r + s]);
    }
    const float2 av = a[((size_t)b * r + s) * n1 + i];
    v.re -= av.x;
    v.im -= av.y;
    gxn += v.re * v.re + v.im * v.im;
    const float2 x = X[(size_t)s * n1 + i];
    xn += (double)x.x * x.x + (double)x.y * x.y;
  }
  for (long e = tid; e < (long)n1 * n2; e += 256) {
    const long i = e / n2, j = e % n2;
    const size_t idx = ((size_t)i * nb + b) * n2 + j;
    const float2 w = mixed ? unpack_bf16x2(((const uint32_t*)wt)[idx]) : ((const float2*)wt)[idx];
    wn += (double)w.x * w.x + (double)w.y * w.y;
  }
  const double cw = bin_weight(b, n3);
  gxn = block_sum_d(gxn, red);
  gyn = block_sum_d(gyn, red);
  xn = block_sum_d(xn, red);
  yn = block_sum_d(yn, red);
  wn = block_sum_d(wn, red);
  if (tid == 0) {
    out[8 * b + 0] = cw * gxn;
    out[8 * b + 1] = cw * gyn;
    out[8 * b + 2] = cw * xn;
    out[8 * b + 3] = cw * yn;
    out[8 * b + 4] = cw * wn;
  }
}

__global__ void k_stat_final(const double* __restrict__ part, int nb, const double* __restrict__ kkt, int n1,
                             double* __restrict__ out) {
  __shared__ double red[16];
  double g = 0.0, x = 0.0, y = 0.0, w = 0.0, ru = 0.0, ro = 0.0, zm = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    g += part[8 * b] + part[8 * b + 1];
    x += part[8 * b + 2];
    y += part[8 * b + 3];
    w += part[8 * b + 4];
  }
  for (int i = threadIdx.x; i < n1; i += blockDim.x) {
    ru = fmax(ru, kkt[3 * i]);
    ro = fmax(ro, kkt[3 * i + 1]);
    zm = fmax(zm, kkt[3 * i + 2]);
  }
  g = block_sum_d(g, red);
  x = block_sum_d(x, red);
  y = block_sum_d(y, red);
  w = block_sum_d(w, red);
  ru = block_max_d(ru, red);
  ro = block_max_d(ro, red);
  zm = block_max_d(zm, red);
  if (threadIdx.x == 0) {
    const double den = sqrt(w) * (sqrt(x) + sqrt(y));
    out[0] = sqrt(g) / fmax(den, 1e-300);
    out[1] = ru / fmax(zm, 1e-300);
    out[2] = ro;
  }
}

void launch_stationarity(const Plan& p, int w_from_g) {
  launch_agemm(p, 1);   // A = W~ Y~^* into the right-hand-side buffer
  launch_gramx(p);      // G_X
  launch_bgemm(p);      // X~^* W~
  k_stat_bin<<<p.nb, 256, 0, p.stream>>>(p.xt, p.yt, p.wt, p.rhs, p.bpart, p.gxm, p.stat_work, p.n1,
                                         p.n2, p.n3, p.r, p.nb, p.rho1, p.mixed);
  launch_zgemm(p);
  launch_slice(p, SLICE_KKT, nullptr, nullptr, w_from_g);
  k_stat_final<<<1, 256, 0, p.stream>>>(p.stat_work, p.nb, p.kkt, p.n1, p.scal + 8);
}

}  // namespace tctf

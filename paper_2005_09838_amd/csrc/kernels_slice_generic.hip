// The slice work (steps 3, 4 and 7 of the algorithm box) for any tube length n3 and any
// slice size: used where the fused LDS slice kernel does not apply (n3 outside the generated
// transform lengths, or an n2 x n3 slice larger than its LDS).  Three launches through the
// spatial buffers Z and W ([n1][n2][n3] FP32 in the workspace):
//   k_gen_inv    Z(i, j, k) = 1/n3 sum_b c_b Re(omega^{-b k} Z~(i, b, j))      (eq. (barAAk))
//   k_gen_wstep  the W-step of eq. (subquKKT) along every row (i, :, k), one block per OD
//                row i, with the objective's per-row partial sums (fit, ridge, K term) or,
//                for the stationarity check, the KKT residual maxima
//   k_gen_fwd    W~(i, b, j) = sum_k omega^{b k} W(i, j, k)                     (eq. (bar BA-k))
// The transforms are direct sums over a table of the n3 roots of unity (FP64), accumulated in
// FP64; they are not the iteration's hot path at the generated lengths.
#include "kernels.h"

namespace tctf {

// twg[m] = (cos, sin)(2 pi m / n3), m = 0..n3-1
__global__ void k_gen_twiddles(double2* __restrict__ twg, int n3) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n3) return;
  double s, c;
  sincospi(2.0 * (double)m / n3, &s, &c);
  twg[m] = make_double2(c, s);
}

// One thread per (tube (i, j), k).  z_out (optional): a copy of Z for the caller.
__global__ void __launch_bounds__(256) k_gen_inv(const float2* __restrict__ zt, const double2* __restrict__ twg,
                                                 float* __restrict__ zsp, float* __restrict__ z_out, int n1, int n2,
                                                 int n3, int nb) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)n1 * n2 * n3) return;
  const int k = (int)(g % n3);
  const long t = g / n3, i = t / n2, j = t % n2;
  const float2* src = zt + i * nb * n2 + j;
  double acc = 0.0;
  int m = 0;   // (b k) mod n3
  for (int b = 0; b < nb; ++b) {
    const float2 v = src[(long)b * n2];
    const double2 w = twg[m];
    acc += bin_weight(b, n3) * ((double)v.x * w.x + (double)v.y * w.y);   // Re(e^{-i th} v)
    m += k;
    if (m >= n3) m -= n3;
  }
  const float z = (float)(acc / n3);
  zsp[g] = z;
  if (z_out) z_out[g] = z;
}

// One thread per (tube (i, j), stored frequency b); W~ in FP32 or BF16 (stochastic rounding,
// rounding bits keyed by the entry and the iteration counter).
__global__ void __launch_bounds__(256) k_gen_fwd(const float* __restrict__ wsp, const double2* __restrict__ twg,
                                                 void* __restrict__ wt, int n1, int n2, int n3, int nb, int mixed,
                                                 const uint32_t* __restrict__ ctr) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)n1 * n2 * nb) return;
  const int b = (int)(g % nb);
  const long t = g / nb, i = t / n2, j = t % n2;
  const float* src = wsp + t * n3;
  double re = 0.0, im = 0.0;
  int m = 0;   // (b k) mod n3
  for (int k = 0; k < n3; ++k) {
    const double2 w = twg[m];
    const double v = src[k];
    re += w.x * v;
    im += w.y * v;
    m += b;
    if (m >= n3) m -= n3;
  }
  if (bin_is_real(b, n3)) im = 0.0;
  const size_t idx = ((size_t)i * nb + b) * n2 + j;
  if (mixed) {
    const uint32_t key = fmix32(ctr[0] * 0x9e3779b9u + 0x7f4a7c15u);
    ((uint32_t*)wt)[idx] = pack_bf16x2_sr((float)re, (float)im, fmix32((uint32_t)idx ^ key));
  } else {
    ((float2*)wt)[idx] = make_float2((float)re, (float)im);
  }
}

// One block per OD row i; thread k takes the rows (i, :, k), k = tid, tid + blockDim, ...
// Thomas elimination over the whole row: observed entries are identity equations (w = g),
// unobserved ones (1 + mu + rho2 deg_j) w_j - rho2 (w_{j-1} + w_{j+1}) = z_j; strictly
// diagonally dominant, so no pivoting.  c' of the elimination goes to cbuf.
// mode: SLICE_INIT (W = P_Omega(G)), SLICE_ITER, SLICE_RESULT, SLICE_KKT; w_from_g: W is
// P_Omega(G) instead of the W-step's solution.
__global__ void __launch_bounds__(256) k_gen_wstep(const float* __restrict__ zsp, const float* __restrict__ gp,
                                                   float* __restrict__ wsp, float* __restrict__ cbuf,
                                                   float* __restrict__ w_out, double* __restrict__ slice_obj,
                                                   double* __restrict__ kkt, int n1, int n2, int n3, double mu,
                                                   double rho2, int mode, int w_from_g) {
  __shared__ double red[16];
  const long i = blockIdx.x;
  const float r2 = (float)rho2;
  const bool solve = mode != SLICE_INIT && !w_from_g;
  double fit = 0.0, ridge = 0.0, sm = 0.0;
  for (int k = threadIdx.x; k < n3; k += blockDim.x) {
    const long base = i * n2 * n3 + k;   // entry (i, j, k) at base + j n3 (packed G too, on this path)
    auto deg = [&](int j) { return n2 == 1 ? 0.0f : ((j == 0 || j == n2 - 1) ? 1.0f : 2.0f); };
    if (solve) {
      float cp = 0.0f, dp = 0.0f;
      for (int j = 0; j < n2; ++j) {
        const long e = base + (long)j * n3;
        const float g = gp[e];
        float c, d;
        if (!is_unobserved(g)) {
          c = 0.0f;
          d = g;
        } else {
          const float a = j > 0 ? -r2 : 0.0f, up = j + 1 < n2 ? -r2 : 0.0f;
          const float piv = 1.0f + (float)mu + r2 * deg(j) - a * cp;
          c = up / piv;
          d = (zsp[e] - a * dp) / piv;
        }
        cbuf[e] = c;
        wsp[e] = d;
        cp = c;
        dp = d;
      }
      float wn = 0.0f;
      for (int j = n2 - 1; j >= 0; --j) {
        const long e = base + (long)j * n3;
        wn = wsp[e] - cbuf[e] * wn;
        wsp[e] = wn;
      }
    } else {
      for (int j = 0; j < n2; ++j) {
        const long e = base + (long)j * n3;
        const float g = gp[e];
        wsp[e] = is_unobserved(g) ? 0.0f : g;
      }
    }
    // objective partial sums (or KKT maxima) of the row
    for (int j = 0; j < n2; ++j) {
      const long e = base + (long)j * n3;
      const float w = wsp[e], z = zsp[e];
      const bool obs = !is_unobserved(gp[e]);
      if (w_out) w_out[e] = w;
      if (mode == SLICE_KKT) {
        const double l = j > 0 ? (double)wsp[e - n3] : 0.0, r = j + 1 < n2 ? (double)wsp[e + n3] : 0.0;
        if (!obs && solve) fit = fmax(fit, fabs((1.0 + mu + rho2 * deg(j)) * w - rho2 * (l + r) - (double)z));
        else if (obs) ridge = fmax(ridge, fabs((double)w - (double)gp[e]));
        sm = fmax(sm, fabs((double)z));
      } else {
        const double d = (double)z - (double)w;
        fit += d * d;
        ridge += (double)w * w;
        if (j + 1 < n2) {
          const double dr = (double)wsp[e + n3] - (double)w;
          sm += dr * dr;
        }
      }
    }
  }
  if (mode == SLICE_KKT) {
    fit = block_max_d(fit, red);
    ridge = block_max_d(ridge, red);
    sm = block_max_d(sm, red);
    if (threadIdx.x == 0) {
      kkt[3 * i + 0] = fit;
      kkt[3 * i + 1] = ridge;
      kkt[3 * i + 2] = sm;
    }
  } else if (mode != SLICE_RESULT) {
    fit = block_sum_d(fit, red);
    ridge = block_sum_d(ridge, red);
    sm = block_sum_d(sm, red);
    if (threadIdx.x == 0) {
      slice_obj[3 * i + 0] = fit;
      slice_obj[3 * i + 1] = ridge;
      slice_obj[3 * i + 2] = sm;
    }
  }
}

void launch_gen_twiddles(const Plan& p) {
  k_gen_twiddles<<<(p.n3 + 255) / 256, 256, 0, p.stream>>>(p.twg, p.n3);
}

void launch_slice_generic(const Plan& p, int mode, float* w_out, float* z_out, int w_from_g) {
  const long n = (long)p.n1 * p.n2 * p.n3;
  const bool need_z = !(mode == SLICE_RESULT && w_from_g && z_out == nullptr);
  if (need_z)
    k_gen_inv<<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>(p.zt, p.twg, p.zsp, z_out, p.n1, p.n2, p.n3, p.nb);
  else
    launch_zero(p, p.zsp, (size_t)n * 4);
  const int threads = p.n3 >= 256 ? 256 : ((p.n3 + 63) / 64) * 64;
  k_gen_wstep<<<p.n1, threads, 0, p.stream>>>(p.zsp, p.gp, p.wsp, p.csp, w_out, p.slice_obj, p.kkt, p.n1, p.n2, p.n3,
                                              p.mu, p.rho2, mode, w_from_g);
  if (mode == SLICE_INIT || mode == SLICE_ITER) {
    const long nf = (long)p.n1 * p.n2 * p.nb;
    k_gen_fwd<<<(unsigned)((nf + 255) / 256), 256, 0, p.stream>>>(p.wsp, p.twg, p.wt, p.n1, p.n2, p.n3, p.nb,
                                                                 p.mixed, p.ctr);
  }
}

}  // namespace tctf

// Setup kernels: packing of the observations, constant tables, initial transforms,
// the objective reduction and the termination / stationarity measures.
#include "kernels.h"

namespace tctf {

size_t wt_elem_bytes(const Plan& p) { return p.mixed ? 4 : 8; }

// One thread per row (i, k) along mode 2.  Observed entries keep their value (they must
// be finite); unobserved ones become NaNs carrying their position in the run of
// consecutive unobserved entries (section 3.3: the equality constraints of the W-step
// are eliminated row by row, leaving one tridiagonal system per run).  The packed copy is
// stored row by row, [n1][n3][n2], for the cooperative slice kernel (a wavefront reads entry
// (i, j, k) for 64 consecutive tubes j at once), else like G, [n1][n2][n3]: kernels with
// one thread per tube or per row then read contiguous runs, and each wavefront keeps more
// cache lines in flight.
__global__ void k_pack_g(const float* __restrict__ g, const uint8_t* __restrict__ om,
                         float* __restrict__ gp, int n1, int n2, int n3, int rows, int* flag) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (long)n1 * n3) return;
  const long i = row / n3, k = row % n3;
  int run_start = -1;          // index of the first unobserved entry of the current run
  bool seen_obs = false;
  for (int j = 0; j < n2; ++j) {
    const long idx = (i * n2 + j) * n3 + k, out = rows ? (i * n3 + k) * n2 + j : idx;
    if (om[idx]) {
      const float v = g[idx];
      if (!isfinite(v)) atomicOr(flag, 1);
      gp[out] = v;
      seen_obs = true;
      run_start = -1;
    } else {
      if (run_start < 0) run_start = j;
      const uint32_t starts_row = seen_obs ? 0u : 1u;
      gp[out] = __uint_as_float(pack_unobserved((uint32_t)(j - run_start), starts_row));
    }
  }
}

void launch_pack_g(const Plan& p, const float* G, const uint8_t* omega) {
  const long rows = (long)p.n1 * p.n3;
  k_pack_g<<<(unsigned)((rows + 255) / 256), 256, 0, p.stream>>>(G, omega, p.gp, p.n1, p.n2, p.n3, p.g_rows,
                                                                  p.flag);
}

// Reciprocal pivots of the W-step row systems (eq. (subquKKT)), in FP64 then rounded.
// Along a run of unobserved entries the system matrix is tridiagonal with off-diagonal
// -rho2 and diagonal (K_{mu rho2})_jj = 1 + mu + rho2 deg(j) (deg = 1 at the row ends,
// 2 inside).  Elimination without pivoting gives pivots alpha_t that depend only on the
// position t in the run, on whether the run starts at j = 0, and on whether j = n2 - 1.
//   wtab[0][t]: run starting at j = 0, interior j      wtab[1][t]: run after an observed entry
//   wtab[2][t]: as [0] but j = n2 - 1                   wtab[3][t]: as [1] but j = n2 - 1
// The H_rho1 = I + rho1 H^T H tables (Thomas coefficients along mode 1):
//   htab[0][i] = rho1 / alpha_{i-1} (0 for i = 0), htab[1][i] = 1/alpha_i,
//   htab[2][i] = rho1 / alpha_i.
__global__ void k_tables(float* __restrict__ wtab, float* __restrict__ htab, int n1, int n2,
                         double mu, double rho1, double rho2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double dint = 1.0 + mu + 2.0 * rho2, dend = 1.0 + mu + rho2, r2 = rho2 * rho2;
    if (n2 == 1) {
      for (int q = 0; q < 4; ++q) wtab[q] = (float)(1.0 / (1.0 + mu));
    } else {
      double a0 = 0.0, a1 = 0.0;   // previous pivots of the two run types
      for (int t = 0; t < n2; ++t) {
        // run starting at row start: j = t
        const double p0 = (t == 0) ? dend : dint - r2 / a0;
        const double l0 = (t == 0) ? dend : dend - r2 / a0;       // if j = t = n2 - 1
        // run after an observed entry
        const double p1 = (t == 0) ? dint : dint - r2 / a1;
        const double l1 = (t == 0) ? dend : dend - r2 / a1;
        wtab[0 * n2 + t] = (float)(1.0 / p0);
        wtab[1 * n2 + t] = (float)(1.0 / p1);
        wtab[2 * n2 + t] = (float)(1.0 / l0);
        wtab[3 * n2 + t] = (float)(1.0 / l1);
        a0 = p0;
        a1 = p1;
      }
    }
    double prev = 0.0;
    for (int i = 0; i < n1; ++i) {
      const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
      const double d = 1.0 + rho1 * deg;
      const double alpha = (i == 0) ? d : d - rho1 * rho1 / prev;
      htab[0 * n1 + i] = (i == 0) ? 0.0f : (float)(rho1 / prev);
      htab[1 * n1 + i] = (float)(1.0 / alpha);
      htab[2 * n1 + i] = (float)(rho1 / alpha);
      prev = alpha;
    }
  }
}

void launch_tables(const Plan& p) {
  k_tables<<<1, 64, 0, p.stream>>>(p.wtab, p.htab, p.n1, p.n2, p.mu, p.rho1, p.rho2);
}

// Transform of eq. (bar BA-k) of real tubes src[p][q][0..n3) into stored frequencies
// b = 0..n3/2: dst[b*sb + p*sp + q*sq] = sum_l exp(+2 pi i b l / n3) src[p][q][l].
// Direct FP64 sums, one thread per (tube, frequency): used only to bring the initial
// factors into the Fourier domain.
__global__ void k_tube_dft_setup(const float* __restrict__ src, float2* __restrict__ dst, int P, int Q,
                                 int n3, int nb, long sb, long sp, long sq) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)P * Q * nb) return;
  const long t = g / nb;
  const int b = (int)(g % nb);
  const long p = t / Q, q = t % Q;
  const float* a = src + t * n3;
  double re = 0.0, im = 0.0;
  for (int l = 0; l < n3; ++l) {
    double s, c;
    sincospi(2.0 * (double)((long)b * l % n3) / n3, &s, &c);
    re += c * a[l];
    im += s * a[l];
  }
  if (bin_is_real(b, n3)) im = 0.0;
  dst[b * sb + p * sp + q * sq] = make_float2((float)re, (float)im);
}

// Inverse of eq. (barAAk) from the stored frequencies (conjugates fill the rest), one
// thread per (tube, position).
__global__ void k_tube_idft_setup(const float2* __restrict__ src, float* __restrict__ dst, int P, int Q,
                                  int n3, int nb, long sb, long sp, long sq) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)P * Q * n3) return;
  const long t = g / n3;
  const int l = (int)(g % n3);
  const long p = t / Q, q = t % Q;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) {
    const float2 v = src[b * sb + p * sp + q * sq];
    double s, c;
    sincospi(2.0 * (double)((long)b * l % n3) / n3, &s, &c);
    const double w = bin_weight(b, n3);
    // Re(X_b exp(-i theta)) = re cos + im sin
    acc += w * ((double)v.x * c + (bin_is_real(b, n3) ? 0.0 : (double)v.y * s));
  }
  dst[t * n3 + l] = (float)(acc / n3);
}

static inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_tube_dft_setup(const Plan& p, const float* src, float2* dst, int P, int Q, long sb, long sp, long sq) {
  k_tube_dft_setup<<<blocks_for((long)P * Q * p.nb, 256), 256, 0, p.stream>>>(src, dst, P, Q, p.n3, p.nb, sb,
                                                                               sp, sq);
}
void launch_tube_idft_setup(const Plan& p, const float2* src, float* dst, int P, int Q, long sb, long sp, long sq) {
  k_tube_idft_setup<<<blocks_for((long)P * Q * p.n3, 256), 256, 0, p.stream>>>(src, dst, P, Q, p.n3, p.nb, sb,
                                                                               sp, sq);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed, counter = thread
// index; Box-Muller turns its four uniforms into four standard normals.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void k_normal(float* __restrict__ out, long n, uint64_t seed) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t * 4 >= n) return;
  uint32_t c[4] = {(uint32_t)t, (uint32_t)(t >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  for (int h = 0; h < 2; ++h) {
    const double u1 = ((double)c[2 * h] + 0.5) * (1.0 / 4294967296.0);
    const double u2 = ((double)c[2 * h + 1] + 0.5) * (1.0 / 4294967296.0);
    const double rad = sqrt(-2.0 * log(u1));
    double s, co;
    sincospi(2.0 * u2, &s, &co);
    if (t * 4 + 2 * h < n) out[t * 4 + 2 * h] = (float)(rad * co);
    if (t * 4 + 2 * h + 1 < n) out[t * 4 + 2 * h + 1] = (float)(rad * s);
  }
}

void launch_normal(const Plan& p, float* dst, size_t n, uint64_t seed) {
  k_normal<<<blocks_for(((long)n + 3) / 4, 256), 256, 0, p.stream>>>(dst, (long)n, seed);
}

__global__ void k_zero(uint32_t* __restrict__ d, long words) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < words) d[t] = 0u;
}

void launch_zero(const Plan& p, void* dst, size_t bytes) {
  const long words = (long)(bytes / 4);
  if (words > 0) k_zero<<<blocks_for(words, 256), 256, 0, p.stream>>>((uint32_t*)dst, words);
}

// f0 of eq. (TETP-optim): 1/2 fit + mu/2 ridge + rho2/2 (mode-2 differences) from the
// W-step rows, and rho1/2 ||H unfold(Z,1)||^2 = rho1/(2 n3) sum_b c_b tr(...) from the
// Fourier form eq. (fun-XYW).  Fixed-order FP64 sums.
__global__ void k_objective(const double* __restrict__ so, int n1, const double* __restrict__ bo, int nb,
                            double mu, double rho1, double rho2, int n3, double* out) {
  __shared__ double red[16];
  double fit = 0.0, ridge = 0.0, sm = 0.0, h = 0.0;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) {
    fit += so[3 * i];
    ridge += so[3 * i + 1];
    sm += so[3 * i + 2];
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) h += bo[b];
  fit = block_sum_d(fit, red);
  ridge = block_sum_d(ridge, red);
  sm = block_sum_d(sm, red);
  h = block_sum_d(h, red);
  if (threadIdx.x == 0) out[0] = 0.5 * fit + 0.5 * mu * ridge + 0.5 * rho2 * sm + 0.5 * rho1 * h / n3;
}

void launch_objective(const Plan& p) {
  k_objective<<<1, 256, 0, p.stream>>>(p.slice_obj, p.n1, p.bin_obj, p.nb, p.mu, p.rho1, p.rho2, p.n3, p.scal);
}

// Step 6 quantities between the snapshot and the current iterate:
// max |dX~|, max |dY~| (the maxima over stored frequencies equal those over all of them)
// and ||dW||_F from the stored frequencies by Parseval: ||dW||^2 = 1/n3 sum_b c_b ||dW~_b||^2.
// A non-finite difference counts as +inf in the maxima (fmax would drop a NaN) and stays NaN
// in the sum, so a non-finite iterate shows in the result.  Grid-stride loops over a grid
// that covers every compute unit; per-block partials, then one block combines them in a
// fixed order.
#define TERM_BLOCKS 1024
__global__ void __launch_bounds__(256) k_termination(const float2* __restrict__ x, const float2* __restrict__ xp, long nx,
                              const float2* __restrict__ y, const float2* __restrict__ yp, long ny,
                              const void* __restrict__ w, const void* __restrict__ wp, int mixed,
                              int n1, int nb, int n2, int n3, double* part) {
  __shared__ double red[16];
  double mx = 0.0, my = 0.0, sw = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long e = t0; e < nx; e += stride) {
    const double d = hypot((double)x[e].x - xp[e].x, (double)x[e].y - xp[e].y);
    mx = (d == d) ? fmax(mx, d) : INFINITY;
  }
  for (long e = t0; e < ny; e += stride) {
    const double d = hypot((double)y[e].x - yp[e].x, (double)y[e].y - yp[e].y);
    my = (d == d) ? fmax(my, d) : INFINITY;
  }
  const long nw = (long)n1 * nb * n2;
  for (long e = t0; e < nw; e += stride) {
    const int b = (int)((e / n2) % nb);
    float2 a, c;
    if (mixed) { a = unpack_bf16x2(((const uint32_t*)w)[e]); c = unpack_bf16x2(((const uint32_t*)wp)[e]); }
    else { a = ((const float2*)w)[e]; c = ((const float2*)wp)[e]; }
    const double dr = (double)a.x - c.x, di = (double)a.y - c.y;
    sw += bin_weight(b, n3) * (dr * dr + di * di);
  }
  mx = block_max_d(mx, red);
  my = block_max_d(my, red);
  sw = block_sum_d(sw, red);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = mx;
    part[3 * blockIdx.x + 1] = my;
    part[3 * blockIdx.x + 2] = sw;
  }
}

__global__ void __launch_bounds__(256) k_termination_final(const double* __restrict__ part, int nblk, int n3, double* out) {
  __shared__ double red[16];
  double mx = 0.0, my = 0.0, sw = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    mx = fmax(mx, part[3 * b]);
    my = fmax(my, part[3 * b + 1]);
    sw += part[3 * b + 2];
  }
  mx = block_max_d(mx, red);
  my = block_max_d(my, red);
  sw = block_sum_d(sw, red);
  if (threadIdx.x == 0) {
    out[0] = mx;
    out[1] = my;
    out[2] = sqrt(sw / n3);
  }
}

size_t termination_work_doubles() { return 3 * TERM_BLOCKS; }

void launch_termination(const Plan& p) {
  const long nw = (long)p.n1 * p.nb * p.n2;
  int nblk = (int)((nw + 1023) / 1024);
  if (nblk > TERM_BLOCKS) nblk = TERM_BLOCKS;
  if (nblk < 1) nblk = 1;
  k_termination<<<nblk, 256, 0, p.stream>>>(p.xt, p.xt_prev, (long)p.nb * p.r * p.n1, p.yt, p.yt_prev,
                                            (long)p.nb * p.r * p.n2, p.wt, p.wt_prev, p.mixed, p.n1, p.nb,
                                            p.n2, p.n3, p.stat_work);
  k_termination_final<<<1, 256, 0, p.stream>>>(p.stat_work, nblk, p.n3, p.scal + 4);
}

}  // namespace tctf

// Reverse-mode derivatives of one TCTF2R iteration, in FP64 throughout.
//
// The forward iteration (section 4.1, algorithm box steps 1-4 and 7) with full-rank Grams
// and the common step eta maps (X~, Y~, W) to
//   X~+ = (1 - eta) X~ + eta H_rho1^{-1} W~ Y~^* G_Y^{-1},        G_Y = Y~ Y~^*,
//   Y~+ = (1 - eta) Y~ + eta G_X^{-1} X~+^* W~,                   G_X = X~+^* H_rho1 X~+,
//   Z   = Re idft(X~+ Y~+)                                         (eq. (barAAk)),
//   W+  = the W-step of eq. (subquKKT) at Z,  W~ = dft(W)          (eq. (bar BA-k)),
// (the pseudo-inverse updates of eq. (updataXYW1) reduce to these when the Grams have full
// rank, since grad_X = H_rho1 X~ G_Y - W~ Y~^* and grad_Y = G_X Y~ - X~^* W~).
// The kernels below run the reverse pass of that map.  Adjoint convention for a real loss
// L: the adjoint of a complex entry z is dL/dRe z + i dL/dIm z; a stored frequency b
// carries the adjoint it has in the sum over all n3 frequencies.  Per frequency the rules
// are those of products (C = A B: A_bar += C_bar B^*, B_bar += A^* C_bar), inverses
// (C = G^{-1}: G_bar = -C^* C_bar C^*) and Grams (G = Y Y^*: Y_bar += (G_bar + G_bar^*) Y);
// across frequencies only the tube transforms and the weight adjoints couple them, through
// the bin weights c_b.  The W-step's adjoint solves the same tridiagonal system restricted
// to the unobserved entries of each row (i, :, k) (K_{mu rho2} is symmetric).
//
// Simple building blocks, chosen for clarity over speed (this is not the iteration's hot
// path): a batched complex GEMM on 16 x 16 LDS tiles over strided views (FP32 forward
// values or FP64 adjoints), tridiagonal H_rho1 applications and solves along n1, direct
// tube transforms, FP64 Gram inverses by the library's Hermitian pseudo-inverse, and
// fixed-order reductions for the weights' adjoints.
#include "kernels.h"
#include "pinv.h"

namespace tctf {

// ---------------------------------------------------------------- batched complex GEMM
__device__ __forceinline__ cd ld_view(const CView& v, int b, long i, long j) {
  const long e = (long)b * v.bs + i * v.rs + j * v.cs;
  cd z;
  if (v.f32) {
    const float2 f = ((const float2*)v.p)[e];
    z = cd_make(f.x, f.y);
  } else {
    const double2 d = ((const double2*)v.p)[e];
    z = cd_make(d.x, d.y);
  }
  if (v.conj) z.im = -z.im;
  return z;
}

// C = alpha A B + beta C for every batch b (blockIdx.z); A is M x K, B is K x N, C is M x N
// FP64 complex at C + b cbs + i crs + j ccs.  beta = 0 does not read C.
__global__ void __launch_bounds__(256) k_zgemm64(int M, int N, int K, cd alpha, CView A, CView B, cd beta,
                                                 double2* __restrict__ C, long cbs, long crs, long ccs) {
  __shared__ cd As[16][17];
  __shared__ cd Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4, b = blockIdx.z;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  cd acc = cd_make(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += 16) {
    As[ty][tx] = (i < M && k0 + tx < K) ? ld_view(A, b, i, k0 + tx) : cd_make(0.0, 0.0);
    Bs[ty][tx] = (k0 + ty < K && j < N) ? ld_view(B, b, k0 + ty, j) : cd_make(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) cd_fma(acc, As[ty][kk], Bs[kk][tx]);
    __syncthreads();
  }
  if (i < M && j < N) {
    double2* c = C + (long)b * cbs + (long)i * crs + (long)j * ccs;
    cd v = cd_mul(alpha, acc);
    if (beta.re != 0.0 || beta.im != 0.0) v = cd_add(v, cd_mul(beta, cd_make(c->x, c->y)));
    *c = make_double2(v.re, v.im);
  }
}

static void gemm(const Plan& p, int M, int N, int K, cd alpha, CView A, CView B, cd beta, double2* C, long cbs,
                 long crs, long ccs) {
  dim3 grid((N + 15) / 16, (M + 15) / 16, p.nb);
  k_zgemm64<<<grid, 256, 0, p.stream>>>(M, N, K, alpha, A, B, beta, C, cbs, crs, ccs);
}

static CView view(const void* ptr, long bs, long rs, long cs, int f32) {
  CView v;
  v.p = ptr;
  v.bs = bs;
  v.rs = rs;
  v.cs = cs;
  v.f32 = f32;
  v.conj = 0;
  return v;
}
static CView ctr(CView v) {   // conjugate transpose of a view
  const long t = v.rs;
  v.rs = v.cs;
  v.cs = t;
  v.conj ^= 1;
  return v;
}

// ---------------------------------------------------------------- elementwise helpers
__global__ void k_adj_axpby(long n, double a, const double2* __restrict__ x, double b, double2* y, double2* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double2 xv = x[e];
  double2 v = make_double2(a * xv.x, a * xv.y);
  if (b != 0.0) {
    const double2 yv = y[e];
    v.x += b * yv.x;
    v.y += b * yv.y;
  }
  out[e] = v;
}
static void axpby(const Plan& p, long n, double a, const double2* x, double b, double2* y, double2* out) {
  k_adj_axpby<<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>(n, a, x, b, y, out);
}

// Imaginary parts of the real frequencies (b = 0 and the Nyquist bin) set to 0: the forward
// update does this to its results, and the map is its own adjoint.  a: [nb][per] complex.
__global__ void k_adj_realbins(double2* a, long per, int nb, int n3) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  a[e].y = 0.0;
  if (n3 % 2 == 0 && nb - 1 == n3 / 2 && nb > 1) a[(long)(nb - 1) * per + e].y = 0.0;
}
static void realbins(const Plan& p, double2* a, long per) {
  k_adj_realbins<<<(unsigned)((per + 255) / 256), 256, 0, p.stream>>>(a, per, p.nb, p.n3);
}

// S = G + G^* per frequency (r x r)
__global__ void k_adj_herm(const double2* __restrict__ g, double2* __restrict__ s, int r, int nb) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long rr = (long)r * r;
  if (e >= rr * nb) return;
  const long b = e / rr, k = e % rr, i = k / r, j = k % r;
  const double2 u = g[e], v = g[b * rr + j * r + i];
  s[e] = make_double2(u.x + v.x, u.y - v.y);
}

// out(b, s, i) = (a + c deg_i) x_i - c (x_{i-1} + x_{i+1}) along n1 for X-shaped arrays
// [nb][r][n1] (deg_i = number of neighbours of row i): H_rho1 with (1, rho1), D^T D with (0, 1).
template <typename T>
__global__ void k_adj_happly(const T* __restrict__ x, double2* __restrict__ out, int n1, long total, double a,
                             double c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int i = (int)(e % n1);
  const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
  auto get = [&](long k) { return cd_make((double)x[k].x, (double)x[k].y); };
  cd v = cd_scale(get(e), a + c * deg);
  if (i > 0) v = cd_sub(v, cd_scale(get(e - 1), c));
  if (i + 1 < n1) v = cd_sub(v, cd_scale(get(e + 1), c));
  out[e] = make_double2(v.re, v.im);
}

// Thomas coefficients of H_rho1 = I + rho1 D^T D along n1 (one thread): tab[i] = 1 / pivot_i,
// tab[n1 + i] = the superdiagonal factor c'_i.
__global__ void k_adj_htab(int n1, double rho1, double* tab) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double cp = 0.0;
  for (int i = 0; i < n1; ++i) {
    const double deg = (n1 == 1) ? 0.0 : ((i == 0 || i == n1 - 1) ? 1.0 : 2.0);
    const double piv = 1.0 + rho1 * deg - (i > 0 ? -rho1 * cp : 0.0);
    tab[i] = 1.0 / piv;
    cp = (i + 1 < n1) ? -rho1 / piv : 0.0;
    tab[n1 + i] = cp;
  }
}

// y = H_rho1^{-1} x for every column (b, s) of X-shaped arrays (one thread per column).
__global__ void k_adj_hsolve(const double2* __restrict__ x, double2* __restrict__ y, int n1, long ncol,
                             double rho1, const double* __restrict__ tab) {
  const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  const double2* xc = x + col * n1;
  double2* yc = y + col * n1;
  double dr = 0.0, di = 0.0;
  for (int i = 0; i < n1; ++i) {   // forward: d'_i = (x_i + rho1 d'_{i-1}) / pivot_i
    const double2 v = xc[i];
    dr = (v.x + rho1 * dr) * tab[i];
    di = (v.y + rho1 * di) * tab[i];
    yc[i] = make_double2(dr, di);
  }
  double wr = 0.0, wi = 0.0;
  for (int i = n1 - 1; i >= 0; --i) {   // backward: y_i = d'_i - c'_i y_{i+1}
    const double2 d = yc[i];
    wr = d.x - tab[n1 + i] * wr;
    wi = d.y - tab[n1 + i] * wi;
    yc[i] = make_double2(wr, wi);
  }
}

// G^{-1} of every frequency's r x r Gram (FP64 pseudo-inverse of Lemma SVPMPI, which is
// the inverse at full rank); flag[0] = 1 if some Gram is rank deficient.
__global__ void __launch_bounds__(256) k_adj_inv(const double2* __restrict__ g, double2* __restrict__ gi, int r,
                                                 int* flag) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int b = blockIdx.x, rr = r * r;
  cd* a = (cd*)sm;
  cd* p = a + rr;
  PinvScratch ps;
  ps.work = p + rr;
  ps.vec = ps.work + rr;
  ps.colk = ps.vec + rr;
  ps.rowk = ps.colk + r;
  ps.rot = (double*)(ps.rowk + r);
  ps.red = ps.rot + 96;
  for (int e = threadIdx.x; e < rr; e += blockDim.x) a[e] = cd_make(g[(long)b * rr + e].x, g[(long)b * rr + e].y);
  __syncthreads();
  const int full = pinv_herm(a, p, r, 0, ps);
  for (int e = threadIdx.x; e < rr; e += blockDim.x) gi[(long)b * rr + e] = make_double2(p[e].re, p[e].im);
  if (threadIdx.x == 0 && !full) flag[0] = 1;
}

// ---------------------------------------------------------------- tube transforms
// Spatial tubes -> stored frequencies: out(b, p, q) = s sum_l omega^{b l} in(p, q, l),
// omega = exp(+2 pi i / n3) (eq. (bar BA-k)); one thread per (tube, b).
__global__ void k_adj_tube_fwd(const double* __restrict__ in, long isp, long isq, double2* __restrict__ out,
                               long obs, long ops, long oqs, int P, int Q, int n3, int nb, double s) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)P * Q * nb) return;
  const int b = (int)(g % nb);
  const long t = g / nb, pp = t / Q, qq = t % Q;
  const double* a = in + pp * isp + qq * isq;
  double re = 0.0, im = 0.0;
  for (int l = 0; l < n3; ++l) {
    double sn, cs;
    sincospi(2.0 * (double)((long)b * l % n3) / n3, &sn, &cs);
    re += cs * a[l];
    im += sn * a[l];
  }
  out[b * obs + pp * ops + qq * oqs] = make_double2(s * re, s * im);
}

// Stored frequencies -> spatial tubes: out(p, q, l) = s sum_b c_b Re(omega^{-b l} in(b, p, q))
// (the sum over all n3 frequencies of a conjugate-symmetric spectrum); one thread per
// (tube, l).  T: float2 (forward values) or double2 (adjoints).
template <typename T>
__global__ void k_adj_tube_inv(const T* __restrict__ in, long ibs, long ips, long iqs, double* __restrict__ out,
                               long osp, long osq, int P, int Q, int n3, int nb, double s) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)P * Q * n3) return;
  const int l = (int)(g % n3);
  const long t = g / n3, pp = t / Q, qq = t % Q;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) {
    const T v = in[b * ibs + pp * ips + qq * iqs];
    double sn, cs;
    sincospi(2.0 * (double)((long)b * l % n3) / n3, &sn, &cs);
    acc += bin_weight(b, n3) * ((double)v.x * cs + (double)v.y * sn);   // Re(e^{-i th} v)
  }
  out[pp * osp + qq * osq + l] = s * acc;
}

// ---------------------------------------------------------------- W-step adjoint
// For every row (i, :, k): lambda solves K_uu lambda_u = w_bar_u with lambda_o = 0
// (K_{mu rho2} = (1 + mu) I + rho2 K^T K restricted to the unobserved entries), z_bar = lambda;
// partial sums of -<lambda, w> (mu) and -<lambda, K^T K w> (rho2) per block.  One thread per
// row; cbuf holds the forward-elimination factors.
__global__ void __launch_bounds__(256) k_adj_wstep(const double* __restrict__ wbar, const double* __restrict__ w,
                                                   const float* __restrict__ gp, double* __restrict__ zbar,
                                                   double* __restrict__ cbuf, int n1, int n2, int n3, double mu,
                                                   double rho2, int g_rows, double* __restrict__ part) {
  __shared__ double red[16];
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double smu = 0.0, srho = 0.0;
  if (row < (long)n1 * n3) {
    const long i = row / n3, k = row % n3;
    const long base = i * n2 * n3 + k;   // element (i, j, k) at base + j n3
    auto deg = [&](int j) { return n2 == 1 ? 0.0 : ((j == 0 || j == n2 - 1) ? 1.0 : 2.0); };
    auto unobs = [&](int j) {   // packed G by rows or by tubes (Plan::g_rows)
      return is_unobserved(gp[g_rows ? (i * n3 + k) * n2 + j : base + (long)j * n3]);
    };
    double cprev = 0.0, dprev = 0.0;
    bool uprev = false;
    for (int j = 0; j < n2; ++j) {
      const long e = base + (long)j * n3;
      const bool u = unobs(j);
      double cj = 0.0, dj = 0.0;
      if (u) {
        const double a = uprev ? -rho2 : 0.0;                              // coupling to j - 1
        const double c = (j + 1 < n2 && unobs(j + 1)) ? -rho2 : 0.0;      // coupling to j + 1
        const double piv = 1.0 + mu + rho2 * deg(j) - a * cprev;
        cj = c / piv;
        dj = (wbar[e] - a * dprev) / piv;
      }
      cbuf[e] = cj;
      zbar[e] = dj;
      cprev = cj;
      dprev = dj;
      uprev = u;
    }
    double lnext = 0.0;
    for (int j = n2 - 1; j >= 0; --j) {
      const long e = base + (long)j * n3;
      const double lam = zbar[e] - cbuf[e] * lnext;   // 0 on observed entries (d = c = 0)
      zbar[e] = lam;
      lnext = lam;
      const double wj = w[e];
      double ktk = deg(j) * wj;
      if (j > 0) ktk -= w[e - n3];
      if (j + 1 < n2) ktk -= w[e + n3];
      smu -= lam * wj;
      srho -= lam * ktk;
    }
  }
  smu = block_sum_d(smu, red);
  srho = block_sum_d(srho, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smu;
    part[2 * blockIdx.x + 1] = srho;
  }
}

// theta[k0] += sum of part[2 b], theta[k1] += sum of part[2 b + 1] (fixed order)
__global__ void k_adj_reduce2(const double* __restrict__ part, int nblk, double* theta, int k0, int k1) {
  __shared__ double red[16];
  double a = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    a += part[2 * b];
    c += part[2 * b + 1];
  }
  a = block_sum_d(a, red);
  c = block_sum_d(c, red);
  if (threadIdx.x == 0) {
    theta[k0] += a;
    theta[k1] += c;
  }
}

// theta[k] += coef sum_b c_b Re sum_e conj(A(b, e)) B(b, e); A, B: [nb][per] complex.
// Partials per block in part[], then one block adds them in a fixed order.
__global__ void __launch_bounds__(256) k_adj_wdot(const double2* __restrict__ A, const double2* __restrict__ B,
                                                  long per, int nb, int n3, double* __restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  const long n = per * nb;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double2 a = A[e], b = B[e];
    s += bin_weight((int)(e / per), n3) * (a.x * b.x + a.y * b.y);
  }
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void k_adj_reduce1(const double* __restrict__ part, int nblk, double coef, double* theta, int k) {
  __shared__ double red[16];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += part[b];
  a = block_sum_d(a, red);
  if (threadIdx.x == 0) theta[k] += coef * a;
}

__global__ void k_adj_flag_zero(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}

// ---------------------------------------------------------------- host side
#define ADJ_DOT_BLOCKS 256

size_t adjoint_work_bytes(const Plan& p) {
  const size_t N = (size_t)p.n1 * p.n2 * p.n3, nh = (size_t)p.nb * p.n1 * p.n2;
  const size_t fx = (size_t)p.nb * p.r * p.n1, fy = (size_t)p.nb * p.r * p.n2, g = (size_t)p.nb * p.r * p.r;
  const size_t wpart = ((N / p.n2 + 255) / 256) * 2 + ADJ_DOT_BLOCKS;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return 3 * al(N * 8) + 2 * al(nh * 16) + 9 * al(fx * 16) + 4 * al(fy * 16) + 11 * al(g * 16) +
         al(2 * (size_t)p.n1 * 8) + al(wpart * 8) + al(64);
}

void adjoint_carve(const Plan& p, void* ws, AdjWork* w) {
  const size_t N = (size_t)p.n1 * p.n2 * p.n3, nh = (size_t)p.nb * p.n1 * p.n2;
  const size_t fx = (size_t)p.nb * p.r * p.n1, fy = (size_t)p.nb * p.r * p.n2, g = (size_t)p.nb * p.r * p.r;
  const size_t wpart = ((N / p.n2 + 255) / 256) * 2 + ADJ_DOT_BLOCKS;
  unsigned char* o = (unsigned char*)ws;
  auto take = [&](size_t bytes) { unsigned char* at = o; o += (bytes + 255) & ~(size_t)255; return (void*)at; };
  w->w1s = (double*)take(N * 8);
  w->cbuf = (double*)take(N * 8);
  w->zbar = (double*)take(N * 8);
  w->ztb = (double2*)take(nh * 16);
  w->wtb = (double2*)take(nh * 16);
  double2** xs[9] = {&w->x1b, &w->hx1, &w->a, &w->pp, &w->q, &w->pb, &w->qb, &w->ab, &w->dt};
  for (auto q : xs) *q = (double2*)take(fx * 16);
  double2** ys[4] = {&w->y1b, &w->bm, &w->bb, &w->rb};
  for (auto q : ys) *q = (double2*)take(fy * 16);
  double2** gs[11] = {&w->gy, &w->gyi, &w->gx, &w->gxi, &w->gyib, &w->gxib, &w->gyb, &w->gxb, &w->S, &w->T, &w->tmp};
  for (auto q : gs) *q = (double2*)take(g * 16);
  w->htab = (double*)take(2 * (size_t)p.n1 * 8);
  w->part = (double*)take(wpart * 8);
  w->flag = (int*)take(64);
}

void adjoint_set_attr(int r) {
  if (pinvy_lds_bytes(r) > 65536)
    (void)hipFuncSetAttribute((const void*)k_adj_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pinvy_lds_bytes(r));
}

static void inv(const Plan& p, const AdjWork& w, const double2* g, double2* gi) {
  k_adj_inv<<<p.nb, 256, pinvy_lds_bytes(p.r), p.stream>>>(g, gi, p.r, w.flag);
}

static void wdot_add(const Plan& p, const AdjWork& w, const double2* A, const double2* B, long per, double coef,
                     double* theta, int k) {
  k_adj_wdot<<<ADJ_DOT_BLOCKS, 256, 0, p.stream>>>(A, B, per, p.nb, p.n3, w.part);
  k_adj_reduce1<<<1, 256, 0, p.stream>>>(w.part, ADJ_DOT_BLOCKS, coef, theta, k);
}

template <typename T>
static void happly(const Plan& p, const T* x, double2* out, double a, double c) {
  const long total = (long)p.nb * p.r * p.n1;
  k_adj_happly<T><<<(unsigned)((total + 255) / 256), 256, 0, p.stream>>>(x, out, p.n1, total, a, c);
}

static void hsolve(const Plan& p, const AdjWork& w, const double2* x, double2* y) {
  const long ncol = (long)p.nb * p.r;
  k_adj_hsolve<<<(unsigned)((ncol + 63) / 64), 64, 0, p.stream>>>(x, y, p.n1, ncol, p.rho1, w.htab);
}

static void herm(const Plan& p, const double2* g, double2* s) {
  const long n = (long)p.nb * p.r * p.r;
  k_adj_herm<<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>(g, s, p.r, p.nb);
}

template <typename T>
static void tube_inv(const Plan& p, const T* in, long ibs, long ips, long iqs, double* out, long osp, long osq, int P,
                     int Q, double s) {
  const long n = (long)P * Q * p.n3;
  k_adj_tube_inv<T><<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>(in, ibs, ips, iqs, out, osp, osq, P, Q, p.n3,
                                                                      p.nb, s);
}

void launch_adjoint_step(const Plan& p, const AdjWork& w, const AdjState& in, const AdjState& out, double2* xt_bar,
                         double2* yt_bar, double* w_bar, double* theta) {
  const int n1 = p.n1, n2 = p.n2, n3 = p.n3, r = p.r, nb = p.nb;
  const long fx = (long)nb * r * n1, fy = (long)nb * r * n2;
  const cd one = cd_make(1.0, 0.0), zero = cd_make(0.0, 0.0), mone = cd_make(-1.0, 0.0);
  const double eta = p.eta;
  // matrix views of the forward values (FP32): X [nb][r][n1] as n1 x r, Y [nb][r][n2] as
  // r x n2, W~ [n1][nb][n2] as n1 x n2
  const CView X = view(in.xt, (long)r * n1, 1, n1, 1), Y = view(in.yt, (long)r * n2, n2, 1, 1);
  const CView Wt = view(in.wt, n2, (long)nb * n2, 1, 1);
  const CView X1 = view(out.xt, (long)r * n1, 1, n1, 1), Y1 = view(out.yt, (long)r * n2, n2, 1, 1);
  (void)X;
  auto xv = [&](const double2* a) { return view(a, (long)r * n1, 1, n1, 0); };      // n1 x r, [nb][r][n1]
  auto yv = [&](const double2* a) { return view(a, (long)r * n2, n2, 1, 0); };      // r x n2
  auto gv = [&](const double2* a) { return view(a, (long)r * r, r, 1, 0); };        // r x r
  auto hv = [&](const double2* a) { return view(a, (long)n1 * n2, n2, 1, 0); };     // n1 x n2, [nb][n1][n2]

  k_adj_flag_zero<<<1, 64, 0, p.stream>>>(w.flag);
  k_adj_htab<<<1, 64, 0, p.stream>>>(n1, p.rho1, w.htab);
  // W+ in the spatial domain, from its stored spectrum
  tube_inv<float2>(p, out.wt, n2, (long)nb * n2, 1, w.w1s, (long)n2 * n3, n3, n1, n2, 1.0 / n3);
  // step 4: W-step adjoint -> z_bar, and the mu, rho2 adjoints
  const int wblk = (int)(((long)n1 * n3 + 255) / 256);
  k_adj_wstep<<<wblk, 256, 0, p.stream>>>(w_bar, w.w1s, p.gp, w.zbar, w.cbuf, n1, n2, n3, p.mu, p.rho2, p.g_rows,
                                          w.part);
  k_adj_reduce2<<<1, 256, 0, p.stream>>>(w.part, wblk, theta, 0, 2);
  // step 3: Z~_bar = ifft(Z_bar) on the stored frequencies; X~+_bar += Z~_bar Y~+^*,
  // Y~+_bar += X~+^* Z~_bar
  {
    const long n = (long)n1 * n2 * nb;
    k_adj_tube_fwd<<<(unsigned)((n + 255) / 256), 256, 0, p.stream>>>(w.zbar, (long)n2 * n3, n3, w.ztb,
                                                                      (long)n1 * n2, n2, 1, n1, n2, n3, nb,
                                                                      1.0 / n3);
  }
  axpby(p, fx, 1.0, xt_bar, 0.0, nullptr, w.x1b);
  axpby(p, fy, 1.0, yt_bar, 0.0, nullptr, w.y1b);
  gemm(p, n1, r, n2, one, hv(w.ztb), ctr(Y1), one, w.x1b, (long)r * n1, 1, n1);
  gemm(p, r, n2, n1, one, ctr(X1), hv(w.ztb), one, w.y1b, (long)r * n2, n2, 1);
  // step 2: Y~+ = (1 - eta) Y~ + eta G_X^{-1} B,  B = X~+^* W~,  G_X = X~+^* H_rho1 X~+
  realbins(p, w.y1b, (long)r * n2);
  axpby(p, fy, 1.0 - eta, w.y1b, 0.0, nullptr, yt_bar);
  axpby(p, fy, eta, w.y1b, 0.0, nullptr, w.rb);
  happly<float2>(p, (const float2*)out.xt, w.hx1, 1.0, p.rho1);
  gemm(p, r, r, n1, one, ctr(X1), xv(w.hx1), zero, w.gx, (long)r * r, r, 1);
  inv(p, w, w.gx, w.gxi);
  gemm(p, r, n2, n1, one, ctr(X1), Wt, zero, w.bm, (long)r * n2, n2, 1);
  gemm(p, r, r, n2, one, yv(w.rb), ctr(yv(w.bm)), zero, w.gxib, (long)r * r, r, 1);
  gemm(p, r, n2, r, one, ctr(gv(w.gxi)), yv(w.rb), zero, w.bb, (long)r * n2, n2, 1);
  gemm(p, r, r, r, one, ctr(gv(w.gxi)), gv(w.gxib), zero, w.tmp, (long)r * r, r, 1);
  gemm(p, r, r, r, mone, gv(w.tmp), ctr(gv(w.gxi)), zero, w.gxb, (long)r * r, r, 1);
  gemm(p, n1, r, n2, one, Wt, ctr(yv(w.bb)), one, w.x1b, (long)r * n1, 1, n1);
  gemm(p, n1, n2, r, one, X1, yv(w.bb), zero, w.wtb, (long)n1 * n2, n2, 1);
  herm(p, w.gxb, w.S);
  gemm(p, n1, r, r, one, xv(w.hx1), gv(w.S), one, w.x1b, (long)r * n1, 1, n1);
  happly<float2>(p, (const float2*)out.xt, w.dt, 0.0, 1.0);
  gemm(p, r, r, n1, one, ctr(X1), xv(w.dt), zero, w.T, (long)r * r, r, 1);
  wdot_add(p, w, w.gxb, w.T, (long)r * r, 1.0, theta, 1);
  // step 1: X~+ = (1 - eta) X~ + eta Q,  Q = H_rho1^{-1} P,  P = A G_Y^{-1},  A = W~ Y~^*
  realbins(p, w.x1b, (long)r * n1);
  axpby(p, fx, 1.0 - eta, w.x1b, 0.0, nullptr, xt_bar);
  axpby(p, fx, eta, w.x1b, 0.0, nullptr, w.qb);
  gemm(p, r, r, n2, one, Y, ctr(Y), zero, w.gy, (long)r * r, r, 1);
  inv(p, w, w.gy, w.gyi);
  gemm(p, n1, r, n2, one, Wt, ctr(Y), zero, w.a, (long)r * n1, 1, n1);
  gemm(p, n1, r, r, one, xv(w.a), gv(w.gyi), zero, w.pp, (long)r * n1, 1, n1);
  hsolve(p, w, w.pp, w.q);
  hsolve(p, w, w.qb, w.pb);
  happly<double2>(p, w.q, w.dt, 0.0, 1.0);
  wdot_add(p, w, w.pb, w.dt, (long)r * n1, -1.0, theta, 1);
  gemm(p, n1, r, r, one, xv(w.pb), ctr(gv(w.gyi)), zero, w.ab, (long)r * n1, 1, n1);
  gemm(p, r, r, n1, one, ctr(xv(w.a)), xv(w.pb), zero, w.gyib, (long)r * r, r, 1);
  gemm(p, r, r, r, one, ctr(gv(w.gyi)), gv(w.gyib), zero, w.tmp, (long)r * r, r, 1);
  gemm(p, r, r, r, mone, gv(w.tmp), ctr(gv(w.gyi)), zero, w.gyb, (long)r * r, r, 1);
  gemm(p, n1, n2, r, one, xv(w.ab), Y, one, w.wtb, (long)n1 * n2, n2, 1);
  gemm(p, r, n2, n1, one, ctr(xv(w.ab)), Wt, one, yt_bar, (long)r * n2, n2, 1);
  herm(p, w.gyb, w.S);
  gemm(p, r, n2, r, one, gv(w.S), Y, one, yt_bar, (long)r * n2, n2, 1);
  // step 7 of the previous iteration: W~ = dft(W), so W_bar = sum_b c_b Re(omega^{-b l} W~_bar_b)
  tube_inv<double2>(p, w.wtb, (long)n1 * n2, n2, 1, w_bar, (long)n2 * n3, n3, n1, n2, 1.0);
}

void launch_adjoint_initial(const Plan& p, const double2* xt_bar, const double2* yt_bar, double* x0_bar,
                            double* y0_bar) {
  const int n1 = p.n1, n2 = p.n2, n3 = p.n3, r = p.r;
  // X~ [nb][r][n1] -> X0 [n1][r][n3];  Y~ [nb][r][n2] -> Y0 [r][n2][n3]
  if (x0_bar) tube_inv<double2>(p, xt_bar, (long)r * n1, 1, n1, x0_bar, (long)r * n3, n3, n1, r, 1.0);
  if (y0_bar) tube_inv<double2>(p, yt_bar, (long)r * n2, n2, 1, y0_bar, (long)n2 * n3, n3, r, n2, 1.0);
}

void launch_objective_gradient(const Plan& p, const AdjWork& w, double* x_grad, double* y_grad) {
  const int n1 = p.n1, n2 = p.n2, n3 = p.n3, r = p.r, nb = p.nb;
  const cd one = cd_make(1.0, 0.0), zero = cd_make(0.0, 0.0), mone = cd_make(-1.0, 0.0);
  const CView X = view(p.xt, (long)r * n1, 1, n1, 1), Y = view(p.yt, (long)r * n2, n2, 1, 1);
  const CView Wt = view(p.wt, n2, (long)nb * n2, 1, 1);
  auto xv = [&](const double2* a) { return view(a, (long)r * n1, 1, n1, 0); };
  auto gv = [&](const double2* a) { return view(a, (long)r * r, r, 1, 0); };
  // grad_X = H_rho1 X~ G_Y - W~ Y~^*,  grad_Y = G_X Y~ - X~^* W~  (eq. (hkXYDer))
  happly<float2>(p, p.xt, w.hx1, 1.0, p.rho1);
  gemm(p, r, r, n2, one, Y, ctr(Y), zero, w.gy, (long)r * r, r, 1);
  gemm(p, n1, r, n2, mone, Wt, ctr(Y), zero, w.a, (long)r * n1, 1, n1);
  gemm(p, n1, r, r, one, xv(w.hx1), gv(w.gy), one, w.a, (long)r * n1, 1, n1);
  gemm(p, r, r, n1, one, ctr(X), xv(w.hx1), zero, w.gx, (long)r * r, r, 1);
  gemm(p, r, n2, n1, mone, ctr(X), Wt, zero, w.bm, (long)r * n2, n2, 1);
  gemm(p, r, n2, r, one, gv(w.gx), Y, one, w.bm, (long)r * n2, n2, 1);
  // d f0 / d X = Re idft(grad_X): the inverse transform with the 1 / n3 of eq. (barAAk)
  tube_inv<double2>(p, w.a, (long)r * n1, 1, n1, x_grad, (long)r * n3, n3, n1, r, 1.0 / n3);
  tube_inv<double2>(p, w.bm, (long)r * n2, n2, 1, y_grad, (long)n2 * n3, n3, r, n2, 1.0 / n3);
}

}  // namespace tctf

// The slice kernel: for one OD row i (a horizontal slice, n2 x n3) it
//   1. brings Z~(i,:,b) back to the tube domain (eq. (barAAk), step 3 of the algorithm box),
//   2. solves the W-step of every row (i, k) along mode 2 (eq. (subquKKT) / eq. (Wkiom), step 4),
//   3. transforms W(i,:,:) along the tube (eq. (bar BA-k), step 7) and stores W~(i,:,b),
// and emits the FP64 partial sums of the objective terms it can see (fit, ridge, K term).
//
// Thread roles: as "tube" threads, the block's threads take the tubes (i, j, :) in turn
// and hold one in registers for a transform; as "row" threads they take the rows (i, :, k)
// for the W-step.  The slice passes between the two roles through LDS (row stride n3 + 1
// floats, conflict-free).
//
// W-step of a row: observed entries are fixed (w_j = g_j); the unobserved ones solve
//   (1 + mu + rho2 deg_j) w_j - rho2 (w_{j-1} + w_{j+1}) = z_j,
// a tridiagonal system with the observed neighbours on the right-hand side.  Thomas
// elimination needs no pivoting (strict diagonal dominance); its reciprocal pivots depend
// only on the run position, so they come from the precomputed table, and each pass is one
// dependent multiply-add per entry:
//   forward  y_j = (z_j + rho2 y_{j-1}) / alpha_j      (y = g on observed entries)
//   backward w_j = y_j + rho2 / alpha_j * w_{j+1}       (w = g on observed entries)
#include "kernels.h"
#include "tube_dft_gen.h"

namespace tctf {

#define SLICE_THREADS 256

struct SliceArgs {
  const float2* zt;
  const float* gp;
  const float* wtab;
  void* wt;
  double* slice_obj;
  double* kkt;
  float* w_out;
  float* z_out;
  int n1, n2, nb;
  float rho2;
  double mu, rho2d;
  int mode, mixed, w_from_g;
};

template <int N>
__device__ __forceinline__ void load_inverse_tube(const float2* __restrict__ zt, size_t i, int j, int nb, int n2,
                                                  float (&z)[N]) {
  constexpr int NB = N / 2 + 1;
  float re[NB], im[NB];
  const float2* src = zt + i * nb * n2 + j;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const float2 v = src[(size_t)b * n2];
    re[b] = v.x;
    im[b] = v.y;
  }
  tube_inv<N>(re, im, z);
}

template <int N>
__global__ void __launch_bounds__(SLICE_THREADS) k_slice(SliceArgs a) {
  constexpr int NB = N / 2 + 1;
  constexpr int LD = N + 1;
  extern __shared__ float smem[];
  const int n2 = a.n2;
  float* zs = smem;                         // [n2][N+1]
  float* tab = smem + (size_t)n2 * LD;      // [4][n2]
  const size_t red_off = (size_t)n2 * LD + 4 * (size_t)n2;
  double* red = (double*)(smem + red_off + (red_off & 1));
  const size_t i = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const bool thomas = !(a.mode == SLICE_INIT || a.w_from_g);
  const float* gslice = a.gp + i * n2 * N;

  for (int e = tid; e < 4 * n2; e += nt) tab[e] = a.wtab[e];

  // ---- 1. inverse transform of Z~(i, j, :) (skipped when W is P_Omega(G) only)
  const bool need_z = !(a.mode == SLICE_RESULT && a.w_from_g && a.z_out == nullptr);
  for (int j = tid; j < n2; j += nt) {
    float z[N];
    if (need_z) {
      load_inverse_tube<N>(a.zt, i, j, a.nb, n2, z);
    } else {
#pragma unroll
      for (int q = 0; q < N; ++q) z[q] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) zs[j * LD + q] = z[q];
    if (a.z_out) {
      float* dst = a.z_out + (i * n2 + j) * N;
#pragma unroll
      for (int q = 0; q < N; ++q) dst[q] = z[q];
    }
  }
  __syncthreads();

  // ---- 2. W-step along mode 2 for the rows (i, :, k); the fit term of observed entries
  //         (and, for W = P_Omega(G), of all entries) is taken while Z is still in LDS
  double fit = 0.0, ridge = 0.0, sm = 0.0;
  for (int k = tid; k < N; k += nt) {
    const float* g = gslice + k;
    if (!thomas) {
      for (int jj = 0; jj < n2; ++jj) {
        const float gv = g[(size_t)jj * N];
        const float zv = zs[jj * LD + k];
        const float wv = is_unobserved(gv) ? 0.0f : gv;
        const double d = (double)zv - (double)wv;
        fit += d * d;
        zs[jj * LD + k] = wv;
      }
    } else {
      const float rho2 = a.rho2;
      float y = 0.0f;
      for (int jj = 0; jj < n2; ++jj) {
        const float gv = g[(size_t)jj * N];
        const float zv = zs[jj * LD + k];
        if (is_unobserved(gv)) {
          const int sel = (jj == n2 - 1 ? 2 : 0) + (unobs_starts_row(gv) ? 0 : 1);
          const float inv = tab[sel * n2 + unobs_pos(gv)];
          y = fmaf(rho2, y, zv) * inv;
        } else {
          const double d = (double)zv - (double)gv;
          fit += d * d;
          y = gv;
        }
        zs[jj * LD + k] = y;
      }
      float w = 0.0f;
      for (int jj = n2 - 1; jj >= 0; --jj) {
        const float gv = g[(size_t)jj * N];
        const float yv = zs[jj * LD + k];
        if (is_unobserved(gv) && jj < n2 - 1) {
          const int sel = unobs_starts_row(gv) ? 0 : 1;
          const float inv = tab[sel * n2 + unobs_pos(gv)];
          w = fmaf(rho2 * inv, w, yv);
        } else {
          w = yv;
        }
        zs[jj * LD + k] = w;
      }
    }
  }
  __syncthreads();

  // ---- 3. remaining objective terms and forward transform of W(i, j, :)
  // For an unobserved entry the W-step equation gives
  //   z_j - w_j = (mu + rho2 deg_j) w_j - rho2 (w_{j-1} + w_{j+1}),
  // so the fit term there is formed from W alone.
  for (int j = tid; j < n2; j += nt) {
    const float* wrow = zs + j * LD;
    const bool has_l = j > 0, has_r = j + 1 < n2;
    const double cj = a.mu + a.rho2d * ((has_l ? 1.0 : 0.0) + (has_r ? 1.0 : 0.0));
    const float* g = gslice + (size_t)j * N;
    if (a.mode == SLICE_KKT) {
      // residuals of eq. (subquKKT): unobserved (W K_{mu rho2} - Z)_ij, observed W - G
      float z[N];
      load_inverse_tube<N>(a.zt, i, j, a.nb, n2, z);
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const float gv = g[q];
        const double wq = wrow[q];
        if (is_unobserved(gv) && thomas) {
          const double l = has_l ? (double)wrow[q - LD] : 0.0;
          const double r = has_r ? (double)wrow[q + LD] : 0.0;
          fit = fmax(fit, fabs((1.0 + cj) * wq - a.rho2d * (l + r) - (double)z[q]));
        } else if (!is_unobserved(gv)) {
          ridge = fmax(ridge, fabs(wq - (double)gv));
        }
        sm = fmax(sm, fabs((double)z[q]));
      }
      continue;
    }
    for (int q = 0; q < N; ++q) {
      const double wq = wrow[q];
      ridge += wq * wq;
      const double r = has_r ? (double)wrow[q + LD] : 0.0;
      if (has_r) sm += (r - wq) * (r - wq);
      if (thomas && is_unobserved(g[q])) {
        const double l = has_l ? (double)wrow[q - LD] : 0.0;
        const double d = cj * wq - a.rho2d * (l + r);
        fit += d * d;
      }
    }
    if (a.mode == SLICE_RESULT) {
      if (a.w_out) {
        float* dst = a.w_out + (i * n2 + j) * N;
        for (int q = 0; q < N; ++q) dst[q] = wrow[q];
      }
    } else {
      float w[N], re[NB], im[NB];
#pragma unroll
      for (int q = 0; q < N; ++q) w[q] = wrow[q];
      tube_fwd<N>(w, re, im);
      if (a.mixed) {
        uint32_t* dst = (uint32_t*)a.wt + i * a.nb * n2 + j;
#pragma unroll
        for (int b = 0; b < NB; ++b) dst[(size_t)b * n2] = pack_bf16x2(re[b], im[b]);
      } else {
        float2* dst = (float2*)a.wt + i * a.nb * n2 + j;
#pragma unroll
        for (int b = 0; b < NB; ++b) dst[(size_t)b * n2] = make_float2(re[b], im[b]);
      }
    }
  }
  if (a.mode == SLICE_KKT) {
    fit = block_max_d(fit, red);
    ridge = block_max_d(ridge, red);
    sm = block_max_d(sm, red);
    if (tid == 0) {
      a.kkt[3 * i + 0] = fit;
      a.kkt[3 * i + 1] = ridge;
      a.kkt[3 * i + 2] = sm;
    }
  } else if (a.mode != SLICE_RESULT) {
    fit = block_sum_d(fit, red);
    ridge = block_sum_d(ridge, red);
    sm = block_sum_d(sm, red);
    if (tid == 0) {
      a.slice_obj[3 * i + 0] = fit;
      a.slice_obj[3 * i + 1] = ridge;
      a.slice_obj[3 * i + 2] = sm;
    }
  }
}

bool slice_supported(int n3) {
  switch (n3) {
#define TCTF_CASE(n) case n: return true;
    TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
    default: return false;
  }
}

size_t slice_lds_bytes(int n2, int n3) {
  return ((size_t)n2 * (n3 + 1) + 4 * (size_t)n2 + 2) * sizeof(float) + 16 * sizeof(double);
}

void slice_set_attr(int n3, size_t lds) {
  if (lds <= 65536) return;
  switch (n3) {
#define TCTF_CASE(n)                                                                                  \
  case n:                                                                                             \
    (void)hipFuncSetAttribute((const void*)k_slice<n>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    break;
    TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
    default: break;
  }
}

void launch_slice(const Plan& p, int mode, float* w_out, float* z_out, int w_from_g) {
  SliceArgs a;
  a.zt = p.zt;
  a.gp = p.gp;
  a.wtab = p.wtab;
  a.wt = p.wt;
  a.slice_obj = p.slice_obj;
  a.kkt = p.kkt;
  a.w_out = w_out;
  a.z_out = z_out;
  a.n1 = p.n1;
  a.n2 = p.n2;
  a.nb = p.nb;
  a.rho2 = (float)p.rho2;
  a.mu = p.mu;
  a.rho2d = p.rho2;
  a.mode = mode;
  a.mixed = p.mixed;
  a.w_from_g = w_from_g;
  const int need = p.n2 > p.n3 ? p.n2 : p.n3;
  int threads = ((need + 63) / 64) * 64;
  if (threads > SLICE_THREADS) threads = SLICE_THREADS;
  const size_t lds = slice_lds_bytes(p.n2, p.n3);
  switch (p.n3) {
#define TCTF_CASE(n)                                                                   \
  case n:                                                                              \
    k_slice<n><<<p.n1, threads, lds, p.stream>>>(a);                                   \
    break;
    TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
    default: break;
  }
}

}  // namespace tctf

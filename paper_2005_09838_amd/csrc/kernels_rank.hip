// Step 5 of the algorithm box: adjust the rank vector r^(l+1) and the factor sizes.  The
// paper gives no rule; this library keeps, in every stored frequency b, the components of
// Z~_b = X~_b Y~_b whose singular values exceed tol times the largest singular value over
// all frequencies, and zeroes the rest of the factors (their size stays r; the
// pseudo-inverse steps of eq. (updataXYW1) then keep the zero part zero).
//
// The singular values come from r x r Grams in FP64, never from an n1 x n2 matrix: with
// A = X~^* X~, B = Y~ Y~^* = V D V^*, S = B^{1/2} = V D^{1/2} V^* and S+ = V D^{+1/2} V^*
// (eigenvalues below r eps64 max D dropped, as Lemma SVPMPI's rule does), Y^ = S+ Y~ has
// orthonormal rows on the range of B and Z~ = (X~ S) Y^; (X~ S)^*(X~ S) = S A S = Q L Q^*
// gives the singular values sqrt(L) and Z~ = (X~ S Q) (Q^* Y^).  The factors become
// X~ <- X~ (S Q P), Y~ <- (P Q^* S+) Y~ with P keeping the first r_b columns in descending
// singular value order.
#include "kernels.h"
#include "pinv.h"

namespace tctf {

static __host__ __device__ inline size_t rank_lds_bytes(int r) {
  return (size_t)(8 * r * r + 2 * r) * sizeof(cd) + 144 * sizeof(double) + 64 * sizeof(int);
}

// One block per stored frequency b: sig[b][s] (descending), T_x = S Q and T_y = Q^* S+ in
// the same column / row order.
__global__ void __launch_bounds__(256) k_rank_svd(const float2* __restrict__ xt, const float2* __restrict__ yt,
                                                  int n1, int n2, int r, double* __restrict__ sig,
                                                  cd* __restrict__ tx, cd* __restrict__ ty) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, rr = r * r;
  cd* A = (cd*)sm;
  cd* B = A + rr;
  cd* S = B + rr;
  cd* Si = S + rr;
  cd* Mm = Si + rr;
  cd* Qv = Mm + rr;
  PinvScratch ps;
  ps.work = Qv + rr;
  ps.vec = ps.work + rr;
  ps.colk = ps.vec + rr;
  ps.rowk = ps.colk + r;
  ps.rot = (double*)(ps.rowk + r);
  ps.red = ps.rot + 96;
  int* order = (int*)(ps.red + 48);
  const float2* X = xt + (size_t)b * r * n1;
  const float2* Y = yt + (size_t)b * r * n2;
  for (int e = tid; e < rr; e += nt) {
    const int s = e / r, t = e % r;
    cd a = cd_make(0.0, 0.0), g = cd_make(0.0, 0.0);
    for (int i = 0; i < n1; ++i) {   // A(s, t) = sum_i conj(X(i, s)) X(i, t)
      const float2 u = X[(size_t)s * n1 + i], v = X[(size_t)t * n1 + i];
      cd_fma(a, cd_make(u.x, -u.y), cd_make(v.x, v.y));
    }
    for (int j = 0; j < n2; ++j) {   // B(s, t) = sum_j Y(s, j) conj(Y(t, j))
      const float2 u = Y[(size_t)s * n2 + j], v = Y[(size_t)t * n2 + j];
      cd_fma(g, cd_make(u.x, u.y), cd_make(v.x, -v.y));
    }
    A[e] = a;
    B[e] = g;
  }
  __syncthreads();
  // B = V D V^*  ->  S = V D^{1/2} V^*, Si = V D^{+1/2} V^*
  double f2 = 0.0;
  for (int e = tid; e < rr; e += nt) f2 += B[e].re * B[e].re + B[e].im * B[e].im;
  f2 = block_sum_d(f2, ps.red);
  jacobi_herm(B, r, sqrt(f2), ps);
  double dmax = 0.0;
  for (int i = 0; i < r; ++i) dmax = fmax(dmax, ps.work[i * r + i].re);
  const double tau = r * TCTF_EPS64 * dmax;
  for (int e = tid; e < rr; e += nt) {
    const int p = e / r, q = e % r;
    cd s1 = cd_make(0.0, 0.0), s2 = cd_make(0.0, 0.0);
    for (int i = 0; i < r; ++i) {
      const double d = ps.work[i * r + i].re;
      if (d > tau) {
        const cd vv = cd_mulc(ps.vec[p * r + i], ps.vec[q * r + i]);   // V(p, i) conj(V(q, i))
        s1 = cd_add(s1, cd_scale(vv, sqrt(d)));
        s2 = cd_add(s2, cd_scale(vv, 1.0 / sqrt(d)));
      }
    }
    S[e] = s1;
    Si[e] = s2;
  }
  __syncthreads();
  // M = S A S (Hermitian PSD)
  for (int e = tid; e < rr; e += nt) {   // Qv = A S (scratch)
    const int p = e / r, q = e % r;
    cd acc = cd_make(0.0, 0.0);
    for (int k = 0; k < r; ++k) cd_fma(acc, A[p * r + k], S[k * r + q]);
    Qv[e] = acc;
  }
  __syncthreads();
  f2 = 0.0;
  for (int e = tid; e < rr; e += nt) {
    const int p = e / r, q = e % r;
    cd acc = cd_make(0.0, 0.0);
    for (int k = 0; k < r; ++k) cd_fma(acc, S[p * r + k], Qv[k * r + q]);
    Mm[e] = acc;
    f2 += acc.re * acc.re + acc.im * acc.im;
  }
  f2 = block_sum_d(f2, ps.red);   // also orders the M stores before the decomposition
  jacobi_herm(Mm, r, sqrt(f2), ps);
  if (tid == 0) {   // descending order of the eigenvalues (selection sort, r <= 32)
    for (int i = 0; i < r; ++i) order[i] = i;
    for (int i = 0; i < r; ++i) {
      int best = i;
      for (int k = i + 1; k < r; ++k)
        if (ps.work[order[k] * r + order[k]].re > ps.work[order[best] * r + order[best]].re) best = k;
      const int t = order[i];
      order[i] = order[best];
      order[best] = t;
    }
  }
  __syncthreads();
  for (int i = tid; i < r; i += nt) sig[(size_t)b * r + i] = sqrt(fmax(ps.work[order[i] * r + order[i]].re, 0.0));
  // T_x(p, s) = sum_k S(p, k) Q(k, order[s]);  T_y(s, q) = sum_k conj(Q(k, order[s])) Si(k, q)
  for (int e = tid; e < rr; e += nt) {
    const int p = e / r, s = e % r, c = order[s];
    cd acc = cd_make(0.0, 0.0);
    for (int k = 0; k < r; ++k) cd_fma(acc, S[p * r + k], ps.vec[k * r + c]);
    tx[(size_t)b * rr + e] = acc;
  }
  for (int e = tid; e < rr; e += nt) {
    const int s = e / r, q = e % r, c = order[s];
    cd acc = cd_make(0.0, 0.0);
    for (int k = 0; k < r; ++k) cd_fma(acc, cd_conj(ps.vec[k * r + c]), Si[k * r + q]);
    ty[(size_t)b * rr + e] = acc;
  }
}

// smax over every frequency's singular values, then r_b = #{s : sig[b][s] > tol smax}.
__global__ void __launch_bounds__(256) k_rank_decide(const double* __restrict__ sig, int nb, int r, double tol,
                                                     int* __restrict__ ranks) {
  __shared__ double red[16];
  double m = 0.0;
  for (int e = threadIdx.x; e < nb * r; e += blockDim.x) m = fmax(m, sig[e]);
  m = block_max_d(m, red);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    int q = 0;
    for (int s = 0; s < r; ++s) q += (sig[(size_t)b * r + s] > tol * m) ? 1 : 0;
    ranks[b] = q;
  }
}

// In place: X~(b, :, i) <- X~(b, :, i) T_x P and Y~(b, :, j) <- P T_y Y~(b, :, j); one
// thread per factor row (b, i) of X~ or column (b, j) of Y~.  Imaginary parts of the real
// frequencies are set to 0.
template <int RM>
__global__ void __launch_bounds__(256) k_rank_apply(float2* __restrict__ xt, float2* __restrict__ yt, int n1, int n2,
                                                    int r, int nb, int n3, const cd* __restrict__ tx,
                                                    const cd* __restrict__ ty, const int* __restrict__ ranks) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nx = (long)nb * n1, ny = (long)nb * n2;
  if (g >= nx + ny) return;
  const bool isx = g < nx;
  const long h = isx ? g : g - nx;
  const int n = isx ? n1 : n2;
  const int b = (int)(h / n), i = (int)(h % n);
  float2* base = (isx ? xt + (size_t)b * r * n1 : yt + (size_t)b * r * n2) + i;
  const cd* T = (isx ? tx : ty) + (size_t)b * r * r;
  const int q = ranks[b];
  const bool real = bin_is_real(b, n3);
  cd v[RM];
#pragma unroll
  for (int t = 0; t < RM; ++t) {
    if (t < r) {
      const float2 f = base[(size_t)t * n];
      v[t] = cd_make(f.x, f.y);
    }
  }
  for (int s = 0; s < r; ++s) {
    cd acc = cd_make(0.0, 0.0);
    if (s < q) {
#pragma unroll
      for (int t = 0; t < RM; ++t) {
        if (t < r) cd_fma(acc, isx ? v[t] : T[(size_t)s * r + t], isx ? T[(size_t)t * r + s] : v[t]);
      }
    }
    base[(size_t)s * n] = make_float2((float)acc.re, real ? 0.0f : (float)acc.im);
  }
}

// After the rotation: G_Y = Y~ Y~^* into partial slot 0 of every frequency (slots 1.. zero)
// for the pseudo-inverse of the next X-step, and (H X~)^*(H X~) <- T^* D T with T = T_x P
// (the rho1 term of f0 at the adjusted factors).
__global__ void __launch_bounds__(256) k_rank_grams(const float2* __restrict__ yt, int n2, int r, int ny,
                                                    cd* __restrict__ gym, cd* __restrict__ dmat,
                                                    const cd* __restrict__ tx, const int* __restrict__ ranks) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, rr = r * r;
  cd* D = (cd*)sm;
  cd* DT = D + rr;
  const int q = ranks[b];
  const float2* Y = yt + (size_t)b * r * n2;
  for (int e = tid; e < rr; e += nt) {
    const int s = e / r, t = e % r;
    cd g = cd_make(0.0, 0.0);
    for (int j = 0; j < n2; ++j) {
      const float2 u = Y[(size_t)s * n2 + j], v = Y[(size_t)t * n2 + j];
      cd_fma(g, cd_make(u.x, u.y), cd_make(v.x, -v.y));
    }
    gym[(size_t)b * ny * rr + e] = g;
    for (int k = 1; k < ny; ++k) gym[((size_t)b * ny + k) * rr + e] = cd_make(0.0, 0.0);
    D[e] = dmat[(size_t)b * rr + e];
  }
  __syncthreads();
  const cd* T = tx + (size_t)b * rr;
  for (int e = tid; e < rr; e += nt) {   // DT = D T P
    const int p = e / r, s = e % r;
    cd acc = cd_make(0.0, 0.0);
    if (s < q)
      for (int k = 0; k < r; ++k) cd_fma(acc, D[p * r + k], T[k * r + s]);
    DT[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < rr; e += nt) {   // (T P)^* D T P
    const int s = e / r, t = e % r;
    cd acc = cd_make(0.0, 0.0);
    if (s < q)
      for (int k = 0; k < r; ++k) cd_fma(acc, cd_conj(T[k * r + s]), DT[k * r + t]);
    dmat[(size_t)b * rr + e] = acc;
  }
}

__global__ void k_rank_fill(int* ranks, int nb, int r) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) ranks[b] = r;
}

void launch_rank_init(const Plan& p) { k_rank_fill<<<(p.nb + 255) / 256, 256, 0, p.stream>>>(p.ranks, p.nb, p.r); }

void rank_set_attr(int r) {
  if (rank_lds_bytes(r) > 65536)
    (void)hipFuncSetAttribute((const void*)k_rank_svd, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)rank_lds_bytes(r));
}

void launch_rank_adjust(const Plan& p, double tol) {
  k_rank_svd<<<p.nb, 256, rank_lds_bytes(p.r), p.stream>>>(p.xt, p.yt, p.n1, p.n2, p.r, p.rsig, p.rtx, p.rty);
  k_rank_decide<<<1, 256, 0, p.stream>>>(p.rsig, p.nb, p.r, tol, p.ranks);
  const long n = (long)p.nb * (p.n1 + p.n2);
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (p.r <= 8)
    k_rank_apply<8><<<grid, 256, 0, p.stream>>>(p.xt, p.yt, p.n1, p.n2, p.r, p.nb, p.n3, p.rtx, p.rty, p.ranks);
  else if (p.r <= 16)
    k_rank_apply<16><<<grid, 256, 0, p.stream>>>(p.xt, p.yt, p.n1, p.n2, p.r, p.nb, p.n3, p.rtx, p.rty, p.ranks);
  else
    k_rank_apply<32><<<grid, 256, 0, p.stream>>>(p.xt, p.yt, p.n1, p.n2, p.r, p.nb, p.n3, p.rtx, p.rty, p.ranks);
  k_rank_grams<<<p.nb, 256, 2 * (size_t)p.r * p.r * sizeof(cd), p.stream>>>(p.yt, p.n2, p.r, p.ny, p.gym, p.dmat,
                                                                           p.rtx, p.ranks);
  launch_pinvy(p, p.stream);
}

}  // namespace tctf

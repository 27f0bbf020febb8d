// Moore-Penrose inverse of a small Hermitian positive-semidefinite Gram matrix in FP64,
// computed cooperatively by one thread block (Lemma SVPMPI: A^+ = V diag(1/lambda) V^*
// over the kept eigenvalues).
//
// Rule: eigenvalues lambda_i <= tau = r * eps64 * lambda_max are dropped (a zero matrix
// gives 0).  Fast path: Gauss-Jordan elimination (the sweep operator, no pivoting, valid
// for positive-definite input).  Its result is accepted only if it proves that every
// eigenvalue exceeds 8 tau:  lambda_min >= 1/||A^-1||_F > 8 r eps ||A||_F >= 8 tau.
// Then the rule keeps every eigenvalue and A^+ = A^-1.  Otherwise (or when forced) a
// cyclic Jacobi eigen-decomposition with parallel (round-robin) pair ordering is used
// and the rule is applied to its eigenvalues.
#pragma once
#include "common.h"

#define TCTF_EPS64 2.220446049250313e-16

struct PinvScratch {
  cd* work;    // r*r
  cd* vec;     // r*r
  cd* colk;    // r
  cd* rowk;    // r
  double* rot; // 6 * 16 doubles (rotation parameters of one round)
  double* red; // >= 16 doubles
};

// Returns 1 (to every thread) if all eigenvalues were kept, 0 otherwise.
__device__ inline int pinv_herm(const cd* A, cd* P, int r, int force_eigen, PinvScratch s) {
  const int tid = threadIdx.x, nt = blockDim.x, rr = r * r;
  double f2 = 0.0, dmax = -1.0;
  for (int e = tid; e < rr; e += nt) {
    cd a = A[e];
    f2 += a.re * a.re + a.im * a.im;
    if (e / r == e % r) dmax = fmax(dmax, a.re);
  }
  f2 = block_sum_d(f2, s.red);
  dmax = block_max_d(dmax, s.red);
  if (!isfinite(f2)) {
    for (int e = tid; e < rr; e += nt) P[e] = cd_make(NAN, NAN);
    __syncthreads();
    return 0;
  }
  if (!(dmax > 0.0)) {   // PSD with a non-positive diagonal: the zero matrix
    for (int e = tid; e < rr; e += nt) P[e] = cd_make(0.0, 0.0);
    __syncthreads();
    return 0;
  }
  const double fro = sqrt(f2);

  if (!force_eigen) {
    for (int e = tid; e < rr; e += nt) s.work[e] = A[e];
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < r; ++k) {
      const double piv = s.work[k * r + k].re;
      if (!(piv > 0.0)) { ok = false; break; }            // uniform across the block
      for (int e = tid; e < r; e += nt) { s.colk[e] = s.work[e * r + k]; s.rowk[e] = s.work[k * r + e]; }
      __syncthreads();
      const double ip = 1.0 / piv;
      for (int e = tid; e < rr; e += nt) {
        const int p = e / r, q = e % r;
        cd v;
        if (p == k && q == k) v = cd_make(-ip, 0.0);
        else if (p == k) v = cd_scale(s.rowk[q], ip);
        else if (q == k) v = cd_scale(s.colk[p], ip);
        else v = cd_sub(s.work[e], cd_scale(cd_mul(s.colk[p], s.rowk[q]), ip));
        s.work[e] = v;
      }
      __syncthreads();
    }
    if (ok) {
      double g2 = 0.0;
      for (int e = tid; e < rr; e += nt) g2 += s.work[e].re * s.work[e].re + s.work[e].im * s.work[e].im;
      g2 = block_sum_d(g2, s.red);
      if (isfinite(g2) && 8.0 * r * TCTF_EPS64 * fro * sqrt(g2) < 1.0) {
        for (int e = tid; e < rr; e += nt) P[e] = cd_make(-s.work[e].re, -s.work[e].im);
        __syncthreads();
        return 1;
      }
    }
  }

  // Jacobi eigen-decomposition of A into work (eigenvalues on the diagonal) and vec.
  for (int e = tid; e < rr; e += nt) {
    s.work[e] = A[e];
    s.vec[e] = cd_make((e / r == e % r) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int rp = r + (r & 1), npair = rp / 2;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int e = tid; e < rr; e += nt)
      if (e / r != e % r) off += s.work[e].re * s.work[e].re + s.work[e].im * s.work[e].im;
    off = block_sum_d(off, s.red);
    if (sqrt(off) <= 1e-14 * fro) break;
    for (int m = 0; m < rp - 1; ++m) {
      // rotation parameters of every disjoint pair of this round
      for (int i = tid; i < npair; i += nt) {
        int p, q;
        if (i == 0) { p = rp - 1; q = m; }
        else { p = (m + i) % (rp - 1); q = (m - i + rp - 1) % (rp - 1); }
        if (p > q) { int t = p; p = q; q = t; }
        double* R = s.rot + 6 * i;
        R[0] = -1.0;   // p < 0 marks "no rotation"
        if (q < r) {
          const double a = s.work[p * r + p].re, d = s.work[q * r + q].re;
          const cd b = s.work[p * r + q];
          const double ab = hypot(b.re, b.im);
          if (ab > 1e-300 && ab > TCTF_EPS64 * 1e-3 * sqrt(fabs(a * d))) {
            const double ph_re = b.re / ab, ph_im = b.im / ab;
            const double zeta = (d - a) / (2.0 * ab);
            double t;
            if (fabs(zeta) > 1e150) t = 0.5 / zeta;
            else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
            R[0] = p; R[1] = q; R[2] = c; R[3] = sn; R[4] = ph_re; R[5] = ph_im;
          }
        }
      }
      __syncthreads();
      // columns: A <- A U and V <- V U with U_pp = c, U_pq = s, U_qp = -s conj(phi), U_qq = c conj(phi)
      for (int e = tid; e < npair * r; e += nt) {
        const double* R = s.rot + 6 * (e / r);
        if (R[0] < 0.0) continue;
        const int p = (int)R[0], q = (int)R[1], row = e % r;
        const double c = R[2], sn = R[3];
        const cd phc = cd_make(R[4], -R[5]);
        const cd upq = cd_make(sn, 0.0), uqp = cd_scale(phc, -sn), uqq = cd_scale(phc, c);
        for (int pass = 0; pass < 2; ++pass) {
          cd* M = pass ? s.vec : s.work;
          const cd xp = M[row * r + p], xq = M[row * r + q];
          M[row * r + p] = cd_add(cd_scale(xp, c), cd_mul(xq, uqp));
          M[row * r + q] = cd_add(cd_mul(xp, upq), cd_mul(xq, uqq));
        }
      }
      __syncthreads();
      // rows: A <- U^* A
      for (int e = tid; e < npair * r; e += nt) {
        const double* R = s.rot + 6 * (e / r);
        if (R[0] < 0.0) continue;
        const int p = (int)R[0], q = (int)R[1], col = e % r;
        const double c = R[2], sn = R[3];
        const cd ph = cd_make(R[4], R[5]);
        // conj(U_qp) = -s phi, conj(U_qq) = c phi
        const cd xp = s.work[p * r + col], xq = s.work[q * r + col];
        s.work[p * r + col] = cd_add(cd_scale(xp, c), cd_scale(cd_mul(xq, ph), -sn));
        s.work[q * r + col] = cd_add(cd_scale(xp, sn), cd_scale(cd_mul(xq, ph), c));
      }
      __syncthreads();
    }
  }
  double lmax = -1e300;
  for (int i = tid; i < r; i += nt) lmax = fmax(lmax, s.work[i * r + i].re);
  lmax = block_max_d(lmax, s.red);
  const double tau = fmax(r * TCTF_EPS64 * lmax, 0.0);
  int kept = 0;
  for (int i = 0; i < r; ++i) kept += (s.work[i * r + i].re > tau) ? 1 : 0;
  for (int e = tid; e < rr; e += nt) {
    const int p = e / r, q = e % r;
    cd acc = cd_make(0.0, 0.0);
    for (int i = 0; i < r; ++i) {
      const double l = s.work[i * r + i].re;
      if (l > tau) acc = cd_add(acc, cd_scale(cd_mulc(s.vec[p * r + i], s.vec[q * r + i]), 1.0 / l));
    }
    P[e] = acc;
  }
  __syncthreads();
  return kept == r ? 1 : 0;
}

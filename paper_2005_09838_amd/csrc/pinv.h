// Moore-Penrose inverse of a small Hermitian positive-semidefinite Gram matrix in FP64,
// computed cooperatively by one thread block (Lemma SVPMPI: A^+ = V diag(1/lambda) V^*
// over the kept eigenvalues).
//
// Rule: eigenvalues lambda_i <= tau = r * eps64 * lambda_max are dropped (a zero matrix
// gives 0).  Fast path: Gauss-Jordan elimination (the sweep operator, no pivoting, valid
// for positive-definite input); for r <= 16 the first wavefront runs it alone with the
// matrix in registers, for larger r the block runs it in LDS.  Its result
// is accepted only if it proves that every eigenvalue exceeds 8 tau:
// lambda_min >= 1/||A^-1||_F > 8 r eps ||A||_F >= 8 tau.  Then the rule keeps every
// eigenvalue and A^+ = A^-1.  Otherwise (or when forced) a cyclic Jacobi
// eigen-decomposition with parallel (round-robin) pair ordering is used by the whole block
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

// Wavefront-level fast path for r <= 16 (called by the 64 lanes of one wavefront).  The
// matrix, padded with the identity to 16 x 16, lives in registers: lane l holds row
// l / 4, columns 4 (l % 4) .. 4 (l % 4) + 3.  Pivot row, pivot column and pivot reach the
// lanes by cross-lane shuffles.
// Returns 1: accepted, P = A^-1;  2: A is not finite, P = NaN;  3: A has no positive
// diagonal entry (the zero PSD matrix), P = 0;  0: rejected, P untouched.
__device__ inline int pinv_gj_wave16(const cd* A, cd* P, int r) {
  const int lane = threadIdx.x & 63, p = lane >> 2, q0 = (lane & 3) * 4, rr = r * r;
  double vr[4], vi[4];
  double f2 = 0.0, dmax = -1.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = q0 + i;
    if (p < r && q < r) {
      const cd a = A[p * r + q];
      vr[i] = a.re;
      vi[i] = a.im;
      f2 += a.re * a.re + a.im * a.im;
      if (p == q) dmax = fmax(dmax, a.re);
    } else {
      vr[i] = (p == q) ? 1.0 : 0.0;
      vi[i] = 0.0;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    f2 += __shfl_xor(f2, off);
    dmax = fmax(dmax, __shfl_xor(dmax, off));
  }
  if (!isfinite(f2)) {
    for (int e = lane; e < rr; e += 64) P[e] = cd_make(NAN, NAN);
    return 2;
  }
  if (!(dmax > 0.0)) {
    for (int e = lane; e < rr; e += 64) P[e] = cd_make(0.0, 0.0);
    return 3;
  }
  bool ok = true;
  for (int k = 0; k < r; ++k) {
    const int ks = k & 3, src_row = 4 * k + (lane & 3), src_col = 4 * p + (k >> 2);
    double wr[4], wi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      wr[i] = __shfl(vr[i], src_row);   // (k, q0 + i)
      wi[i] = __shfl(vi[i], src_row);
    }
    const double ownr = ks == 0 ? vr[0] : ks == 1 ? vr[1] : ks == 2 ? vr[2] : vr[3];
    const double owni = ks == 0 ? vi[0] : ks == 1 ? vi[1] : ks == 2 ? vi[2] : vi[3];
    const double cr = __shfl(ownr, src_col), ci = __shfl(owni, src_col);   // (p, k)
    const double piv = __shfl(ownr, 4 * k + (k >> 2));                      // (k, k)
    ok = ok && piv > 0.0;   // the same in every lane; a failed pivot rejects the result
    const double ip = piv > 0.0 ? 1.0 / piv : 0.0;
    const bool isrow = p == k;
    // branch-free update: pivot -> -1/piv, pivot row -> w/piv, pivot column -> c/piv,
    // elsewhere v - c w / piv
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool iscol = q0 + i == k;
      const double gr = vr[i] - (cr * wr[i] - ci * wi[i]) * ip;
      const double gi = vi[i] - (cr * wi[i] + ci * wr[i]) * ip;
      const double nr = isrow ? (iscol ? -ip : wr[i] * ip) : (iscol ? cr * ip : gr);
      const double ni = isrow ? (iscol ? 0.0 : wi[i] * ip) : (iscol ? ci * ip : gi);
      vr[i] = nr;
      vi[i] = ni;
    }
  }
  if (!ok) return 0;
  double g2 = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (p < r && q0 + i < r) g2 += vr[i] * vr[i] + vi[i] * vi[i];
  for (int off = 32; off > 0; off >>= 1) g2 += __shfl_xor(g2, off);
  if (!(isfinite(g2) && 8.0 * r * TCTF_EPS64 * sqrt(f2) * sqrt(g2) < 1.0)) return 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (p < r && q0 + i < r) P[p * r + q0 + i] = cd_make(-vr[i], -vi[i]);
  return 1;
}

// Returns 1 (to every thread) if all eigenvalues were kept, 0 otherwise.
__device__ inline int pinv_herm(const cd* A, cd* P, int r, int force_eigen, PinvScratch s) {
  const int tid = threadIdx.x, nt = blockDim.x, rr = r * r;
  if (!force_eigen && r <= 16) {
    if (tid < 64) {
      const int f = pinv_gj_wave16(A, P, r);
      if (tid == 0) s.rot[0] = (double)f;
    }
    __syncthreads();
    const int f = (int)s.rot[0];
    __syncthreads();
    if (f == 1) return 1;
    if (f == 2 || f == 3) return 0;
  }
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

  if (!force_eigen && r > 16) {   // block-level Gauss-Jordan for the larger ranks
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

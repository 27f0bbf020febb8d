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
#include "kernels.h"

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
  // Sweeps on the 2 x 2 pivot blocks K = {k0, k0 + 1} (an odd r ends with a block that
  // holds one padding index; sweeping it leaves the leading r x r block unchanged):
  // A_KK -> -A_KK^-1, A_iK -> A_iK A_KK^-1, A_Kj -> A_KK^-1 A_Kj,
  // A_ij -> A_ij - A_iK A_KK^-1 A_Kj.  Sweeping every index yields -A^-1.
  bool ok = true;
  const int pin = p & 1;                     // this lane's row offset within a pivot block
  for (int k0 = 0; k0 < r; k0 += 2) {
    const int g = k0 >> 2, sl = k0 & 3;      // column group and slot of the pivot columns
    // pivot rows k0, k0 + 1 at this lane's columns
    double w0r[4], w0i[4], w1r[4], w1i[4];
    const int src0 = 4 * k0 + (lane & 3), src1 = src0 + 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      w0r[i] = __shfl(vr[i], src0);
      w0i[i] = __shfl(vi[i], src0);
      w1r[i] = __shfl(vr[i], src1);
      w1i[i] = __shfl(vi[i], src1);
    }
    // pivot columns k0, k0 + 1 of this lane's row (both in lane 4 p + g, slots sl, sl + 1)
    const double o0r = sl == 0 ? vr[0] : vr[2], o0i = sl == 0 ? vi[0] : vi[2];
    const double o1r = sl == 0 ? vr[1] : vr[3], o1i = sl == 0 ? vi[1] : vi[3];
    const int srcc = 4 * p + g;
    const double c0r = __shfl(o0r, srcc), c0i = __shfl(o0i, srcc);
    const double c1r = __shfl(o1r, srcc), c1i = __shfl(o1i, srcc);
    // the pivot block [[pa, pb], [conj(pb), pd]] from rows k0 and k0 + 1
    const int sp0 = 4 * k0 + g, sp1 = sp0 + 4;
    const double pa = __shfl(o0r, sp0), pbr = __shfl(o1r, sp0), pbi = __shfl(o1i, sp0);
    const double pd = __shfl(o1r, sp1);
    const double det = pa * pd - (pbr * pbr + pbi * pbi);
    ok = ok && pa > 0.0 && det > 0.0;        // the same in every lane
    const double idet = det > 0.0 ? 1.0 / det : 0.0;
    // A_KK^-1 = [[e00, e01], [e10, e11]]
    const double e00 = pd * idet, e11 = pa * idet;
    const double e01r = -pbr * idet, e01i = -pbi * idet;   // -pb / det
    const double e10r = -pbr * idet, e10i = pbi * idet;    // -conj(pb) / det
    // (R0, R1) = A_pK A_KK^-1 for this lane's row
    const double r0r = c0r * e00 + (c1r * e10r - c1i * e10i), r0i = c0i * e00 + (c1r * e10i + c1i * e10r);
    const double r1r = (c0r * e01r - c0i * e01i) + c1r * e11, r1i = (c0r * e01i + c0i * e01r) + c1i * e11;
    const bool inrow = (p >> 1) == (k0 >> 1);   // p is k0 or k0 + 1
    // this lane's pivot-block row of A_KK^-1: (f0, f1) = row (p - k0)
    const double f0r = pin ? e10r : e00, f0i = pin ? e10i : 0.0;
    const double f1r = pin ? e11 : e01r, f1i = pin ? 0.0 : e01i;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + i;
      const bool incol = (q >> 1) == (k0 >> 1);
      const int qin = q & 1;
      // general entry: v - R0 w0 - R1 w1
      const double gr = vr[i] - (r0r * w0r[i] - r0i * w0i[i]) - (r1r * w1r[i] - r1i * w1i[i]);
      const double gi = vi[i] - (r0r * w0i[i] + r0i * w0r[i]) - (r1r * w1i[i] + r1i * w1r[i]);
      // pivot rows: f0 w0 + f1 w1
      const double hr = (f0r * w0r[i] - f0i * w0i[i]) + (f1r * w1r[i] - f1i * w1i[i]);
      const double hi = (f0r * w0i[i] + f0i * w0r[i]) + (f1r * w1i[i] + f1i * w1r[i]);
      // pivot columns: R_qin; pivot block: -(A_KK^-1)_(p - k0, q - k0) = -f_qin
      const double cr = qin ? r1r : r0r, ci = qin ? r1i : r0i;
      const double br = qin ? -f1r : -f0r, bi = qin ? -f1i : -f0i;
      vr[i] = inrow ? (incol ? br : hr) : (incol ? cr : gr);
      vi[i] = inrow ? (incol ? bi : hi) : (incol ? ci : gi);
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

// Cyclic Jacobi eigen-decomposition of a Hermitian r x r matrix A by the whole block, with
// parallel (round-robin) pair ordering: on return s.work holds the rotated matrix (the
// eigenvalues on its diagonal, unsorted) and s.vec the eigenvectors as columns.  fro is
// ||A||_F (the sweeps stop when the off-diagonal part falls below 1e-14 fro).
__device__ inline void jacobi_herm(const cd* A, int r, double fro, PinvScratch s) {
  const int tid = threadIdx.x, nt = blockDim.x, rr = r * r;
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
  jacobi_herm(A, r, fro, s);
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

// Bytes of LDS pinvy_block needs at rank r.
__host__ __device__ inline size_t pinvy_lds_bytes(int r) {
  return (size_t)(4 * r * r + 2 * r) * sizeof(cd) + 144 * sizeof(double);
}

// Inputs and outputs of pinvy_block ([nb][r][r] FP64 complex unless noted).
struct PinvyArgs {
  const cd* gyq;      // [nb][ny][r][r] partial Grams of Y~ over column blocks
  int ny;
  const cd* dmat;     // (H X~)^*(H X~)
  double* bin_obj;    // [nb] c_b tr((H X~)^*(H X~) G_Y): the rho1 term of eq. (fun-XYW)
  int n3;
  cd* gyp;            // G_Y^+
  cd* qy;             // I - eta P_Y
  int* qy_zero;       // [nb] 1 when I - eta P_Y is exactly 0
  int r;
  double eta;
  int force_eigen;
};

static inline PinvyArgs pinvy_args(const tctf::Plan& p) {
  PinvyArgs a;
  a.gyq = p.gym;
  a.ny = p.ny;
  a.dmat = p.dmat;
  a.bin_obj = p.bin_obj;
  a.n3 = p.n3;
  a.gyp = p.gyp;
  a.qy = p.qy;
  a.qy_zero = p.qy_zero;
  a.r = p.r;
  a.eta = p.eta;
  a.force_eigen = p.force_eigen;
  return a;
}

// Per frequency b, by a whole block: G_Y as the sum of the column-block partials (fixed
// order), the objective term c_b tr(D G_Y), G_Y^+ and, unless it is exactly 0,
// q = I - eta G_Y G_Y^+ for the next X-update (first line of eq. (updataXYW1)); qy_zero[b] = 1
// marks q = 0.  sm: pinvy_lds_bytes(r) bytes of LDS.
__device__ inline void pinvy_block(int b, const PinvyArgs& a, unsigned char* sm) {
  const int tid = threadIdx.x, nt = blockDim.x, r = a.r, rr = r * r;
  cd* gy = (cd*)sm;
  cd* gp = gy + rr;
  PinvScratch ps;
  ps.work = gp + rr;
  ps.vec = ps.work + rr;
  ps.colk = ps.vec + rr;
  ps.rowk = ps.colk + r;
  ps.rot = (double*)(ps.rowk + r);
  ps.red = ps.rot + 96;
  double tr = 0.0;
  for (int e = tid; e < rr; e += nt) {
    cd g = a.gyq[(size_t)b * a.ny * rr + e];
    for (int k = 1; k < a.ny; ++k) g = cd_add(g, a.gyq[((size_t)b * a.ny + k) * rr + e]);
    gy[e] = g;
    const cd d = a.dmat[(size_t)b * rr + (e % r) * r + e / r];   // D(t, s) for G_Y(s, t)
    tr += d.re * g.re - d.im * g.im;
  }
  tr = block_sum_d(tr, ps.red);   // also orders the G_Y stores before their reads
  if (tid == 0) a.bin_obj[b] = bin_weight(b, a.n3) * tr;
  const int fully = pinv_herm(gy, gp, r, a.force_eigen, ps);
  const bool qyz = fully && a.eta == 1.0;
  for (int e = tid; e < rr; e += nt) {
    cd qv = cd_make(0.0, 0.0);
    if (!qyz) {
      const int s = e / r, t = e % r;
      cd acc = cd_make(0.0, 0.0);
      for (int u = 0; u < r; ++u) cd_fma(acc, gy[s * r + u], gp[u * r + t]);
      qv = cd_make((s == t ? 1.0 : 0.0) - a.eta * acc.re, -a.eta * acc.im);
    }
    a.qy[(size_t)b * rr + e] = qv;
    a.gyp[(size_t)b * rr + e] = gp[e];
  }
  if (tid == 0) a.qy_zero[b] = qyz ? 1 : 0;
}

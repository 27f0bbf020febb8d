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
// only on the position in the run of unobserved entries (and on whether the run starts
// at the first slot), so they come from the precomputed table.  The row's observed flags
// sit in an LDS bitmask; the forward pass counts the run position, the backward pass
// recovers each run's start from the flags.  Each pass is one dependent multiply-add per
// entry, entirely in LDS:
//   forward  y_j = (z_j + rho2 y_{j-1}) / alpha_j      (y = g on observed entries)
//   backward w_j = y_j + rho2 / alpha_j * w_{j+1}       (w = g on observed entries)
#include <type_traits>
#include "kernels.h"
#include "pinv.h"
#include "tube_dft_gen.h"
#include "tube_lds.h"

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
  int npinv;     // SLICE_ITER: blocks n1 .. n1 + npinv - 1 form G_Y^+ of frequency blockIdx.x - n1
  const uint32_t* ctr;   // counter of the BF16 rounding bits (mixed precision)
  PinvyArgs pa;
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

// LDS row stride of one tube: odd (bank-conflict-free across tubes) and, for the LDS
// transforms, at least N floats of workspace.
template <int N>
__host__ __device__ constexpr int slice_ld() { return (N % 2 == 0) ? N + 3 : N + 2; }

template <int N, int MODE>
__global__ void __launch_bounds__(SLICE_THREADS) k_slice(SliceArgs a) {
  constexpr int NB = N / 2 + 1;
  constexpr int LD = slice_ld<N>();
  constexpr bool LDSFFT = TubeLds<N>::enabled;
  constexpr int M = N / 2;
  extern __shared__ float smem[];
  const int n2 = a.n2, nwr = (n2 + 31) >> 5;
  float* zs = smem;                                   // [n2][LD]
  float* tab = zs + (size_t)n2 * LD;                  // [4][n2]
  uint32_t* obits = (uint32_t*)(tab + 4 * n2);        // [N][nwr]: bit j of row k = (i, j, k) observed
  int* cstate = (int*)(obits + N * nwr);              // [N][nwr]: run position and "seen" at each 32-column chunk
  size_t off = (size_t)n2 * LD + 4 * (size_t)n2 + 2 * (size_t)N * nwr;
  off += off & 1;
  float2* twm = (float2*)(smem + off);                // [M]   (LDS transforms only)
  float2* twn = twm + (LDSFFT ? M : 0);               // [M+1]
  double* red = (double*)(twn + (LDSFFT ? M + 1 : 0));
  const size_t i = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  const bool thomas = MODE != SLICE_INIT && !a.w_from_g;
  const float* gslice = a.gp + i * n2 * N;

  // ---- 0. tables
  for (int e = tid; e < 4 * n2; e += nt) tab[e] = a.wtab[e];
  if constexpr (LDSFFT) tube_twiddles<N>(twm, twn);
  __syncthreads();

  // ---- 1. inverse transform of Z~(i, j, :); observed entries take G, the others Z; the
  //         fit term of observed entries (of all entries when W = P_Omega(G)) is taken here
  //         and the observed flags of each row (i, :, k) become a bitmask over j (wave
  //         ballots: the tube loop keeps each wave on 64 consecutive tubes).
  double fit = 0.0, ridge = 0.0, sm = 0.0;
  const bool need_z = !(MODE == SLICE_RESULT && a.w_from_g && a.z_out == nullptr);
  for (int j = tid; j < n2; j += nt) {
    float* row = zs + j * LD;
    float z[N];
    if (need_z) {
      if constexpr (LDSFFT) {
        tube_inv_lds<N>(a.zt + i * a.nb * n2 + j, n2, row, twm, twn);
        constexpr float inv_m = 1.0f / M;
#pragma unroll
        for (int q = 0; q < N; ++q) z[q] = row[TubeLds<N>::xpos(q)] * inv_m;
      } else {
        load_inverse_tube<N>(a.zt, i, j, a.nb, n2, z);
      }
    } else {
#pragma unroll
      for (int q = 0; q < N; ++q) z[q] = 0.0f;
    }
    if (a.z_out) {
      float* dst = a.z_out + (i * n2 + j) * N;
#pragma unroll
      for (int q = 0; q < N; ++q) dst[q] = z[q];
    }
    const float* g = gslice + (size_t)j * N;   // packed G by tubes on this path
    const int jw0 = (j - lane) >> 5;   // first flag word of this wave's tubes
    float facc = 0.0f;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const float gv = g[q];
      const bool obs = !is_unobserved(gv);
      float wv, d;
      if (!thomas) {
        wv = obs ? gv : 0.0f;
        d = z[q] - wv;
      } else {
        wv = obs ? gv : z[q];
        d = obs ? z[q] - gv : 0.0f;
      }
      facc = fmaf(d, d, facc);
      row[q] = wv;
      // the wave's 64 consecutive tubes give two words of row q's flags
      const uint64_t bal = __ballot(obs);
      if (lane < 2 && jw0 + lane < nwr) obits[q * nwr + jw0 + lane] = (uint32_t)(bal >> (32 * lane));
    }
    fit += (double)facc;
  }
  __syncthreads();

  // ---- 2. W-step along mode 2 for the rows (i, :, k), 32 columns at a time: the values
  //         and pivots of a chunk are read from LDS together, then the recurrence runs in
  //         registers.  The run position at each chunk start is kept for the backward pass.
  if (thomas) {
    const float rho2 = a.rho2;
    for (int k = tid; k < N; k += nt) {
      const uint32_t* ob = obits + k * nwr;
      int* cs = cstate + k * nwr;
      float y = 0.0f;
      int pos = 0, seen = 0;
      for (int c = 0; c < nwr; ++c) {
        const int j0 = c * 32, cnt = min(32, n2 - j0);
        const uint32_t word = ob[c];
        cs[c] = pos | (seen << 20);
        float v[32], inv[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = zs[min(j0 + u, n2 - 1) * LD + k];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int o = (word >> u) & 1u;
          const int sel = (j0 + u == n2 - 1 ? 2 : 0) + seen;
          inv[u] = tab[o ? 0 : sel * n2 + min(pos, n2 - 1)];
          seen |= o;
          pos = o ? 0 : pos + 1;
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int o = (word >> u) & 1u;
          y = o ? v[u] : fmaf(rho2, y, v[u]) * inv[u];
          if (u < cnt) zs[(j0 + u) * LD + k] = y;
        }
      }
      float w = 0.0f;
      for (int c = nwr - 1; c >= 0; --c) {
        const int j0 = c * 32, cnt = min(32, n2 - j0);
        const uint32_t word = ob[c];
        const int st = cs[c];
        int p = st & 0xfffff, sn = st >> 20;
        float v[32], cf[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = zs[min(j0 + u, n2 - 1) * LD + k];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int o = (word >> u) & 1u;
          // interior pivot; observed entries and the last column take no right neighbour
          const float inv = tab[o ? 0 : sn * n2 + min(p, n2 - 1)];
          cf[u] = (o || j0 + u >= n2 - 1) ? 0.0f : rho2 * inv;
          sn |= o;
          p = o ? 0 : p + 1;
        }
#pragma unroll
        for (int u = 31; u >= 0; --u) {
          if (u < cnt) {
            w = fmaf(cf[u], w, v[u]);
            zs[(j0 + u) * LD + k] = w;
          }
        }
      }
    }
  }
  __syncthreads();

  if (MODE == SLICE_KKT) fit = ridge = sm = 0.0;   // phase 3 takes maxima instead of sums
  // ---- 3. remaining objective terms, then the forward transform of W(i, j, :).
  // For an unobserved entry the W-step equation gives
  //   z_j - w_j = (mu + rho2 deg_j) w_j - rho2 (w_{j-1} + w_{j+1}),
  // so the fit term there is formed from W alone.
  for (int j = tid; j < n2; j += nt) {
    const float* wrow = zs + j * LD;
    const bool has_l = j > 0, has_r = j + 1 < n2;
    const double cj = a.mu + a.rho2d * ((has_l ? 1.0 : 0.0) + (has_r ? 1.0 : 0.0));
    const int jw = j >> 5;
    const uint32_t jb = 1u << (j & 31);
    if constexpr (MODE == SLICE_KKT) {
      // residuals of eq. (subquKKT): unobserved (W K_{mu rho2} - Z)_ij, observed W - G
      const float* g = gslice + (size_t)j * N;
      float z[N];
      load_inverse_tube<N>(a.zt, i, j, a.nb, n2, z);
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const bool obs = obits[q * nwr + jw] & jb;
        const double wq = wrow[q];
        if (!obs && thomas) {
          const double l = has_l ? (double)wrow[q - LD] : 0.0;
          const double r = has_r ? (double)wrow[q + LD] : 0.0;
          fit = fmax(fit, fabs((1.0 + cj) * wq - a.rho2d * (l + r) - (double)z[q]));
        } else if (obs) {
          ridge = fmax(ridge, fabs(wq - (double)g[q]));
        }
        sm = fmax(sm, fabs((double)z[q]));
      }
    } else {
      const float cjf = (float)cj, r2f = a.rho2;
      float fr = 0.0f, fs = 0.0f, ff = 0.0f;
#pragma unroll 8
      for (int q = 0; q < N; ++q) {
        const float wq = wrow[q];
        const float r = has_r ? wrow[q + LD] : 0.0f;
        const float l = has_l ? wrow[q - LD] : 0.0f;
        const bool un = thomas && !(obits[q * nwr + jw] & jb);
        const float d = un ? fmaf(cjf, wq, -r2f * (l + r)) : 0.0f;
        const float dr = has_r ? r - wq : 0.0f;
        fr = fmaf(wq, wq, fr);
        fs = fmaf(dr, dr, fs);
        ff = fmaf(d, d, ff);
      }
      ridge += (double)fr;
      sm += (double)fs;
      fit += (double)ff;
      if constexpr (MODE == SLICE_RESULT) {
        if (a.w_out) {
          float* dst = a.w_out + (i * n2 + j) * N;
          for (int q = 0; q < N; ++q) dst[q] = wrow[q];
        }
      }
    }
  }
  if constexpr (MODE == SLICE_INIT || MODE == SLICE_ITER) {
    if constexpr (LDSFFT) __syncthreads();   // the transforms below overwrite the rows
    for (int j = tid; j < n2; j += nt) {
      float* row = zs + j * LD;
      const size_t base = i * a.nb * n2 + j;
      if constexpr (LDSFFT) {
        if (a.mixed) {
          uint32_t* dst = (uint32_t*)a.wt + base;
          const uint32_t key = fmix32(a.ctr[0] * 0x9e3779b9u + 0x7f4a7c15u);
          tube_fwd_lds<N>(row, twm, twn, [&](int b, float re, float im) {
            dst[(size_t)b * n2] = pack_bf16x2_sr(re, im, fmix32((uint32_t)(base + (size_t)b * n2) ^ key));
          });
        } else {
          float2* dst = (float2*)a.wt + base;
          tube_fwd_lds<N>(row, twm, twn, [&](int b, float re, float im) { dst[(size_t)b * n2] = make_float2(re, im); });
        }
      } else {
        float w[N], re[NB], im[NB];
#pragma unroll
        for (int q = 0; q < N; ++q) w[q] = row[q];
        tube_fwd<N>(w, re, im);
        if (a.mixed) {
          uint32_t* dst = (uint32_t*)a.wt + base;
          const uint32_t key = fmix32(a.ctr[0] * 0x9e3779b9u + 0x7f4a7c15u);
#pragma unroll
          for (int b = 0; b < NB; ++b)
            dst[(size_t)b * n2] = pack_bf16x2_sr(re[b], im[b], fmix32((uint32_t)(base + (size_t)b * n2) ^ key));
        } else {
          float2* dst = (float2*)a.wt + base;
#pragma unroll
          for (int b = 0; b < NB; ++b) dst[(size_t)b * n2] = make_float2(re[b], im[b]);
        }
      }
    }
  }
  if constexpr (MODE == SLICE_KKT) {
    fit = block_max_d(fit, red);
    ridge = block_max_d(ridge, red);
    sm = block_max_d(sm, red);
    if (tid == 0) {
      a.kkt[3 * i + 0] = fit;
      a.kkt[3 * i + 1] = ridge;
      a.kkt[3 * i + 2] = sm;
    }
  } else if constexpr (MODE != SLICE_RESULT) {
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



// Value of lane - d (up) or lane + d (down) within the S-lane group of a row.  For S <= 16
// the group lies in one 16-lane DPP row and the move is a row shift of the VALU (lanes whose
// source falls outside the row read 0; callers only use lanes whose source is in the group);
// wider groups go through the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int S>
__device__ __forceinline__ float seg_up(float v, int d) {
  if constexpr (S <= 16) {
    switch (d) {
      case 1: return dpp_mov<0x111>(v);   // row_shr:1
      case 2: return dpp_mov<0x112>(v);
      case 4: return dpp_mov<0x114>(v);
      default: return dpp_mov<0x118>(v);
    }
  } else {
    return __shfl_up(v, d, S);
  }
}
template <int S>
__device__ __forceinline__ float seg_down(float v, int d) {
  if constexpr (S <= 16) {
    switch (d) {
      case 1: return dpp_mov<0x101>(v);   // row_shl:1
      case 2: return dpp_mov<0x102>(v);
      case 4: return dpp_mov<0x104>(v);
      default: return dpp_mov<0x108>(v);
    }
  } else {
    return __shfl_down(v, d, S);
  }
}

// W-step of every row (i, :, k) with S threads per row: thread (k, s) takes columns
// [s L, (s+1) L).  Both Thomas passes are first-order affine recurrences,
//   forward  y_j = a_j y_{j-1} + b_j  (a = rho2 / alpha_j, b = v_j / alpha_j; a = 0, b = g_j observed)
//   backward w_j = c_j w_{j+1} + y_j  (c = rho2 / alpha_j; c = 0 observed or at the last column),
// so each thread composes its segment's map, the S maps of a row are combined by a
// scan across the S lanes, and each thread then runs its segment once more from the
// right boundary value.  S divides 64 and is a power of two; L <= LMAX <= 32.
// OBJ: also the row's terms of f0 from the solved values still in registers (the
// neighbours across segment ends from the adjacent lanes): ridge sum w_j^2, K term
// sum (w_{j+1} - w_j)^2 and, on unobserved entries, the fit residual z_j - w_j, which the
// row's equation gives as (mu + rho2 deg_j) w_j - rho2 (w_{j-1} + w_{j+1}); added to fr, fs,
// ff.
template <int LMAX, int S, bool OBJ>
__device__ __forceinline__ void wstep_segmented(float* zs, int LD, const float* tab, const uint32_t* obits, int nwr,
                                                int n2, int N, float rho2, float mu, float& fr, float& fs,
                                                float& ff) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int L = (n2 + S - 1) / S;
  for (int kk = tid; kk < N * S; kk += nt) {
    const int k = kk / S, s = kk - k * S;
    const int ja = min(n2, s * L), jb = min(n2, ja + L);
    const uint32_t* ob = obits + k * nwr;
    // the segment's observed flags (it spans at most two flag words): bit u = entry ja + u
    const int w0 = ja >> 5;
    const uint64_t wpair = (uint64_t)ob[min(w0, nwr - 1)] | ((uint64_t)ob[min(w0 + 1, nwr - 1)] << 32);
    const uint32_t obm = (uint32_t)(wpair >> (ja & 31));
    // run state at ja: position in the current run of unobserved entries, and whether
    // an observed entry precedes it
    int seen, pos;
    {
      int w = w0;
      uint32_t m = ja > 0 ? ((uint32_t)wpair & ((1u << (ja & 31)) - 1u)) : 0u;
      while (m == 0u && w > 0) m = ob[--w];
      const int last = (m == 0u) ? -1 : (w * 32 + 31 - __clz(m));
      seen = last >= 0;
      pos = ja - last - 1;
    }
    float av[LMAX], bv[LMAX], cv[LMAX];
    float A = 1.0f, B = 0.0f;
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
      const int j = ja + u;
      if (j < jb) {
        const bool o = (obm >> u) & 1u;
        const float v = zs[j * LD + k];
        const float invf = tab[o ? 0 : ((j == n2 - 1 ? 2 : 0) + seen) * n2 + pos];
        const float invb = tab[o ? 0 : seen * n2 + pos];
        av[u] = o ? 0.0f : rho2 * invf;
        bv[u] = o ? v : v * invf;
        cv[u] = (o || j == n2 - 1) ? 0.0f : rho2 * invb;
        seen |= o;
        pos = o ? 0 : pos + 1;
        B = fmaf(av[u], B, bv[u]);
        A *= av[u];
      }
    }
    // forward: combine the segment maps of the row (lanes k*S .. k*S+S-1)
#pragma unroll
    for (int d = 1; d < S; d <<= 1) {
      const float a2 = seg_up<S>(A, d), b2 = seg_up<S>(B, d);
      if (s >= d) { B = fmaf(A, b2, B); A *= a2; }
    }
    float y = seg_up<S>(B, 1);
    if (s == 0) y = 0.0f;
    float C = 1.0f, D = 0.0f;
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
      if (ja + u < jb) {
        y = fmaf(av[u], y, bv[u]);
        bv[u] = y;   // y_j
      }
    }
#pragma unroll
    for (int u = LMAX - 1; u >= 0; --u) {
      if (ja + u < jb) {
        D = fmaf(cv[u], D, bv[u]);
        C *= cv[u];
      }
    }
#pragma unroll
    for (int d = 1; d < S; d <<= 1) {
      const float c2 = seg_down<S>(C, d), d2 = seg_down<S>(D, d);
      if (s + d < S) { D = fmaf(C, d2, D); C *= c2; }
    }
    float w = seg_down<S>(D, 1);
    if (s == S - 1) w = 0.0f;
#pragma unroll
    for (int u = LMAX - 1; u >= 0; --u) {
      const int j = ja + u;
      if (j < jb) {
        w = fmaf(cv[u], w, bv[u]);
        bv[u] = w;   // w_j
        zs[j * LD + k] = w;
      }
    }
    if constexpr (OBJ) {
      // the segments before the last non-empty one are full, so lane s - 1's last value is
      // w_{ja - 1} and lane s + 1's first value is w_{jb} wherever they exist
      float last = 0.0f;
#pragma unroll
      for (int u = 0; u < LMAX; ++u)
        if (ja + u < jb) last = bv[u];
      const float left = seg_up<S>(last, 1), right = seg_down<S>(bv[0], 1);
      float wl = left;
#pragma unroll
      for (int u = 0; u < LMAX; ++u) {
        const int j = ja + u;
        if (j < jb) {
          const float wq = bv[u];
          const float wr = (u + 1 < LMAX && j + 1 < jb) ? bv[u + 1 < LMAX ? u + 1 : u] : right;
          const bool has_l = j > 0, has_r = j + 1 < n2;
          const float l = has_l ? wl : 0.0f, r = has_r ? wr : 0.0f;
          const float cj = fmaf(rho2, (has_l ? 1.0f : 0.0f) + (has_r ? 1.0f : 0.0f), mu);
          const float d = ((obm >> u) & 1u) ? 0.0f : fmaf(cj, wq, -rho2 * (l + r));
          const float dr = has_r ? r - wq : 0.0f;
          fr = fmaf(wq, wq, fr);
          fs = fmaf(dr, dr, fs);
          ff = fmaf(d, d, ff);
          wl = wq;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- cooperative slice kernel
// The same three steps with T threads per tube (thread (t, j) = t * n2p + j, n2p = n2
// rounded up to 64 so that every wavefront holds 64 consecutive tubes of one t; rounding to
// 32 instead, which leaves no lane idle at n2 = 96, ran 2 % slower: the W-step then takes
// five passes over the block instead of four).  The tube
// transforms run through the tube's LDS row stage by stage.  T = M1 / 2 where that still
// gives each thread at most two groups of every stage (else T = M1): the smaller blocks and
// W-step segments of at most COOP_WS_L entries keep the registers low enough for three row
// blocks per compute unit, so that a few hundred rows are all in flight at once and the
// latency of one block's barriers and LDS round trips is hidden behind the others.  In an
// iteration, nb more blocks after the rows form G_Y^+ and I - eta P_Y for the next X-step
// (pinvy_block); the register cap keeps their allocation from raising the row blocks'.
// Used when the block (T * n2p threads) fits 1024 threads.
#define COOP_WS_L 8
template <int N>
__host__ __device__ constexpr int coop_tube_threads() {
  constexpr int m1 = TubePlan<N>::M1, m2 = TubePlan<N>::M2;
  return (m1 % 2 == 0 && m1 / 2 < m2 && m2 <= m1) ? m1 / 2 : m1;
}
template <int N, int MODE>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(7))) k_slice_coop(SliceArgs a) {
  using TL = TubeLds<N>;
  constexpr int T = coop_tube_threads<N>(), M1 = TL::M1, M2 = TL::M2, M = N / 2;
  using FC = typename std::conditional<(T < M2), Fft4C2<M1, M2, T>, Fft4C<M1, M2>>::type;
  constexpr int LD = slice_ld<N>();
  extern __shared__ __align__(16) float smem[];
  if constexpr (MODE == SLICE_ITER) {
    if ((int)blockIdx.x >= a.n1) {
      pinvy_block((int)blockIdx.x - a.n1, a.pa, (unsigned char*)smem);
      return;
    }
  }
  const int n2 = a.n2, nwr = (n2 + 31) >> 5, n2p = (n2 + 63) & ~63;
  float* zs = smem;                                   // [n2][LD]
  float* tab = zs + (size_t)n2 * LD;                  // [4][n2]
  uint32_t* obits = (uint32_t*)(tab + 4 * n2);        // [N][nwr]
  int* cstate = (int*)(obits + N * nwr);              // [N][nwr]
  size_t off = (size_t)n2 * LD + 4 * (size_t)n2 + 2 * (size_t)N * nwr;
  off += off & 1;
  float2* twm = (float2*)(smem + off);                // [M]
  float2* twn = twm + M;                              // [M+1]
  double* red = (double*)(twn + M + 1);
  const size_t i = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  const int t = tid / n2p, j = tid - t * n2p;
  const bool act = j < n2;
  const bool thomas = MODE != SLICE_INIT && !a.w_from_g;
  float* row = zs + (size_t)(act ? j : 0) * LD;
  const float* gtube = a.gp + i * n2 * N + (act ? j : 0);   // packed G by rows on this path: entry q at gtube[q n2]

  for (int e = tid; e < 4 * n2; e += nt) tab[e] = a.wtab[e];
  tube_twiddles<N>(twm, twn);
  __syncthreads();

  // ---- 1. inverse transform of Z~(i, j, :) (natural order in the row)
  const bool need_z = !(MODE == SLICE_RESULT && a.w_from_g && a.z_out == nullptr);
  if (need_z) {
    if (act) tube_inv_pre<N>(a.zt + i * a.nb * n2 + j, n2, row, twn, t, T);
    __syncthreads();
    if (act) fft4_step_a<M1, M2, -1>(row, twm, t, T);
    __syncthreads();
    FC sc;
    if (act) sc.read(row, t);
    __syncthreads();
    if (act) sc.template write<-1>(row, t);
    __syncthreads();
  }
  // observed entries take G, the others Z; fit term of observed entries (all entries when
  // W = P_Omega(G)); observed flags of each row (i, :, k) by wave ballots
  double fit = 0.0, ridge = 0.0, sm = 0.0;
  {
    constexpr float inv_m = 1.0f / M;
    constexpr int B = 7;   // G entries loaded ahead of their use: one load latency per seven
    float facc = 0.0f;
    for (int q0 = t; q0 < N; q0 += B * T) {
      float gb[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int q = q0 + u * T;
        gb[u] = ld_or(gtube, (size_t)q * n2, act && q < N, 0.0f);
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int q = q0 + u * T;
        if (q >= N) break;   // the same in the whole wavefront (one t per wavefront)
        const float zq = (act && need_z) ? row[q] * inv_m : 0.0f, gv = gb[u];
        const bool obs = act && !is_unobserved(gv);
        float wv, d;
        if (!thomas) {
          wv = obs ? gv : 0.0f;
          d = zq - wv;
        } else {
          wv = obs ? gv : zq;
          d = obs ? zq - gv : 0.0f;
        }
        if (act) {
          facc = fmaf(d, d, facc);
          row[q] = wv;
          if (a.z_out) a.z_out[(i * n2 + j) * N + q] = zq;
        }
        // each half wavefront: the 32 tubes of flag word j / 32
        const uint64_t bal = __ballot(obs);
        if ((lane & 31) == 0 && act) obits[q * nwr + (j >> 5)] = (uint32_t)(bal >> lane);
      }
    }
    fit += (double)facc;
  }
  __syncthreads();

  // ---- 2. W-step along mode 2 for the rows (i, :, k), S threads per row
  // in an iteration the f0 terms of the solved rows come from the W-step's registers
  constexpr bool OBJ = MODE == SLICE_ITER;
  float wfr = 0.0f, wfs = 0.0f, wff = 0.0f;
  if (thomas) {
    int S = 1;
    while (S < 64 && 2 * S * N <= nt) S <<= 1;
    while ((n2 + S - 1) / S > COOP_WS_L) S <<= 1;   // segment length within the register budget
    const float muf = (float)a.mu;
    switch (S) {   // the segment count is a compile-time constant of the shuffles
#define TCTF_WSTEP(SS) \
  case SS: wstep_segmented<COOP_WS_L, SS, OBJ>(zs, LD, tab, obits, nwr, n2, N, a.rho2, muf, wfr, wfs, wff); break;
      TCTF_WSTEP(1)
      TCTF_WSTEP(2)
      TCTF_WSTEP(4)
      TCTF_WSTEP(8)
      TCTF_WSTEP(16)
      TCTF_WSTEP(32)
#undef TCTF_WSTEP
      default: wstep_segmented<COOP_WS_L, 64, OBJ>(zs, LD, tab, obits, nwr, n2, N, a.rho2, muf, wfr, wfs, wff); break;
    }
  }
  __syncthreads();

  if (MODE == SLICE_KKT) fit = ridge = sm = 0.0;   // phase 3 takes maxima instead of sums
  ridge += (double)wfr;
  sm += (double)wfs;
  fit += (double)wff;
  // ---- 3. remaining objective terms (see k_slice; in an iteration the W-step gave them),
  // then the forward transform
  if (act && !(OBJ && thomas)) {
    const bool has_l = j > 0, has_r = j + 1 < n2;
    const int jw = j >> 5;
    const uint32_t jb = 1u << (j & 31);
    const double cj = a.mu + a.rho2d * ((has_l ? 1.0 : 0.0) + (has_r ? 1.0 : 0.0));
    if constexpr (MODE == SLICE_KKT) {
      if (t == 0) {
        float z[N];
        load_inverse_tube<N>(a.zt, i, j, a.nb, n2, z);
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const bool obs = obits[q * nwr + jw] & jb;
          const double wq = row[q];
          if (!obs && thomas) {
            const double l = has_l ? (double)row[q - LD] : 0.0;
            const double r = has_r ? (double)row[q + LD] : 0.0;
            fit = fmax(fit, fabs((1.0 + cj) * wq - a.rho2d * (l + r) - (double)z[q]));
          } else if (obs) {
            ridge = fmax(ridge, fabs(wq - (double)gtube[(size_t)q * n2]));
          }
          sm = fmax(sm, fabs((double)z[q]));
        }
      }
    } else {
      const float cjf = (float)cj, r2f = a.rho2;
      float fr = 0.0f, fs = 0.0f, ff = 0.0f;
      for (int q = t; q < N; q += T) {
        const float wq = row[q];
        const float r = has_r ? row[q + LD] : 0.0f;
        const float l = has_l ? row[q - LD] : 0.0f;
        const bool un = thomas && !(obits[q * nwr + jw] & jb);
        const float d = un ? fmaf(cjf, wq, -r2f * (l + r)) : 0.0f;
        const float dr = has_r ? r - wq : 0.0f;
        fr = fmaf(wq, wq, fr);
        fs = fmaf(dr, dr, fs);
        ff = fmaf(d, d, ff);
        if constexpr (MODE == SLICE_RESULT) {
          if (a.w_out) a.w_out[(i * n2 + j) * N + q] = wq;
        }
      }
      ridge += (double)fr;
      sm += (double)fs;
      fit += (double)ff;
    }
  }
  if constexpr (MODE == SLICE_INIT || MODE == SLICE_ITER) {
    __syncthreads();   // the transform below overwrites the rows
    if (act) fft4_step_a<M1, M2, +1>(row, twm, t, T);
    __syncthreads();
    FC sc;
    if (act) sc.read(row, t);
    __syncthreads();
    if (act) sc.template write<+1>(row, t);
    __syncthreads();
    if (act) {
      const size_t base = i * a.nb * n2 + j;
      if (a.mixed) {
        uint32_t* dst = (uint32_t*)a.wt + base;
        const uint32_t key = fmix32(a.ctr[0] * 0x9e3779b9u + 0x7f4a7c15u);
        tube_fwd_post_nat<N>(row, twn, t, T, [&](int b, float re, float im) {
          dst[(size_t)b * n2] = pack_bf16x2_sr(re, im, fmix32((uint32_t)(base + (size_t)b * n2) ^ key));
        });
      } else {
        float2* dst = (float2*)a.wt + base;
        tube_fwd_post_nat<N>(row, twn, t, T, [&](int b, float re, float im) { dst[(size_t)b * n2] = make_float2(re, im); });
      }
    }
  }
  if constexpr (MODE == SLICE_KKT) {
    fit = block_max_d(fit, red);
    ridge = block_max_d(ridge, red);
    sm = block_max_d(sm, red);
    if (tid == 0) {
      a.kkt[3 * i + 0] = fit;
      a.kkt[3 * i + 1] = ridge;
      a.kkt[3 * i + 2] = sm;
    }
  } else if constexpr (MODE != SLICE_RESULT) {
    block_sum3_d(fit, ridge, sm, red);
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
  const size_t nwr = ((size_t)n2 + 31) / 32;
  const size_t ld = (n3 % 2 == 0) ? n3 + 3 : n3 + 2;
  size_t floats = (size_t)n2 * ld + 4 * (size_t)n2 + 2 * (size_t)n3 * nwr + 1;
  floats += 2 * (size_t)(n3 + 1);   // twiddles of the LDS transforms
  return floats * sizeof(float) + 48 * sizeof(double) + 16;
}

static int coop_threads(int n2, int n3) {
  int m1 = 0;
  switch (n3) {
#define TCTF_CASE(n) case n: m1 = TubePlan<n>::M1 > 0 ? coop_tube_threads<n>() : 0; break;
    TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
    default: break;
  }
  const int n2p = (n2 + 63) / 64 * 64;
  return (m1 > 0 && m1 * n2p <= 1024) ? m1 * n2p : 0;
}

void slice_set_attr(int n3, size_t lds) {
  if (lds <= 65536) return;
  switch (n3) {
#define TCTF_CASE(n)                                                                                          \
  case n:                                                                                                     \
    (void)hipFuncSetAttribute((const void*)k_slice<n, SLICE_INIT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    (void)hipFuncSetAttribute((const void*)k_slice<n, SLICE_ITER>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    (void)hipFuncSetAttribute((const void*)k_slice<n, SLICE_RESULT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    (void)hipFuncSetAttribute((const void*)k_slice<n, SLICE_KKT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
    if constexpr (TubePlan<n>::M1 > 0) {                                                                      \
      (void)hipFuncSetAttribute((const void*)k_slice_coop<n, SLICE_INIT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      (void)hipFuncSetAttribute((const void*)k_slice_coop<n, SLICE_ITER>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      (void)hipFuncSetAttribute((const void*)k_slice_coop<n, SLICE_RESULT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      (void)hipFuncSetAttribute((const void*)k_slice_coop<n, SLICE_KKT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    }                                                                                                         \
    break;
    TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
    default: break;
  }
}

bool slice_fused(int n2, int n3) { return slice_supported(n3) && slice_lds_bytes(n2, n3) <= TCTF_SLICE_LDS_MAX; }

int slice_default_path(int n2, int n3) {
  if (!slice_fused(n2, n3)) return SPATH_SPLIT;
  return coop_threads(n2, n3) > 0 ? SPATH_COOP : SPATH_THREAD;
}

bool slice_path_valid(int path, int n2, int n3) {
  switch (path) {
    case SPATH_COOP: return slice_fused(n2, n3) && coop_threads(n2, n3) > 0;
    case SPATH_THREAD: return slice_fused(n2, n3);
    case SPATH_SPLIT: return true;
    default: return false;
  }
}

bool slice_hosts_pinvy(const Plan& p) { return p.spath == SPATH_COOP; }

size_t slice_launch_lds_bytes(const Plan& p) {
  if (p.spath == SPATH_SPLIT) return 0;
  const size_t a = slice_lds_bytes(p.n2, p.n3), b = p.spath == SPATH_COOP ? pinvy_lds_bytes(p.r) : 0;
  return a > b ? a : b;
}

void launch_slice(const Plan& p, int mode, float* w_out, float* z_out, int w_from_g) {
  if (p.spath == SPATH_SPLIT) {
    launch_slice_generic(p, mode, w_out, z_out, w_from_g);
    return;
  }
  SliceArgs a;
  a.npinv = (mode == SLICE_ITER && slice_hosts_pinvy(p)) ? p.nb : 0;
  a.pa = pinvy_args(p);
  a.ctr = p.ctr;
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
  const size_t lds = slice_launch_lds_bytes(p);
  const int coop = p.spath == SPATH_COOP ? coop_threads(p.n2, p.n3) : 0;
  if (coop > 0) {
    switch (p.n3) {
#define TCTF_CASE(n)                                                                                   \
  case n:                                                                                              \
    if constexpr (TubePlan<n>::M1 > 0) {                                                               \
      if (mode == SLICE_INIT) k_slice_coop<n, SLICE_INIT><<<p.n1, coop, lds, p.stream>>>(a);           \
      else if (mode == SLICE_ITER) k_slice_coop<n, SLICE_ITER><<<p.n1 + a.npinv, coop, lds, p.stream>>>(a); \
      else if (mode == SLICE_RESULT) k_slice_coop<n, SLICE_RESULT><<<p.n1, coop, lds, p.stream>>>(a);  \
      else k_slice_coop<n, SLICE_KKT><<<p.n1, coop, lds, p.stream>>>(a);                               \
    }                                                                                                  \
    break;
      TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
      default: break;
    }
    return;
  }
  const int need = p.n2 > p.n3 ? p.n2 : p.n3;
  int threads = ((need + 63) / 64) * 64;
  if (threads > SLICE_THREADS) threads = SLICE_THREADS;
  switch (p.n3) {
#define TCTF_CASE(n)                                                                   \
  case n:                                                                              \
    if (mode == SLICE_INIT) k_slice<n, SLICE_INIT><<<p.n1, threads, lds, p.stream>>>(a);        \
    else if (mode == SLICE_ITER) k_slice<n, SLICE_ITER><<<p.n1, threads, lds, p.stream>>>(a);   \
    else if (mode == SLICE_RESULT) k_slice<n, SLICE_RESULT><<<p.n1, threads, lds, p.stream>>>(a); \
    else k_slice<n, SLICE_KKT><<<p.n1, threads, lds, p.stream>>>(a);                             \
    break;
    TUBE_DFT_SIZES(TCTF_CASE)
#undef TCTF_CASE
    default: break;
  }
}

}  // namespace tctf

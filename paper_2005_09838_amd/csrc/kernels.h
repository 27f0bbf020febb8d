// Kernel launchers of the TCTF2R gfx950 library (host-callable, stream-ordered).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.h"

namespace tctf {

#define HINV_KMAX 12   // widest stencil of H_rho1^{-1} applied inside the X-update

// Device buffers and sizes of one completion (carved from the caller's workspace).
struct Plan {
  int n1, n2, n3, r, nb;       // nb = n3/2 + 1 stored frequencies
  int bcg;                     // complex columns per X~^* W~ block (16 or 32)
  int ny, ycw;                 // column blocks of the Y-step per frequency, columns per block
  int spath;                   // slice path: SPATH_COOP, SPATH_THREAD or SPATH_SPLIT
  int ncu;                     // compute units of the device
  double mu, rho1, rho2, eta;
  // H_rho1^{-1} as a stencil of half-width hk inside the X-update (k_agemm), hk = -1: the
  // X-update forms the right-hand side and k_hsolve solves (see hinv_stencil)
  int hk;
  double htap[2 * HINV_KMAX + 2];
  int mixed, force_eigen;
  hipStream_t stream;

  float* gp;        // observed values, unobserved entries NaN-coded (run position); g_rows = 1:
                    // [n1][n3][n2] (entry (i, j, k) at (i n3 + k) n2 + j: the cooperative slice
                    // kernel reads 64 tubes per wave instruction), 0: [n1][n2][n3] (one thread
                    // per tube or per row reads its own run of entries)
  int g_rows;
  void* wt;         // W~ [n1][nb][n2] float2 (FP32) or packed bf16x2 (mixed)
  float2* zt;       // Z~ [n1][nb][n2]
  float2* xt;       // X~ [nb][r][n1]
  float2* yt;       // Y~ [nb][r][n2]
  float2* rhs;      // right-hand side of the H_rho1 solve [nb][r][n1]
  double2* bpart;   // X~^* W~ [nb][r][n2] (FP64)
  cd* gxpart;       // partial Grams of X~ over row groups [nb][ngroup][2][r][r] (FP64)
  cd* gxm;          // G_X = X~^* H_rho1 X~ [nb][r][r]
  cd* dmat;         // (H X~)^* (H X~) [nb][r][r]
  cd* gxp;          // G_X^+ [nb][r][r]
  cd* qx;           // I - eta P_X [nb][r][r]
  int* qx_zero;     // [nb] 1 when I - eta P_X is exactly 0
  cd* gym;          // partial Y~ Y~^* over column blocks [nb][ny][r][r]
  cd* gyp;          // (Y~ Y~^*)^+ [nb][r][r]
  cd* qy;           // I - eta P_Y [nb][r][r]
  int* qy_zero;     // [nb] 1 when I - eta P_Y is exactly 0 (eta = 1, full rank)
  double* slice_obj;// [n1][3] fit, ridge and mode-2 difference sums of the last W-step
  double* bin_obj;  // [nb] c_b tr((H X~_b)^*(H X~_b) Y~_b Y~_b^*)
  float* wtab;      // [4][n2] reciprocal pivots of the W-step row systems
  float* htab;      // [3][n1] Thomas coefficients of H_rho1
  int* flag;        // non-finite detector
  uint32_t* ctr;    // iteration counter of the BF16 rounding bits (advanced by each X-step)
  // the three-launch slice path (tube lengths outside the generated set, or slices larger
  // than the fused kernel's LDS): spatial Z, W and elimination factors, roots of unity
  float* zsp;       // [n1][n2][n3]
  float* wsp;       // [n1][n2][n3]
  float* csp;       // [n1][n2][n3]
  double2* twg;     // [n3] (cos, sin)(2 pi m / n3)
  // step 5 (rank adjustment)
  double* rsig;     // [nb][r] singular values of Z~_b, descending
  cd* rtx;          // [nb][r][r] factor rotations of X~ and Y~
  cd* rty;
  int* ranks;       // [nb] the rank vector r_b
  double* scal;     // [16] scalar results (objective, termination, stationarity)
  float2* xt_prev;  // snapshots for the termination test
  float2* yt_prev;
  void* wt_prev;
  double* stat_work;// [nb][8] stationarity partial sums (and termination partials)
  double* kkt;      // [n1][3] W-KKT residual maxima of the slices
};

size_t wt_elem_bytes(const Plan& p);

// setup
void launch_pack_g(const Plan& p, const float* G, const uint8_t* omega);
void launch_tables(const Plan& p);
void launch_tube_dft_setup(const Plan& p, const float* src, float2* dst, int P, int Q,
                           long sb, long sp, long sq);   // real [P][Q][n3] -> half spectrum
void launch_tube_idft_setup(const Plan& p, const float2* src, float* dst, int P, int Q,
                            long sb, long sp, long sq);  // half spectrum -> real [P][Q][n3]
void launch_normal(const Plan& p, float* dst, size_t n, uint64_t seed);
void launch_zero(const Plan& p, void* dst, size_t bytes);

// iteration
enum SliceMode { SLICE_INIT = 0, SLICE_ITER = 1, SLICE_RESULT = 2, SLICE_KKT = 3 };
// How steps 3, 4 and 7 run: one fused kernel per OD row with several threads per tube
// (COOP) or one thread per tube (THREAD), or three launches through spatial buffers (SPLIT).
enum SlicePath { SPATH_COOP = 1, SPATH_THREAD = 2, SPATH_SPLIT = 3 };
int slice_default_path(int n2, int n3);
bool slice_path_valid(int path, int n2, int n3);
bool slice_supported(int n3);
bool slice_fused(int n2, int n3);          // the fused LDS slice kernel applies
void launch_gen_twiddles(const Plan& p);
void launch_slice_generic(const Plan& p, int mode, float* w_out, float* z_out, int w_from_g);
bool slice_hosts_pinvy(const Plan& p);   // the iteration's slice launch also forms G_Y^+
size_t slice_launch_lds_bytes(const Plan& p);
void launch_slice(const Plan& p, int mode, float* w_out, float* z_out, int w_from_g);
void launch_zgemm(const Plan& p, int with_pinv = 0);   // with_pinv: also G_Y^+ (pinvy_block)
// advance: next rounding-bit counter; scratch_out: with the stencil, X~ goes to the rhs
// buffer instead of X~ itself (a stage timing that leaves the state as it was)
void launch_agemm(const Plan& p, int raw_a = 0, int advance = 0, int scratch_out = 0);
// Half-width k and taps c lambda^d (d = 0 .. 2k + 1) of H_rho1^{-1} as a stencil, or -1
// where the stencil would be wider than HINV_KMAX, r > 16 or n1 < 2k + 2
int hinv_stencil(double rho1, int n1, int r, double* tap);
void launch_hsolve(const Plan& p);
void launch_bgemm(const Plan& p);   // X~^* W~ over all rows
void launch_gramx(const Plan& p);   // G_X, (H X~)^*(H X~), G_X^+ and I - eta P_X
int gramx_groups(int n1);
void gramx_set_attr(int r);
size_t bgemm_lds_bytes(int r, int bcg);
bool bgemm_cols_valid(int r, int bcg);

void bgemm_set_attr();
void launch_ystep(const Plan& p, int init);
void ystep_split(int n2, int r, int nb, int* ny, int* cw);
size_t ystep_lds_bytes(int r, int cw);
void ystep_set_attr(size_t lds);
void launch_pinvy(const Plan& p, hipStream_t stream);
void pinvy_set_attr(int r);
void zgemm_set_attr(int r);
void launch_objective(const Plan& p);
void launch_termination(const Plan& p);
void launch_rank_init(const Plan& p);
void launch_rank_adjust(const Plan& p, double tol);
void rank_set_attr(int r);
size_t termination_work_doubles();   // partials of the step-6 reduction held in stat_work
void launch_stationarity(const Plan& p, int w_from_g);

// differentiation (reverse mode) of one iteration, FP64 (kernels_adjoint.hip)
// Complex matrix batch view: element (b, i, j) at b bs + i rs + j cs of float2 (f32 = 1) or
// double2 storage, conjugated on load when conj = 1.
struct CView {
  const void* p;
  long bs, rs, cs;
  int f32, conj;
};
struct AdjState {        // forward values of one iterate (inside a checkpoint blob)
  const float2* xt;      // X~ [nb][r][n1]
  const float2* yt;      // Y~ [nb][r][n2]
  const float2* wt;      // W~ [n1][nb][n2]
};
struct AdjWork {         // adjoint scratch carved from the caller's adjoint workspace
  double *w1s, *cbuf, *zbar;
  double2 *ztb, *wtb;
  double2 *x1b, *hx1, *a, *pp, *q, *pb, *qb, *ab, *dt;
  double2 *y1b, *bm, *bb, *rb;
  double2 *gy, *gyi, *gx, *gxi, *gyib, *gxib, *gyb, *gxb, *S, *T, *tmp;
  double* htab;
  double* part;
  int* flag;
};
size_t adjoint_work_bytes(const Plan& p);
void adjoint_carve(const Plan& p, void* ws, AdjWork* w);
void adjoint_set_attr(int r);
void launch_adjoint_step(const Plan& p, const AdjWork& w, const AdjState& in, const AdjState& out, double2* xt_bar,
                         double2* yt_bar, double* w_bar, double* theta);
void launch_adjoint_initial(const Plan& p, const double2* xt_bar, const double2* yt_bar, double* x0_bar,
                            double* y0_bar);
void launch_objective_gradient(const Plan& p, const AdjWork& w, double* x_grad, double* y_grad);

}  // namespace tctf

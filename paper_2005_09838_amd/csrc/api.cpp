// C ABI of the TCTF2R library: argument checks, workspace carve-up, the iteration
// schedule and result / checkpoint transfers.  Every computation runs in the HIP kernels
// launched from here; this file only validates, lays out memory and enqueues work.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tctf2r.h"
#include "kernels.h"

namespace tctf {
size_t slice_lds_bytes(int n2, int n3);
void slice_set_attr(int n3, size_t lds);
}  // namespace tctf

using tctf::Plan;

static thread_local std::string g_err;

static tctf_status fail(tctf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(TCTF_E_HIP, "%s: %s", #call, hipGetErrorString(e_));    \
  } while (0)

static const uint64_t kStateMagic = 0x54435446324bULL;   // "TCTF2K"

struct StateHeader {
  uint64_t magic;
  int32_t n1, n2, n3, r, precision, pad;
  int64_t iters;
  uint64_t reserved[4];
};

struct Layout {
  size_t gp, wt, zt, xt, yt, rhs, bpart, gxpart, gxm, dmat, gxp, qx, qx_zero, gym, gyp, qy, qy_zero, slice_obj, bin_obj, wtab, htab,
      flag, ctr, zsp, wsp, csp, twg, rsig, rtx, rty, ranks, scal, xt_prev, yt_prev, wt_prev, stat_work, kkt, total;
  size_t state_bytes;
  bool split;   // the three-launch slice path's buffers exist
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Complex columns per X~^* W~ block: 32 (half the re-reads of X~, and fewer blocks than
// compute units at 529 x 96 x 112, so that the G_X launches beside it find free ones)
// unless that leaves fewer than 128 blocks, then 16.
static int default_bcg(int n2, int nb, int r) {
  (void)r;
  return (long)((n2 + 31) / 32) * nb >= 128 ? 32 : 16;
}

// Tunable execution shape of one context: the slice path (tctf::SlicePath, the fusion
// depth of steps 3, 4 and 7), the columns per X~^* W~ block and per Y-step block.
struct Knobs {
  int spath, bcg, ycw;
  int hstencil;   // 1: the X-update applies H_rho1^{-1} as a stencil where hinv_stencil allows
};
#define TUNE_MIN_YCW 8

static Knobs default_knobs(const tctf_params& p) {
  Knobs k;
  int ny;
  const int nb = p.n3 / 2 + 1;
  k.spath = tctf::slice_default_path(p.n2, p.n3);
  k.bcg = default_bcg(p.n2, nb, p.r);
  tctf::ystep_split(p.n2, p.r, nb, &ny, &k.ycw);
  k.hstencil = p.xsolve == 0;
  return k;
}

static Layout make_layout(const tctf_params& p) {
  Layout L;
  const size_t n1 = p.n1, n2 = p.n2, n3 = p.n3, r = p.r, nb = n3 / 2 + 1;
  // buffers sized for the default shape, or for every shape the autotuner may pick
  const Knobs dk = default_knobs(p);
  const int ycw = p.autotune ? (TUNE_MIN_YCW < p.n2 ? TUNE_MIN_YCW : p.n2) : dk.ycw;
  const size_t ny = (n2 + ycw - 1) / ycw;
  const size_t welem = p.precision == TCTF_MIXED_BF16 ? 4 : 8;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  L.gp = take(n1 * n2 * n3 * 4);
  L.wt = take(n1 * nb * n2 * welem + 256 * 8);   // slack read (and discarded) by the A = W~ Y~^* loads
  L.zt = take(n1 * nb * n2 * 8);
  L.xt = take(nb * r * n1 * 8);
  L.yt = take(nb * r * n2 * 8);
  L.rhs = take(nb * r * n1 * 8);
  L.bpart = take(nb * r * n2 * 16);
  L.gxpart = take(nb * (size_t)tctf::gramx_groups(p.n1) * 2 * r * r * 16);
  L.gxm = take(nb * r * r * 16);
  L.dmat = take(nb * r * r * 16);
  L.gxp = take(nb * r * r * 16);
  L.qx = take(nb * r * r * 16);
  L.qx_zero = take(nb * 4);
  L.gym = take(nb * ny * r * r * 16);
  L.gyp = take(nb * r * r * 16);
  L.qy = take(nb * r * r * 16);
  L.qy_zero = take(nb * 4);
  L.slice_obj = take(n1 * 3 * 8);
  L.bin_obj = take(nb * 8);
  L.wtab = take(4 * n2 * 4);
  L.htab = take(3 * n1 * 4);
  L.flag = take(64);
  L.ctr = take(64);
  const bool gen = p.autotune || dk.spath == tctf::SPATH_SPLIT;   // the three-launch slice path
  L.zsp = take(gen ? n1 * n2 * n3 * 4 : 0);
  L.wsp = take(gen ? n1 * n2 * n3 * 4 : 0);
  L.csp = take(gen ? n1 * n2 * n3 * 4 : 0);
  L.twg = take(gen ? n3 * 16 : 0);
  L.split = gen;
  L.rsig = take(nb * r * 8);
  L.rtx = take(nb * r * r * 16);
  L.rty = take(nb * r * r * 16);
  L.ranks = take(nb * 4);
  L.scal = take(16 * 8);
  L.xt_prev = take(nb * r * n1 * 8);
  L.yt_prev = take(nb * r * n2 * 8);
  L.wt_prev = take(n1 * nb * n2 * welem);
  const size_t sw = nb * 8 > tctf::termination_work_doubles() ? nb * 8 : tctf::termination_work_doubles();
  L.stat_work = take((sw + 256) * 8);
  L.kkt = take(n1 * 3 * 8);
  L.total = o;
  L.state_bytes = sizeof(StateHeader) + nb * r * n1 * 8 + nb * r * n2 * 8 + n1 * nb * n2 * welem +
                  2 * nb * r * r * 16 + nb * 4 + n1 * 3 * 8 + nb * 8 + 4 + nb * 4;
  return L;
}

struct tctf_ctx {
  tctf_params prm;
  Plan plan;
  Layout lay;
  unsigned char* ws;
  int device;
  int ncu;   // compute units of the device
  int64_t iters;
  bool term_valid;
  Knobs knobs;
  int tuned_from_cache = 0;
  bool track = false;   // step 6 evaluated after every tctf_step call (tctf_track_termination)
  bool eager = false;   // never capture or replay a graph (the allocation-free entry point)
  // stage timing of tctf_step (tctf_profile): one event pair per profiled launch
  uint32_t prof_mask = 0;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_stage;
  size_t prof_used = 0;
  // GRAPH_ITERS iterations captured once as a HIP graph (on a private stream) and replayed
  // on the context's stream
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // inside the captured graph, G_X and its inverse run on a branch beside the X~^* W~ products
  hipStream_t br_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool capturing = false;
};

#define GRAPH_ITERS 10

static tctf_status validate(const tctf_params* p) {
  if (!p) return fail(TCTF_E_ARG, "params is NULL");
  if (p->n1 < 1 || p->n2 < 1 || p->n3 < 1) return fail(TCTF_E_SHAPE, "sizes must be >= 1 (got %d x %d x %d)", p->n1, p->n2, p->n3);
  if (p->r < 1 || p->r > TCTF_RMAX || p->r > p->n1 || p->r > p->n2)
    return fail(TCTF_E_SHAPE, "rank r=%d must satisfy 1 <= r <= min(n1, n2, %d)", p->r, TCTF_RMAX);
  if (p->n1 > TCTF_N1MAX) return fail(TCTF_E_SHAPE, "n1=%d exceeds %d", p->n1, TCTF_N1MAX);
  if (p->n2 > TCTF_N2MAX) return fail(TCTF_E_SHAPE, "n2=%d exceeds %d", p->n2, TCTF_N2MAX);
  if (p->n3 > TCTF_N3MAX) return fail(TCTF_E_SHAPE, "n3=%d exceeds %d", p->n3, TCTF_N3MAX);
  if (!(std::isfinite(p->mu) && p->mu >= 0) || !(std::isfinite(p->rho1) && p->rho1 >= 0) ||
      !(std::isfinite(p->rho2) && p->rho2 >= 0))
    return fail(TCTF_E_ARG, "mu, rho1, rho2 must be finite and >= 0");
  if (!(p->eta > 0.0 && p->eta < 2.0)) return fail(TCTF_E_ARG, "eta=%g must lie in (0, 2)", p->eta);
  if (p->precision != TCTF_FP32 && p->precision != TCTF_MIXED_BF16) return fail(TCTF_E_ARG, "unknown precision %d", p->precision);
  if (p->pinv_mode != 0 && p->pinv_mode != 1) return fail(TCTF_E_ARG, "pinv_mode must be 0 or 1");
  if (!(p->eps >= 0.0)) return fail(TCTF_E_ARG, "eps must be >= 0");
  if (!(std::isfinite(p->rank_tol) && p->rank_tol >= 0.0)) return fail(TCTF_E_ARG, "rank_tol must be finite and >= 0");
  if (p->autotune != 0 && p->autotune != 1) return fail(TCTF_E_ARG, "autotune must be 0 or 1");
  if (p->rank_every < 0) return fail(TCTF_E_ARG, "rank_every must be >= 0");
  if (p->xsolve != 0 && p->xsolve != 1) return fail(TCTF_E_ARG, "xsolve must be 0 or 1");
  return TCTF_OK;
}

extern "C" {

void tctf_default_params(tctf_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mu = 1e-2;
  p->rho1 = 1e-2;
  p->rho2 = 1e-2;
  p->eta = 1.0;
  p->precision = TCTF_FP32;
  p->pinv_mode = 0;
  p->eps = 1e-6;
}

tctf_status tctf_workspace_bytes(const tctf_params* p, size_t* bytes) {
  tctf_status s = validate(p);
  if (s != TCTF_OK) return s;
  if (!bytes) return fail(TCTF_E_ARG, "bytes is NULL");
  *bytes = make_layout(*p).total;
  return TCTF_OK;
}

static void fill_plan(tctf_ctx* c, hipStream_t stream) {
  const tctf_params& p = c->prm;
  Plan& q = c->plan;
  const Layout& L = c->lay;
  unsigned char* w = c->ws;
  q.n1 = p.n1;
  q.n2 = p.n2;
  q.n3 = p.n3;
  q.r = p.r;
  q.nb = p.n3 / 2 + 1;
  q.spath = c->knobs.spath;
  q.ncu = c->ncu;
  q.g_rows = q.spath == tctf::SPATH_COOP ? 1 : 0;   // the packed G's layout follows the slice path
  q.bcg = c->knobs.bcg;
  q.ycw = c->knobs.ycw;
  q.ny = (p.n2 + q.ycw - 1) / q.ycw;
  q.mu = p.mu;
  q.rho1 = p.rho1;
  q.rho2 = p.rho2;
  q.eta = p.eta;
  q.hk = c->knobs.hstencil ? tctf::hinv_stencil(q.rho1, q.n1, q.r, q.htap) : -1;
  q.mixed = p.precision == TCTF_MIXED_BF16;
  q.force_eigen = p.pinv_mode == 1;
  q.stream = stream;
  q.gp = (float*)(w + L.gp);
  q.wt = (void*)(w + L.wt);
  q.zt = (float2*)(w + L.zt);
  q.xt = (float2*)(w + L.xt);
  q.yt = (float2*)(w + L.yt);
  q.rhs = (float2*)(w + L.rhs);
  q.bpart = (double2*)(w + L.bpart);
  q.gxpart = (cd*)(w + L.gxpart);
  q.gxm = (cd*)(w + L.gxm);
  q.dmat = (cd*)(w + L.dmat);
  q.gxp = (cd*)(w + L.gxp);
  q.qx = (cd*)(w + L.qx);
  q.qx_zero = (int*)(w + L.qx_zero);
  q.gym = (cd*)(w + L.gym);
  q.gyp = (cd*)(w + L.gyp);
  q.qy = (cd*)(w + L.qy);
  q.qy_zero = (int*)(w + L.qy_zero);
  q.slice_obj = (double*)(w + L.slice_obj);
  q.bin_obj = (double*)(w + L.bin_obj);
  q.wtab = (float*)(w + L.wtab);
  q.htab = (float*)(w + L.htab);
  q.flag = (int*)(w + L.flag);
  q.ctr = (uint32_t*)(w + L.ctr);
  q.zsp = (float*)(w + L.zsp);
  q.wsp = (float*)(w + L.wsp);
  q.csp = (float*)(w + L.csp);
  q.twg = (double2*)(w + L.twg);
  q.rsig = (double*)(w + L.rsig);
  q.rtx = (cd*)(w + L.rtx);
  q.rty = (cd*)(w + L.rty);
  q.ranks = (int*)(w + L.ranks);
  q.scal = (double*)(w + L.scal);
  q.xt_prev = (float2*)(w + L.xt_prev);
  q.yt_prev = (float2*)(w + L.yt_prev);
  q.wt_prev = (void*)(w + L.wt_prev);
  q.stat_work = (double*)(w + L.stat_work);
  q.kkt = (double*)(w + L.kkt);
}

static tctf_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TCTF_E_HIP, "kernel launch: %s", hipGetErrorString(e));
  return TCTF_OK;
}

// Launch one stage; when its bit is set in the profile mask, bracket it with two HIP events
// on the context's stream (events come from a pool that grows as needed).
extern "C++" template <typename F>
static tctf_status stage(tctf_ctx* c, int id, F&& launch) {
  if (!(c->prof_mask & (1u << id))) {
    launch();
    return TCTF_OK;
  }
  while (c->prof_used + 2 > c->prof_ev.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    c->prof_ev.push_back(e);
  }
  HIP_TRY(hipEventRecord(c->prof_ev[c->prof_used], c->plan.stream));
  launch();
  HIP_TRY(hipEventRecord(c->prof_ev[c->prof_used + 1], c->plan.stream));
  c->prof_stage.push_back(id);
  c->prof_used += 2;
  return TCTF_OK;
}

static tctf_status enqueue_iteration(tctf_ctx* c) {
  const Plan& p = c->plan;
  tctf_status s = TCTF_OK;
  if (s == TCTF_OK) s = stage(c, 2, [&] { tctf::launch_agemm(p, 0, 1); });
  if (s == TCTF_OK && p.hk < 0) s = stage(c, 3, [&] { tctf::launch_hsolve(p); });   // else inside the X-update
  if (s == TCTF_OK && c->capturing) {
    // G_X, its pseudo-inverse and I - eta P_X are needed first by the Y-step: in the graph they
    // form a branch that runs beside the X~^* W~ chunk products and joins before the Y-step
    hipError_t e = hipEventRecord(c->ev_fork, p.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->br_stream, c->ev_fork, 0);
    if (e == hipSuccess) {
      Plan pb = p;
      pb.stream = c->br_stream;
      tctf::launch_gramx(pb);
      e = hipEventRecord(c->ev_join, c->br_stream);
    }
    tctf::launch_bgemm(p);
    if (e == hipSuccess) e = hipStreamWaitEvent(p.stream, c->ev_join, 0);
    if (e != hipSuccess) s = fail(TCTF_E_HIP, "branch of the G_X launches: %s", hipGetErrorString(e));
  } else if (s == TCTF_OK) {
    s = stage(c, 4, [&] {
      tctf::launch_gramx(p);
      tctf::launch_bgemm(p);
    });
  }
  if (s == TCTF_OK) s = stage(c, 5, [&] { tctf::launch_ystep(p, 0); });
  // Z~ = X~Y~; G_Y^+ and I - eta P_Y for the next X-step ride along in extra blocks of the
  // cooperative slice launch, or of this launch on the other slice paths
  if (s == TCTF_OK) s = stage(c, 1, [&] { tctf::launch_zgemm(p, tctf::slice_hosts_pinvy(p) ? 0 : 1); });
  if (s == TCTF_OK) s = stage(c, 0, [&] { tctf::launch_slice(p, tctf::SLICE_ITER, nullptr, nullptr, 0); });
  // step 5 after iterations rank_every, 2 rank_every, ... (c->iters counts the iterations
  // before this one; such contexts never replay graphs, so the count is exact)
  if (s == TCTF_OK && c->prm.rank_every > 0 && (c->iters + 1) % c->prm.rank_every == 0)
    tctf::launch_rank_adjust(p, c->prm.rank_tol);
  if (s != TCTF_OK) return s;
  return check_launch();
}

// Set up a context in caller-provided storage (no host or device allocation): validate,
// carve the workspace, pack G and Omega, transform the initial factors, form W0, W~0 and
// the first pseudo-inverses.  On failure the context holds nothing that needs releasing.
static tctf_status ctx_init(tctf_ctx* c, const tctf_params* prm, const float* G, const uint8_t* omega,
                            const float* X0, const float* Y0, uint64_t seed, void* workspace, size_t ws_bytes,
                            void* hip_stream, const Knobs* knobs = nullptr) {
  tctf_status s = validate(prm);
  if (s != TCTF_OK) return s;
  if (!G || !omega) return fail(TCTF_E_ARG, "G and omega must be device pointers");
  const Layout L = make_layout(*prm);
  if (!workspace) return fail(TCTF_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255u) != 0) return fail(TCTF_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(TCTF_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
  c->prm = *prm;
  c->lay = L;
  c->ws = (unsigned char*)workspace;
  c->iters = 0;
  c->term_valid = false;
  c->knobs = knobs ? *knobs : default_knobs(*prm);
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return fail(TCTF_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  e = hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess) return fail(TCTF_E_HIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
  fill_plan(c, (hipStream_t)hip_stream);
  const Plan& p = c->plan;
  tctf::slice_set_attr(p.n3, tctf::slice_launch_lds_bytes(p));
  tctf::ystep_set_attr(tctf::ystep_lds_bytes(p.r, p.ycw));
  tctf::bgemm_set_attr();
  tctf::gramx_set_attr(p.r);
  tctf::pinvy_set_attr(p.r);
  tctf::zgemm_set_attr(p.r);
  tctf::launch_zero(p, p.flag, 64);
  tctf::launch_zero(p, p.ctr, 64);
  tctf::launch_rank_init(p);
  tctf::rank_set_attr(p.r);
  tctf::launch_zero(p, p.qy_zero, (size_t)p.nb * 4);
  tctf::launch_pack_g(p, G, omega);
  tctf::launch_tables(p);
  if (c->lay.split) tctf::launch_gen_twiddles(p);   // the three-launch path's roots of unity
  if (X0) tctf::launch_tube_dft_setup(p, X0, p.xt, p.n1, p.r, (long)p.r * p.n1, 1, p.n1);
  else tctf::launch_zero(p, p.xt, (size_t)p.nb * p.r * p.n1 * 8);
  const float* y0 = Y0;
  if (!y0) {
    tctf::launch_normal(p, (float*)p.zt, (size_t)p.r * p.n2 * p.n3, seed);
    y0 = (const float*)p.zt;
  }
  tctf::launch_tube_dft_setup(p, y0, p.yt, p.r, p.n2, (long)p.r * p.n2, p.n2, 1);
  tctf::launch_zgemm(p);
  tctf::launch_slice(p, tctf::SLICE_INIT, nullptr, nullptr, 1);
  tctf::launch_gramx(p);
  tctf::launch_bgemm(p);
  tctf::launch_ystep(p, 1);
  tctf::launch_pinvy(p, p.stream);
  s = check_launch();
  if (s != TCTF_OK) return s;
  int flag = 0;
  e = hipMemcpyAsync(&flag, p.flag, sizeof(int), hipMemcpyDeviceToHost, p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e != hipSuccess) return fail(TCTF_E_HIP, "create: %s", hipGetErrorString(e));
  if (flag) return fail(TCTF_E_NONFINITE, "an observed value of G is NaN or Inf");
  return TCTF_OK;
}

// Release what a context created after ctx_init (events, graph, capture stream).
static void ctx_release(tctf_ctx* c) {
  for (hipEvent_t e : c->prof_ev) hipEventDestroy(e);
  c->prof_ev.clear();
  if (c->graph_exec) {
    (void)hipStreamSynchronize(c->plan.stream);   // no replay of the graph may be in flight
    hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) hipGraphDestroy(c->graph);
  c->graph = nullptr;
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  if (c->br_stream) hipStreamDestroy(c->br_stream);
  c->br_stream = nullptr;
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  c->ev_fork = c->ev_join = nullptr;
}

static tctf_status enqueue_iteration(tctf_ctx* c);

// ---- autotuning of the execution shape: the fusion depth of steps 3, 4 and 7 (the slice
// path) and two tile shapes (rows per X~^* W~ chunk, columns per Y-step block), chosen per
// problem shape by timing and kept for the process (per device).
static std::mutex g_tune_mu;
static std::map<std::array<int, 7>, Knobs> g_tune_cache;

static std::array<int, 7> tune_key(const tctf_params& p, int device) {
  return {p.n1, p.n2, p.n3, p.r, p.precision, p.xsolve, device};
}

// Mean duration of one iteration over `reps` eager iterations after `warm`, from HIP events
// on the context's stream.  The iterate advances (the caller rebuilds it).
static tctf_status time_iterations(tctf_ctx* c, int warm, int reps, float* ms) {
  const hipStream_t st = c->plan.stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  tctf_status s = TCTF_OK;
  for (int k = 0; k < warm && s == TCTF_OK; ++k) s = enqueue_iteration(c);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int k = 0; k < reps && s == TCTF_OK; ++k) s = enqueue_iteration(c);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (s != TCTF_OK) return s;
  if (e != hipSuccess) return fail(TCTF_E_HIP, "autotune timing: %s", hipGetErrorString(e));
  *ms = t / reps;
  return TCTF_OK;
}

// Coordinate search from the default shape: each slice path the sizes allow, then the
// columns per X~^* W~ block, then the Y-step columns; every trial times a few iterations, after which the
// initial iterate is built again.  The context ends at its initial iterate with the best
// shape.
static tctf_status autotune(tctf_ctx* c, const tctf_params* prm, const float* G, const uint8_t* omega,
                            const float* X0, const float* Y0, uint64_t seed, void* ws, size_t ws_bytes,
                            void* stream) {
  const auto key = tune_key(*prm, c->device);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      const Knobs k = it->second;
      c->tuned_from_cache = 1;
      return ctx_init(c, prm, G, omega, X0, Y0, seed, ws, ws_bytes, stream, &k);
    }
  }
  const int warm = 2, reps = 6;
  Knobs best = c->knobs;
  float tbest = 0.f;
  tctf_status s = time_iterations(c, warm, reps, &tbest);
  auto trial = [&](const Knobs& k) {
    if (s != TCTF_OK) return;
    s = ctx_init(c, prm, G, omega, X0, Y0, seed, ws, ws_bytes, stream, &k);
    float t = 0.f;
    if (s == TCTF_OK) s = time_iterations(c, warm, reps, &t);
    if (s == TCTF_OK && t < tbest) {
      tbest = t;
      best = k;
    }
  };
  for (int path : {tctf::SPATH_COOP, tctf::SPATH_THREAD, tctf::SPATH_SPLIT})
    if (path != best.spath && tctf::slice_path_valid(path, prm->n2, prm->n3))
      trial({path, best.bcg, best.ycw, best.hstencil});
  for (int bcg : {16, 32})
    if (bcg != best.bcg && tctf::bgemm_cols_valid(prm->r, bcg)) trial({best.spath, bcg, best.ycw, best.hstencil});
  const int ymax = 512 / prm->r < prm->n2 ? 512 / prm->r : prm->n2;   // the Y-step block holds r x ycw <= 512
  for (int ycw : {8, 16, 32, 64, ymax})
    if (ycw != best.ycw && ycw >= TUNE_MIN_YCW && ycw <= ymax) trial({best.spath, best.bcg, ycw, best.hstencil});
  double tap[2 * HINV_KMAX + 2];
  if (best.hstencil && tctf::hinv_stencil(prm->rho1, prm->n1, prm->r, tap) >= 0)
    trial({best.spath, best.bcg, best.ycw, 0});
  if (s != TCTF_OK) return s;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = best;
  }
  return ctx_init(c, prm, G, omega, X0, Y0, seed, ws, ws_bytes, stream, &best);
}

tctf_status tctf_tuning(tctf_ctx* c, int32_t out[5]) {
  if (!c || !out) return fail(TCTF_E_ARG, "NULL argument");
  out[0] = c->knobs.spath;
  out[1] = c->knobs.bcg;
  out[2] = c->knobs.ycw;
  out[3] = c->tuned_from_cache;
  out[4] = c->plan.hk;
  return TCTF_OK;
}

tctf_status tctf_create(const tctf_params* prm, const float* G, const uint8_t* omega, const float* X0,
                        const float* Y0, uint64_t seed, void* workspace, size_t ws_bytes, void* hip_stream,
                        tctf_ctx** out) {
  if (!out) return fail(TCTF_E_ARG, "out is NULL");
  *out = nullptr;
  tctf_status s = validate(prm);
  if (s != TCTF_OK) return s;
  tctf_ctx* c = new (std::nothrow) tctf_ctx();
  if (!c) return fail(TCTF_E_ARG, "out of host memory");
  s = ctx_init(c, prm, G, omega, X0, Y0, seed, workspace, ws_bytes, hip_stream);
  if (s == TCTF_OK && prm->autotune) s = autotune(c, prm, G, omega, X0, Y0, seed, workspace, ws_bytes, hip_stream);
  if (s != TCTF_OK) {
    ctx_release(c);
    delete c;
    return s;
  }
  *out = c;
  return TCTF_OK;
}

// Capture GRAPH_ITERS iterations into a graph (once per context, by the first tctf_step call
// whatever its length, so that a warm-up pays for it).  The kernels take the same buffers
// every iteration, so one graph serves every later call.  A failed capture leaves no graph.
static tctf_status ensure_graph(tctf_ctx* c) {
  if (c->graph_exec) return TCTF_OK;
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  if (!c->br_stream) HIP_TRY(hipStreamCreateWithFlags(&c->br_stream, hipStreamNonBlocking));
  if (!c->ev_fork) HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  if (!c->ev_join) HIP_TRY(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  const hipStream_t user = c->plan.stream;
  c->plan.stream = c->cap_stream;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  tctf_status s = TCTF_OK;
  if (e == hipSuccess) {
    c->capturing = true;
    for (int k = 0; k < GRAPH_ITERS && s == TCTF_OK; ++k) s = enqueue_iteration(c);
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (s == TCTF_OK && e2 == hipSuccess) {
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (e == hipSuccess) {
        c->graph = g;
        c->graph_exec = x;
      } else {
        hipGraphDestroy(g);
      }
    } else {
      if (g) hipGraphDestroy(g);
      if (e2 != hipSuccess) e = e2;
    }
  }
  c->plan.stream = user;
  if (s != TCTF_OK) return s;
  if (e != hipSuccess) return fail(TCTF_E_HIP, "graph capture of the iteration: %s", hipGetErrorString(e));
  return TCTF_OK;
}

tctf_status tctf_step(tctf_ctx* c, int32_t iters) {
  if (!c) return fail(TCTF_E_ARG, "context is NULL");
  if (iters < 0) return fail(TCTF_E_ARG, "iters must be >= 0");
  if (iters == 0) return TCTF_OK;
  const Plan& p = c->plan;
  // whole blocks of GRAPH_ITERS iterations as graph replays (not while stages are being
  // timed); when step 6 is tracked the last iteration runs eagerly after the snapshot
  const int32_t body = c->track ? iters - 1 : iters;
  int32_t it = 0;
  if (c->prof_mask == 0 && !c->eager && c->prm.rank_every == 0) {
    tctf_status s = ensure_graph(c);
    if (s != TCTF_OK) return s;
    for (; body - it >= GRAPH_ITERS; it += GRAPH_ITERS) {
      HIP_TRY(hipGraphLaunch(c->graph_exec, p.stream));
      c->iters += GRAPH_ITERS;
    }
  }
  for (; it < iters; ++it) {
    if (c->track && it == iters - 1) {
      const size_t welem = tctf::wt_elem_bytes(p);
      HIP_TRY(hipMemcpyAsync(p.xt_prev, p.xt, (size_t)p.nb * p.r * p.n1 * 8, hipMemcpyDeviceToDevice, p.stream));
      HIP_TRY(hipMemcpyAsync(p.yt_prev, p.yt, (size_t)p.nb * p.r * p.n2 * 8, hipMemcpyDeviceToDevice, p.stream));
      HIP_TRY(hipMemcpyAsync(p.wt_prev, p.wt, (size_t)p.n1 * p.nb * p.n2 * welem, hipMemcpyDeviceToDevice, p.stream));
    }
    tctf_status s = enqueue_iteration(c);
    if (s != TCTF_OK) return s;
    c->iters++;
  }
  if (c->track) {
    tctf::launch_termination(p);
    c->term_valid = true;
  }
  return check_launch();
}

tctf_status tctf_track_termination(tctf_ctx* c, int32_t on) {
  if (!c) return fail(TCTF_E_ARG, "context is NULL");
  c->track = on != 0;
  return TCTF_OK;
}

static tctf_status read_scalars(tctf_ctx* c, int first, int count, double* dst) {
  const Plan& p = c->plan;
  HIP_TRY(hipMemcpyAsync(dst, p.scal + first, count * sizeof(double), hipMemcpyDeviceToHost, p.stream));
  HIP_TRY(hipStreamSynchronize(p.stream));
  return TCTF_OK;
}

tctf_status tctf_objective(tctf_ctx* c, double* f0) {
  if (!c || !f0) return fail(TCTF_E_ARG, "NULL argument");
  tctf::launch_objective(c->plan);
  tctf_status s = check_launch();
  if (s != TCTF_OK) return s;
  s = read_scalars(c, 0, 1, f0);
  if (s != TCTF_OK) return s;
  if (!std::isfinite(*f0)) return fail(TCTF_E_NONFINITE, "objective is not finite");
  return TCTF_OK;
}

tctf_status tctf_termination(tctf_ctx* c, double out[4]) {
  if (!c || !out) return fail(TCTF_E_ARG, "NULL argument");
  if (!c->term_valid)
    return fail(TCTF_E_STATE, "no tracked iteration since create or restore (tctf_track_termination or tctf_run)");
  tctf_status s = read_scalars(c, 4, 3, out);
  if (s != TCTF_OK) return s;
  if (!std::isfinite(out[0]) || !std::isfinite(out[1]) || !std::isfinite(out[2]))
    return fail(TCTF_E_NONFINITE, "the iterate is not finite (step-6 differences %g %g %g)", out[0], out[1], out[2]);
  const double eps = c->prm.eps;
  out[3] = (out[0] <= eps && out[1] <= eps && out[2] <= eps) ? 1.0 : 0.0;
  return TCTF_OK;
}

tctf_status tctf_run(tctf_ctx* c, int32_t max_iters, int32_t check_every, int32_t* iters_run,
                     int32_t* converged) {
  if (!c || !iters_run || !converged) return fail(TCTF_E_ARG, "NULL argument");
  if (max_iters < 0 || check_every < 1) return fail(TCTF_E_ARG, "max_iters must be >= 0 and check_every >= 1");
  *iters_run = 0;
  *converged = 0;
  const bool was_tracking = c->track;
  c->track = true;
  tctf_status s = TCTF_OK;
  while (*iters_run < max_iters) {
    const int32_t k = check_every < max_iters - *iters_run ? check_every : max_iters - *iters_run;
    s = tctf_step(c, k);
    if (s != TCTF_OK) break;
    *iters_run += k;
    double t[4];
    s = tctf_termination(c, t);
    if (s != TCTF_OK) break;
    if (t[3] != 0.0) {
      *converged = 1;
      break;
    }
  }
  c->track = was_tracking;
  return s;
}

tctf_status tctf_stationarity(tctf_ctx* c, double out[3]) {
  if (!c || !out) return fail(TCTF_E_ARG, "NULL argument");
  tctf::launch_stationarity(c->plan, c->iters == 0 ? 1 : 0);
  tctf_status s = check_launch();
  if (s != TCTF_OK) return s;
  s = read_scalars(c, 8, 3, out);
  if (s != TCTF_OK) return s;
  if (!std::isfinite(out[0]) || !std::isfinite(out[1]) || !std::isfinite(out[2]))
    return fail(TCTF_E_NONFINITE, "the iterate is not finite (stationarity %g %g %g)", out[0], out[1], out[2]);
  return TCTF_OK;
}

tctf_status tctf_get_result(tctf_ctx* c, float* W, float* Z, float* X, float* Y) {
  if (!c) return fail(TCTF_E_ARG, "context is NULL");
  const Plan& p = c->plan;
  if (W || Z) {
    tctf::launch_zgemm(p);
    tctf::launch_slice(p, tctf::SLICE_RESULT, W, Z, c->iters == 0 ? 1 : 0);
  }
  if (X) tctf::launch_tube_idft_setup(p, p.xt, X, p.n1, p.r, (long)p.r * p.n1, 1, p.n1);
  if (Y) tctf::launch_tube_idft_setup(p, p.yt, Y, p.r, p.n2, (long)p.r * p.n2, p.n2, 1);
  tctf_status s = check_launch();
  if (s != TCTF_OK) return s;
  HIP_TRY(hipStreamSynchronize(p.stream));
  return TCTF_OK;
}

// checkpoint blob: header, X~, Y~, W~, G_Y^+, I - eta P_Y, flags, objective partials
struct Region { size_t off; size_t bytes; };

static int state_regions(tctf_ctx* c, Region* r) {
  const Plan& p = c->plan;
  const Layout& L = c->lay;
  const size_t welem = tctf::wt_elem_bytes(p);
  int n = 0;
  r[n++] = {L.xt, (size_t)p.nb * p.r * p.n1 * 8};
  r[n++] = {L.yt, (size_t)p.nb * p.r * p.n2 * 8};
  r[n++] = {L.wt, (size_t)p.n1 * p.nb * p.n2 * welem};
  r[n++] = {L.gyp, (size_t)p.nb * p.r * p.r * 16};
  r[n++] = {L.qy, (size_t)p.nb * p.r * p.r * 16};
  r[n++] = {L.qy_zero, (size_t)p.nb * 4};
  r[n++] = {L.slice_obj, (size_t)p.n1 * 3 * 8};
  r[n++] = {L.bin_obj, (size_t)p.nb * 8};
  r[n++] = {L.ctr, 4};
  r[n++] = {L.ranks, (size_t)p.nb * 4};
  return n;
}

tctf_status tctf_state_bytes(tctf_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(TCTF_E_ARG, "NULL argument");
  *bytes = c->lay.state_bytes;
  return TCTF_OK;
}

tctf_status tctf_get_state(tctf_ctx* c, void* dst, size_t bytes) {
  if (!c || !dst) return fail(TCTF_E_ARG, "NULL argument");
  if (bytes < c->lay.state_bytes) return fail(TCTF_E_STATE, "state buffer has %zu bytes, %zu needed", bytes, c->lay.state_bytes);
  const Plan& p = c->plan;
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kStateMagic;
  h.n1 = p.n1; h.n2 = p.n2; h.n3 = p.n3; h.r = p.r; h.precision = c->prm.precision;
  h.iters = c->iters;
  unsigned char* d = (unsigned char*)dst;
  HIP_TRY(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, p.stream));
  size_t off = sizeof(h);
  Region reg[16];
  const int n = state_regions(c, reg);
  for (int k = 0; k < n; ++k) {
    HIP_TRY(hipMemcpyAsync(d + off, c->ws + reg[k].off, reg[k].bytes, hipMemcpyDeviceToDevice, p.stream));
    off += reg[k].bytes;
  }
  HIP_TRY(hipStreamSynchronize(p.stream));
  return TCTF_OK;
}

tctf_status tctf_set_state(tctf_ctx* c, const void* src, size_t bytes) {
  if (!c || !src) return fail(TCTF_E_ARG, "NULL argument");
  if (bytes < c->lay.state_bytes) return fail(TCTF_E_STATE, "state blob has %zu bytes, %zu needed", bytes, c->lay.state_bytes);
  const Plan& p = c->plan;
  StateHeader h;
  const unsigned char* s = (const unsigned char*)src;
  HIP_TRY(hipMemcpyAsync(&h, s, sizeof(h), hipMemcpyDeviceToHost, p.stream));
  HIP_TRY(hipStreamSynchronize(p.stream));
  if (h.magic != kStateMagic || h.n1 != p.n1 || h.n2 != p.n2 || h.n3 != p.n3 || h.r != p.r ||
      h.precision != c->prm.precision)
    return fail(TCTF_E_STATE, "state blob belongs to another problem");
  size_t off = sizeof(h);
  Region reg[16];
  const int n = state_regions(c, reg);
  for (int k = 0; k < n; ++k) {
    HIP_TRY(hipMemcpyAsync(c->ws + reg[k].off, s + off, reg[k].bytes, hipMemcpyDeviceToDevice, p.stream));
    off += reg[k].bytes;
  }
  HIP_TRY(hipStreamSynchronize(p.stream));
  c->iters = h.iters;
  c->term_valid = false;
  return TCTF_OK;
}

tctf_status tctf_rank_vector(tctf_ctx* c, int32_t* ranks) {
  if (!c || !ranks) return fail(TCTF_E_ARG, "NULL argument");
  HIP_TRY(hipMemcpyAsync(ranks, c->plan.ranks, (size_t)c->plan.nb * 4, hipMemcpyDeviceToHost, c->plan.stream));
  HIP_TRY(hipStreamSynchronize(c->plan.stream));
  return TCTF_OK;
}

tctf_status tctf_iterations(tctf_ctx* c, int64_t* iters) {
  if (!c || !iters) return fail(TCTF_E_ARG, "NULL argument");
  *iters = c->iters;
  return TCTF_OK;
}

void tctf_destroy(tctf_ctx* c) {
  if (!c) return;
  ctx_release(c);
  delete c;
}

tctf_status tctf_profile(tctf_ctx* c, uint32_t mask) {
  if (!c) return fail(TCTF_E_ARG, "context is NULL");
  if (mask >> 7) return fail(TCTF_E_ARG, "profile mask 0x%x has bits beyond stage 6", mask);
  if (mask) {
    c->prof_used = 0;
    c->prof_stage.clear();
  }
  c->prof_mask = mask;
  return TCTF_OK;
}

tctf_status tctf_profile_read(tctf_ctx* c, double total_us[7], int64_t launches[7]) {
  if (!c || !total_us || !launches) return fail(TCTF_E_ARG, "NULL argument");
  for (int k = 0; k < 7; ++k) {
    total_us[k] = 0.0;
    launches[k] = 0;
  }
  HIP_TRY(hipStreamSynchronize(c->plan.stream));
  for (size_t q = 0; q < c->prof_stage.size(); ++q) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->prof_ev[2 * q], c->prof_ev[2 * q + 1]));
    total_us[c->prof_stage[q]] += 1000.0 * ms;
    launches[c->prof_stage[q]] += 1;
  }
  return TCTF_OK;
}

tctf_status tctf_complete(const tctf_params* p, const float* G, const uint8_t* omega, const float* X0,
                          const float* Y0, uint64_t seed, int32_t iters, void* workspace, size_t ws_bytes,
                          void* hip_stream, float* W_out, double* f0_out) {
  if (!W_out) return fail(TCTF_E_ARG, "W_out is NULL");
  tctf_ctx* c = nullptr;
  tctf_status s = tctf_create(p, G, omega, X0, Y0, seed, workspace, ws_bytes, hip_stream, &c);
  if (s != TCTF_OK) return s;
  s = tctf_step(c, iters);
  if (s == TCTF_OK) s = tctf_get_result(c, W_out, nullptr, nullptr, nullptr);
  if (s == TCTF_OK && f0_out) s = tctf_objective(c, f0_out);
  tctf_destroy(c);
  return s;
}

}  // extern "C"

// Static scratch of the allocation-free entry point: one copy per device, held by the device
// from module load until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code the name is only a stand-in); it uses the device address that
// hipGetSymbolAddress returns for the current device, fetched once per device.
static __device__ __align__(256) unsigned char scratch[TCTF_NOALLOC_SCRATCH_BYTES];
#define NOALLOC_MAX_DEVICES 64
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static tctf_status scratch_address(int device, void** ptr) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(TCTF_E_HIP, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(TCTF_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return TCTF_OK;
}

extern "C" {

tctf_status tctf_complete_noalloc(const tctf_params* p, const float* G, const uint8_t* omega, const float* X0,
                                  const float* Y0, uint64_t seed, int32_t iters, void* hip_stream, float* W_out,
                                  double* f0_out) {
  if (!W_out) return fail(TCTF_E_ARG, "W_out is NULL");
  if (iters < 0) return fail(TCTF_E_ARG, "iters must be >= 0");
  tctf_status s = validate(p);
  if (s != TCTF_OK) return s;
  const size_t need = make_layout(*p).total;
  if (need > (size_t)TCTF_NOALLOC_SCRATCH_BYTES)
    return fail(TCTF_E_WORKSPACE, "problem needs %zu bytes of scratch; the static scratch holds %zu", need,
                (size_t)TCTF_NOALLOC_SCRATCH_BYTES);
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  void* ws = nullptr;
  s = scratch_address(device, &ws);
  if (s != TCTF_OK) return s;
  tctf_ctx c;   // on the stack: no host allocation either (its vectors stay empty)
  c.eager = true;
  s = ctx_init(&c, p, G, omega, X0, Y0, seed, ws, need, hip_stream);
  if (s == TCTF_OK) s = tctf_step(&c, iters);
  if (s == TCTF_OK) s = tctf_get_result(&c, W_out, nullptr, nullptr, nullptr);
  if (s == TCTF_OK && f0_out) s = tctf_objective(&c, f0_out);
  ctx_release(&c);
  return s;
}

tctf_status tctf_time_stage(tctf_ctx* c, int32_t stage, int32_t reps, double* mean_us) {
  if (!c || !mean_us) return fail(TCTF_E_ARG, "NULL argument");
  if (stage < 0 || stage > 7 || reps < 1) return fail(TCTF_E_ARG, "stage must be 0..7 and reps >= 1");
  const Plan& p = c->plan;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, p.stream));
  for (int k = 0; k < reps; ++k) {
    switch (stage) {
      case 0: tctf::launch_slice(p, tctf::SLICE_ITER, nullptr, nullptr, 0); break;
      case 1: tctf::launch_zgemm(p); break;
      case 2: tctf::launch_agemm(p, 0, 0, 1); break;
      case 3: if (p.hk < 0) tctf::launch_hsolve(p); break;
      case 4: tctf::launch_gramx(p); tctf::launch_bgemm(p); break;
      case 5: tctf::launch_ystep(p, 1); break;
      case 6: tctf::launch_pinvy(p, p.stream); break;
      case 7: enqueue_iteration(c); c->iters++; break;
    }
  }
  HIP_TRY(hipEventRecord(e1, p.stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *mean_us = 1000.0 * ms / reps;
  return check_launch();
}

// ---- differentiation
static tctf_status adjoint_plan(const tctf_params* prm, Plan* q) {
  tctf_status s = validate(prm);
  if (s != TCTF_OK) return s;
  if (prm->precision != TCTF_FP32) return fail(TCTF_E_ARG, "the adjoint supports FP32 contexts only");
  std::memset((void*)q, 0, sizeof(*q));
  q->n1 = prm->n1;
  q->n2 = prm->n2;
  q->n3 = prm->n3;
  q->r = prm->r;
  q->nb = prm->n3 / 2 + 1;
  return TCTF_OK;
}

tctf_status tctf_adjoint_workspace_bytes(const tctf_params* p, size_t* bytes) {
  if (!bytes) return fail(TCTF_E_ARG, "bytes is NULL");
  Plan q;
  tctf_status s = adjoint_plan(p, &q);
  if (s != TCTF_OK) return s;
  *bytes = tctf::adjoint_work_bytes(q);
  return TCTF_OK;
}

static tctf_status adjoint_workspace(tctf_ctx* c, void* ws, size_t ws_bytes, tctf::AdjWork* w) {
  if (c->prm.precision != TCTF_FP32) return fail(TCTF_E_ARG, "the adjoint supports FP32 contexts only");
  if (!ws) return fail(TCTF_E_WORKSPACE, "adjoint workspace is NULL");
  if (((uintptr_t)ws & 255u) != 0) return fail(TCTF_E_WORKSPACE, "adjoint workspace must be 256-byte aligned");
  const size_t need = tctf::adjoint_work_bytes(c->plan);
  if (ws_bytes < need) return fail(TCTF_E_WORKSPACE, "adjoint workspace has %zu bytes, %zu needed", ws_bytes, need);
  tctf::adjoint_carve(c->plan, ws, w);
  tctf::adjoint_set_attr(c->plan.r);
  return TCTF_OK;
}

// Header of a checkpoint blob in device memory, checked against the context.
static tctf_status blob_header(tctf_ctx* c, const void* blob, StateHeader* h) {
  HIP_TRY(hipMemcpyAsync(h, blob, sizeof(*h), hipMemcpyDeviceToHost, c->plan.stream));
  HIP_TRY(hipStreamSynchronize(c->plan.stream));
  if (h->magic != kStateMagic || h->n1 != c->plan.n1 || h->n2 != c->plan.n2 || h->n3 != c->plan.n3 ||
      h->r != c->plan.r || h->precision != c->prm.precision)
    return fail(TCTF_E_STATE, "state blob belongs to another problem");
  return TCTF_OK;
}

static tctf::AdjState blob_state(tctf_ctx* c, const void* blob) {
  const Plan& p = c->plan;
  const unsigned char* b = (const unsigned char*)blob + sizeof(StateHeader);
  tctf::AdjState st;
  st.xt = (const float2*)b;
  st.yt = (const float2*)(b + (size_t)p.nb * p.r * p.n1 * 8);
  st.wt = (const float2*)(b + (size_t)p.nb * p.r * p.n1 * 8 + (size_t)p.nb * p.r * p.n2 * 8);
  return st;
}

tctf_status tctf_adjoint_step(tctf_ctx* c, const void* state_in, const void* state_out, double* xt_bar,
                              double* yt_bar, double* w_bar, double* theta_bar, void* workspace, size_t ws_bytes) {
  if (!c || !state_in || !state_out || !xt_bar || !yt_bar || !w_bar || !theta_bar)
    return fail(TCTF_E_ARG, "NULL argument");
  tctf::AdjWork w;
  tctf_status s = adjoint_workspace(c, workspace, ws_bytes, &w);
  if (s != TCTF_OK) return s;
  StateHeader hi, ho;
  if ((s = blob_header(c, state_in, &hi)) != TCTF_OK) return s;
  if ((s = blob_header(c, state_out, &ho)) != TCTF_OK) return s;
  if (ho.iters != hi.iters + 1)
    return fail(TCTF_E_STATE, "state_out (iteration %lld) must follow state_in (iteration %lld) by one iteration",
                (long long)ho.iters, (long long)hi.iters);
  tctf::launch_adjoint_step(c->plan, w, blob_state(c, state_in), blob_state(c, state_out), (double2*)xt_bar,
                            (double2*)yt_bar, w_bar, theta_bar);
  s = check_launch();
  if (s != TCTF_OK) return s;
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, c->plan.stream));
  HIP_TRY(hipStreamSynchronize(c->plan.stream));
  if (flag) return fail(TCTF_E_STATE, "a Gram of this iteration is rank deficient; the adjoint needs full rank");
  return TCTF_OK;
}

tctf_status tctf_adjoint_initial(tctf_ctx* c, const double* xt_bar, const double* yt_bar, double* x0_bar,
                                 double* y0_bar) {
  if (!c || !xt_bar || !yt_bar) return fail(TCTF_E_ARG, "NULL argument");
  tctf::launch_adjoint_initial(c->plan, (const double2*)xt_bar, (const double2*)yt_bar, x0_bar, y0_bar);
  return check_launch();
}

tctf_status tctf_objective_gradient(tctf_ctx* c, double* x_grad, double* y_grad, void* workspace, size_t ws_bytes) {
  if (!c || !x_grad || !y_grad) return fail(TCTF_E_ARG, "NULL argument");
  tctf::AdjWork w;
  tctf_status s = adjoint_workspace(c, workspace, ws_bytes, &w);
  if (s != TCTF_OK) return s;
  tctf::launch_objective_gradient(c->plan, w, x_grad, y_grad);
  s = check_launch();
  if (s != TCTF_OK) return s;
  HIP_TRY(hipStreamSynchronize(c->plan.stream));
  return TCTF_OK;
}

const char* tctf_status_string(tctf_status s) {
  switch (s) {
    case TCTF_OK: return "ok";
    case TCTF_E_ARG: return "invalid argument";
    case TCTF_E_SHAPE: return "unsupported shape";
    case TCTF_E_NONFINITE: return "non-finite value";
    case TCTF_E_HIP: return "HIP runtime error";
    case TCTF_E_WORKSPACE: return "bad workspace";
    case TCTF_E_STATE: return "bad state";
  }
  return "unknown status";
}

const char* tctf_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------ batches of completions
// Independent completions (the frequencies and rows of one completion are already
// independent work units; several completions are one level up).  Blocks of GRAPH_ITERS
// iterations of every member are captured once into a single graph in which each member's
// chain is its own branch, so one launch runs all members and the runtime may overlap them.
struct tctf_batch {
  std::vector<tctf_ctx*> members;
  std::vector<hipStream_t> streams;   // capture streams, one branch each
  hipStream_t origin = nullptr;       // capture origin
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> done_ev;
  hipGraph_t graph[2] = {nullptr, nullptr};          // [0]: GRAPH_ITERS iterations, [1]: one
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  hipStream_t stream = nullptr;       // the caller's stream
};

#define BATCH_BRANCHES 16

extern "C" {

tctf_status tctf_batch_workspace_bytes(int32_t n, const tctf_params* p, size_t* bytes) {
  if (n < 1 || !p || !bytes) return fail(TCTF_E_ARG, "n must be >= 1 and pointers non-NULL");
  size_t total = 0;
  for (int32_t k = 0; k < n; ++k) {
    size_t b = 0;
    tctf_status s = tctf_workspace_bytes(&p[k], &b);
    if (s != TCTF_OK) return s;
    total += align256(b);
  }
  *bytes = total;
  return TCTF_OK;
}

void tctf_batch_destroy(tctf_batch* b) {
  if (!b) return;
  if (b->graph_exec[0] || b->graph_exec[1]) (void)hipStreamSynchronize(b->stream);
  for (int k = 0; k < 2; ++k) {
    if (b->graph_exec[k]) hipGraphExecDestroy(b->graph_exec[k]);
    if (b->graph[k]) hipGraphDestroy(b->graph[k]);
  }
  for (hipEvent_t e : b->done_ev) hipEventDestroy(e);
  if (b->fork_ev) hipEventDestroy(b->fork_ev);
  for (hipStream_t s : b->streams) hipStreamDestroy(s);
  if (b->origin) hipStreamDestroy(b->origin);
  for (tctf_ctx* c : b->members) tctf_destroy(c);
  delete b;
}

tctf_status tctf_batch_create(int32_t n, const tctf_params* p, const float* const* G, const uint8_t* const* omega,
                              const float* const* X0, const float* const* Y0, const uint64_t* seeds,
                              void* workspace, size_t ws_bytes, void* hip_stream, tctf_batch** out) {
  if (!out) return fail(TCTF_E_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || !p || !G || !omega) return fail(TCTF_E_ARG, "n must be >= 1; p, G and omega non-NULL");
  size_t need = 0;
  tctf_status s = tctf_batch_workspace_bytes(n, p, &need);
  if (s != TCTF_OK) return s;
  if (!workspace) return fail(TCTF_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255u) != 0) return fail(TCTF_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(TCTF_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  tctf_batch* b = new (std::nothrow) tctf_batch();
  if (!b) return fail(TCTF_E_ARG, "out of host memory");
  b->stream = (hipStream_t)hip_stream;
  unsigned char* w = (unsigned char*)workspace;
  for (int32_t k = 0; k < n; ++k) {
    size_t bytes = 0;
    (void)tctf_workspace_bytes(&p[k], &bytes);
    if (p[k].rank_every != 0) {
      tctf_batch_destroy(b);
      return fail(TCTF_E_ARG, "member %d: batches run step 5 never (rank_every must be 0)", k);
    }
    tctf_ctx* c = nullptr;
    s = tctf_create(&p[k], G[k], omega[k], X0 ? X0[k] : nullptr, Y0 ? Y0[k] : nullptr, seeds ? seeds[k] : 0, w,
                    align256(bytes), hip_stream, &c);
    if (s != TCTF_OK) {
      const std::string why = g_err;
      tctf_batch_destroy(b);
      return fail(s, "member %d: %s", k, why.c_str());
    }
    b->members.push_back(c);
    w += align256(bytes);
  }
  *out = b;
  return TCTF_OK;
}

// Graph k of the batch: GRAPH_ITERS iterations (k = 0) or one (k = 1) of every member, each
// member's chain on one of the branches.  A failed capture leaves no graph.
static tctf_status batch_graph(tctf_batch* b, int k) {
  if (b->graph_exec[k]) return TCTF_OK;
  const int iters = k == 0 ? GRAPH_ITERS : 1;
  const int nbr = (int)b->members.size() < BATCH_BRANCHES ? (int)b->members.size() : BATCH_BRANCHES;
  if (!b->origin) HIP_TRY(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking));
  if (!b->fork_ev) HIP_TRY(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  while ((int)b->streams.size() < nbr) {
    hipStream_t st;
    hipEvent_t ev;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    b->streams.push_back(st);
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->done_ev.push_back(ev);
  }
  HIP_TRY(hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipEventRecord(b->fork_ev, b->origin);
  tctf_status s = TCTF_OK;
  for (int q = 0; q < nbr && e == hipSuccess && s == TCTF_OK; ++q) {
    e = hipStreamWaitEvent(b->streams[q], b->fork_ev, 0);
    for (int it = 0; it < iters && e == hipSuccess && s == TCTF_OK; ++it) {
      for (size_t m = q; m < b->members.size() && s == TCTF_OK; m += nbr) {
        tctf_ctx* c = b->members[m];
        const hipStream_t user = c->plan.stream;
        const int ncu = c->plan.ncu;
        c->plan.stream = b->streams[q];
        c->plan.ncu = 0;   // members share the compute units: no launch reserves one for itself
        s = enqueue_iteration(c);
        c->plan.stream = user;
        c->plan.ncu = ncu;
      }
    }
    if (e == hipSuccess) e = hipEventRecord(b->done_ev[q], b->streams[q]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->origin, b->done_ev[q], 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->origin, &g);
  if (s != TCTF_OK || e != hipSuccess || e2 != hipSuccess) {
    if (g) hipGraphDestroy(g);
    if (s != TCTF_OK) return s;
    return fail(TCTF_E_HIP, "graph capture of the batch: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return fail(TCTF_E_HIP, "graph instantiation of the batch: %s", hipGetErrorString(e));
  }
  b->graph[k] = g;
  b->graph_exec[k] = x;
  return TCTF_OK;
}

tctf_status tctf_batch_step(tctf_batch* b, int32_t iters) {
  if (!b) return fail(TCTF_E_ARG, "batch is NULL");
  if (iters < 0) return fail(TCTF_E_ARG, "iters must be >= 0");
  if (iters == 0) return TCTF_OK;
  // every iteration of every member runs inside a graph launch: blocks of GRAPH_ITERS, then
  // the one-iteration graph for the remainder (both captured by the first call)
  for (int k = 0; k < 2; ++k) {
    tctf_status s = batch_graph(b, k);
    if (s != TCTF_OK) return s;
  }
  int32_t it = 0;
  for (; iters - it >= GRAPH_ITERS; it += GRAPH_ITERS) HIP_TRY(hipGraphLaunch(b->graph_exec[0], b->stream));
  for (; it < iters; ++it) HIP_TRY(hipGraphLaunch(b->graph_exec[1], b->stream));
  for (tctf_ctx* c : b->members) {
    c->iters += iters;
    c->term_valid = false;   // step 6 is not evaluated inside batch graphs
  }
  return TCTF_OK;
}

tctf_status tctf_batch_size(tctf_batch* b, int32_t* n) {
  if (!b || !n) return fail(TCTF_E_ARG, "NULL argument");
  *n = (int32_t)b->members.size();
  return TCTF_OK;
}

tctf_status tctf_batch_member(tctf_batch* b, int32_t k, tctf_ctx** member) {
  if (!b || !member) return fail(TCTF_E_ARG, "NULL argument");
  if (k < 0 || k >= (int32_t)b->members.size()) return fail(TCTF_E_ARG, "member %d out of range", k);
  *member = b->members[k];
  return TCTF_OK;
}

}  // extern "C"

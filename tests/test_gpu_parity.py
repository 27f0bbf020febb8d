"""HIP path against the FP64 oracle on the same seeded inputs (needs an MI355X).

Tolerances (FP32 GPU against the FP64 oracle, same inputs and the same initial factors):
* relative Frobenius error <= 1e-5 for W, Z and f0;
* element-wise: max |A_gpu - A_oracle| <= 1e-5 max |A_oracle| for A = W and Z;
* per OD pair (mode-1 slice i): ||A_gpu(i) - A_oracle(i)|| <= TOL_ROW ||A_oracle(i)||, so that
  an error confined to low-volume OD rows (heavy-tailed scales) or to the ragged tails of
  the tiles cannot hide under the norm of the large rows.
"""
import numpy as np
import pytest

from tests.gpu_helpers import gpu_run, make_inputs, make_workload, oracle, oracle_run, rel

pytestmark = pytest.mark.gpu
TOL = 1e-5
TOL_MAX = 1e-5
TOL_ROW = 5e-5


def elementwise(a, ref):
    """(relative Frobenius error, max error / max |ref|, worst per-row relative error, its row)."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    d = (a - ref).reshape(ref.shape[0], -1)
    rn = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    dn = np.linalg.norm(d, axis=1)
    rowrel = np.where(dn == 0.0, 0.0, dn / np.maximum(rn, 1e-30))
    emax = float(np.abs(d).max() / max(np.abs(ref).max(), 1e-30)) if ref.size else 0.0
    worst = int(np.argmax(rowrel)) if ref.size else 0
    return rel(a, ref), emax, float(rowrel.max()) if ref.size else 0.0, worst


def _compare(g, st, info=None, tol=TOL, label="", tol_max=TOL_MAX, tol_row=TOL_ROW):
    msg = label
    ok = True
    for name, ref in (("W", st.w), ("Z", oracle.z_of(st))):
        fro, emax, erow, irow = elementwise(g[name], ref)
        msg += f" | {name} fro {fro:.2e} max {emax:.2e} row {erow:.2e} (i={irow})"
        ok = ok and fro <= tol and emax <= tol_max and erow <= tol_row
    if info is not None and info["f0"]:
        ef = abs(g["f0"][-1] - info["f0"][-1]) / max(abs(info["f0"][-1]), 1e-30)
        msg += f" | f0 {ef:.2e}"
        ok = ok and ef <= tol
    print(msg, flush=True)
    assert ok, msg


def test_smallest_workload_50_iterations():
    """36 x 48 x 7, r = 3, 30 % sampled, 50 iterations, FP32 vs FP64: W, Z and the f0 history."""
    w, d = make_workload("od36x48x7_r3")
    g = gpu_run(d, w.r, w.iters, history=True)
    st, info = oracle_run(d, w.r, w.iters, history=True)
    _compare(g, st, info, label=w.name)
    f_g, f_o = np.array(g["f0"]), np.array(info["f0"])
    assert np.max(np.abs(f_g - f_o) / np.abs(f_o)) <= TOL


@pytest.mark.parametrize("n1,n2,n3,r,p", [
    (70, 50, 9, 5, 0.4),      # ragged against 16-row, 64-column and 64-lane tiles; odd tube
    (33, 17, 12, 4, 0.3),     # even tube with a Nyquist frequency
    (5, 3, 1, 2, 0.5),        # n3 = 1: matrix case
    (1, 9, 4, 1, 0.5),        # n1 = 1: H is empty
    (12, 1, 6, 1, 0.5),       # n2 = 1: K is empty
    (40, 65, 28, 6, 0.25),    # tube of 28 days, n2 just above a 64-column tile
    (130, 20, 16, 8, 0.6),    # several 64-row chunks in the n1 reduction
    (48, 40, 6, 20, 0.7),     # r > 16: the largest rank bucket of the products and pivots
    (1100, 9, 4, 2, 0.5),     # n1 > 1024: the column-in-LDS H solve
    (300, 12, 6, 3, 0.4),     # n1 past one round of compute units, two row groups of G_X
    (20, 30, 24, 3, 0.4),     # tube transforms with two step-C groups per thread: 24 = 2 (4 x 3),
    (24, 70, 32, 4, 0.5),     # 32 = 2 (4 x 4),
    (18, 40, 48, 3, 0.4),     # 48 = 2 (6 x 4),
    (16, 20, 96, 4, 0.5),     # 96 = 2 (8 x 6)
    (12, 130, 128, 5, 0.4),   # and 128 = 2 (8 x 8) with n2 past two 64-column groups
])
def test_ragged_shapes(n1, n2, n3, r, p):
    d = make_inputs(n1, n2, n3, r, p=p, seed=n1 + n2 + n3, weekly=True, sigma_od=1.0, noise=0.02)
    g = gpu_run(d, r, 8)
    st, info = oracle_run(d, r, 8, history=True)
    _compare(g, st, info, label=f"{n1}x{n2}x{n3} r{r}")


@pytest.mark.parametrize("mu,rho1,rho2,eta", [(0.0, 0.0, 0.0, 1.0), (0.3, 0.0, 0.7, 1.0), (0.05, 0.8, 0.0, 1.0),
                                              (1e-2, 1e-2, 1e-2, 0.6), (0.1, 0.2, 0.3, 1.4)])
def test_parameters(mu, rho1, rho2, eta):
    d = make_inputs(24, 30, 10, 3, p=0.4, seed=7)
    g = gpu_run(d, 3, 6, mu=mu, rho1=rho1, rho2=rho2, eta=eta)
    st, info = oracle_run(d, 3, 6, mu=mu, rho1=rho1, rho2=rho2, eta=eta, history=True)
    _compare(g, st, info, label=f"mu{mu} rho1{rho1} rho2{rho2} eta{eta}")


@pytest.mark.parametrize("p", [0.0, 1.0])
def test_sampling_extremes(p):
    """Nothing observed (W = Z / (1 + mu) smoothed) and everything observed (W = G)."""
    d = make_inputs(20, 16, 8, 3, p=p, seed=3)
    g = gpu_run(d, 3, 5)
    st, info = oracle_run(d, 3, 5, history=True)
    _compare(g, st, info, label=f"p={p}")
    if p == 1.0:
        assert np.array_equal(g["W"], d["G"].astype(np.float64))


@pytest.mark.parametrize("n1,n2,n3,r,rho1,eta", [
    (300, 40, 12, 6, 1e-2, 1.0),   # stencil half-width 5, five row blocks per frequency
    (300, 40, 12, 6, 0.1, 0.7),    # half-width 11 with the X~ (I - eta P_Y) term; Nyquist bin
    (12, 20, 8, 3, 1e-2, 0.6),     # n1 = 2 k + 2: one block, both mirror ends in every stencil
    (90, 30, 7, 16, 0.0, 1.0),     # rho1 = 0: H_rho1 = I, half-width 0; r = 16
    (130, 20, 10, 16, 0.15, 0.8),  # the widest stencil, half-width 12: 40 output rows per block
])
def test_x_update_stencil_and_separate_solve(n1, n2, n3, r, rho1, eta):
    """The X-update with H_rho1^{-1} applied as a stencil inside the A = W~ Y~^* launch and with
    the separate tridiagonal solve: each against the oracle, and the two within FP32 rounding."""
    d = make_inputs(n1, n2, n3, r, p=0.4, seed=n1 + r, sigma_od=1.5)
    a = gpu_run(d, r, 6, rho1=rho1, eta=eta)
    b = gpu_run(d, r, 6, rho1=rho1, eta=eta, xsolve=1)
    ka, kb = a["ctx"].tuning()[4], b["ctx"].tuning()[4]
    print(f"{n1}x{n2}x{n3} r{r} rho1 {rho1}: half-width {ka} / {kb}, W rel {rel(a['W'], b['W']):.2e}", flush=True)
    assert ka >= 0 and kb == -1
    st, info = oracle_run(d, r, 6, rho1=rho1, eta=eta, history=True)
    _compare(a, st, info, label=f"stencil k={ka}")
    _compare(b, st, info, label="separate solve")
    assert rel(a["W"], b["W"]) < 2e-6


@pytest.mark.parametrize("n1,rho1,expect", [(40, 0.16, -1), (40, 0.15, 12), (11, 0.01, -1), (12, 0.01, 5)])
def test_x_update_form_follows_the_rule(n1, rho1, expect):
    """The stencil is used up to half-width 12 and for n1 >= 2 k + 2 (else the tridiagonal
    solve), and either way the run matches the oracle."""
    d = make_inputs(n1, 24, 8, 4, p=0.4, seed=n1, sigma_od=1.5)
    g = gpu_run(d, 4, 5, rho1=rho1)
    assert g["ctx"].tuning()[4] == expect
    st, info = oracle_run(d, 4, 5, rho1=rho1, history=True)
    _compare(g, st, info, label=f"n1 {n1} rho1 {rho1} half-width {expect}")


def test_exact_recovery_in_one_sweep():
    """Fully observed exact tubal rank r with rho1 = 0: Z = G after one iteration."""
    rng = np.random.default_rng(4)
    xg, yg = rng.normal(size=(40, 4, 12)), rng.normal(size=(4, 30, 12))
    gt = oracle.tprod(xg, yg).astype(np.float32)
    d = {"G": gt, "omega": np.ones(gt.shape, np.uint8), "X0": np.zeros((40, 4, 12), np.float32),
         "Y0": rng.normal(size=(4, 30, 12)).astype(np.float32)}
    g = gpu_run(d, 4, 1, rho1=0.0)
    assert rel(g["Z"], gt) < 1e-5


def test_objective_never_increases():
    w, d = make_workload("od36x48x7_r3")
    g = gpu_run(d, w.r, 30, history=True, mu=0.05, rho1=0.2, rho2=0.3)
    f = np.array(g["f0"])
    assert np.all(f[1:] <= f[:-1] * (1 + 1e-6)), f


def test_eigen_pseudo_inverse_path_and_rank_deficiency():
    """Forcing the eigen-decomposition route changes nothing beyond rounding; a Y0 with a
    zero row makes Y~ Y~^* singular in every frequency, so the pseudo-inverse drops it."""
    d = make_inputs(30, 24, 7, 4, p=0.5, seed=9)
    a = gpu_run(d, 4, 6)
    b = gpu_run(d, 4, 6, pinv_mode=1)
    assert rel(b["W"], a["W"]) < 1e-6
    d2 = dict(d)
    y0 = d["Y0"].copy()
    y0[2] = 0.0
    d2["Y0"] = y0
    g = gpu_run(d2, 4, 6)
    st, info = oracle_run(d2, 4, 6, history=True)
    _compare(g, st, info, label="rank-deficient start")


def test_workload_144x288x28_p40_full_run():
    """144 x 288 x 28, r = 8, 40 % sampled: the whole 200-iteration run against the oracle."""
    w, d = make_workload("od144x288x28_r8_p40")
    g = gpu_run(d, w.r, w.iters)
    st, info = oracle_run(d, w.r, w.iters)
    info["f0"] = [oracle.objective(info["problem"], st)]
    _compare(g, st, info, label=f"od144x288x28_r8_p40 ({w.iters} it)")


@pytest.mark.parametrize("p", [10, 20, 60, 80])
def test_workload_144x288x28_other_rates(p):
    """The other sampling rates of the same workload, 20 iterations each."""
    w, d = make_workload(f"od144x288x28_r8_p{p}")
    g = gpu_run(d, w.r, 20)
    st, info = oracle_run(d, w.r, 20)
    info["f0"] = [oracle.objective(info["problem"], st)]
    _compare(g, st, info, label=f"od144x288x28_r8_p{p} (20 it)")


def test_precision_workload_full_size_parity():
    """529 x 96 x 112, r = 16 in the configuration the bench times (graph replays): 20
    iterations against the oracle."""
    w, d = make_workload("od529x96x112_r16")
    g = gpu_run(d, w.r, 20)
    st, info = oracle_run(d, w.r, 20)
    info["f0"] = [oracle.objective(info["problem"], st)]
    _compare(g, st, info, label="od529x96x112_r16 (20 it)")


def test_factors_in_spatial_domain():
    d = make_inputs(16, 12, 6, 3, p=0.5, seed=5)
    g = gpu_run(d, 3, 3, want=("W", "Z", "X", "Y"))
    st, _ = oracle_run(d, 3, 3)
    assert rel(g["X"], oracle.idft3(st.xt).real) < TOL
    assert rel(g["Y"], oracle.idft3(st.yt).real) < TOL


def test_stationarity_and_termination_measures():
    d = make_inputs(18, 14, 6, 3, p=0.6, seed=12)
    g = gpu_run(d, 3, 12, track=True)
    c = g["ctx"]
    s = c.stationarity()
    t = c.termination()
    st, info = oracle_run(d, 3, 11)
    prob = info["problem"]
    nxt = oracle.iterate(prob, st)
    so = oracle.stationarity(prob, nxt)
    assert abs(s[0] - so["factor"]) <= 1e-3 * so["factor"] + 1e-7, (s, so)
    assert s[1] < 1e-5 and s[2] == 0.0
    to = oracle.termination(st, nxt)
    assert abs(t[0] - to[0]) <= 1e-3 * to[0] + 1e-6 and abs(t[1] - to[1]) <= 1e-3 * to[1] + 1e-6
    assert abs(t[2] - to[2]) <= 1e-3 * to[2] + 1e-6


def test_checkpoint_resume_is_bitwise():
    import torch
    d = make_inputs(25, 20, 8, 3, p=0.4, seed=21)
    a = gpu_run(d, 3, 10)
    b = gpu_run(d, 3, 5)
    blob = b["ctx"].get_state()
    c = gpu_run(d, 3, 0)
    c["ctx"].set_state(blob)
    c["ctx"].step(5)
    wc = c["ctx"].result()["W"].cpu().numpy()
    assert np.array_equal(wc, a["W"].astype(np.float32))
    assert c["ctx"].iterations == 10
    del torch


def test_runs_are_deterministic():
    d = make_inputs(50, 40, 12, 4, p=0.4, seed=33)
    a = gpu_run(d, 4, 7)
    b = gpu_run(d, 4, 7)
    assert np.array_equal(a["W"], b["W"]) and a["f0"] == b["f0"]


def test_default_initialisation():
    """X0 = NULL (zeros) and Y0 = NULL (counter-based normals): a finite, decreasing run."""
    d = make_inputs(30, 20, 7, 3, p=0.5, seed=2)
    g = gpu_run(d, 3, 10, x0=False, y0=False, seed=123, history=True)
    f = np.array(g["f0"])
    assert np.all(np.isfinite(f)) and f[-1] < f[0]


def test_run_until_termination_stops_where_the_oracle_does():
    """Step 6 driving the loop: with check_every = 1 the run stops at the first iteration
    whose termination quantities all fall below eps, the same iteration as in FP64."""
    from tests.gpu_helpers import to_dev
    from paper_2005_09838_amd import Completion
    d = make_inputs(18, 14, 6, 3, p=0.6, seed=12)
    prob = oracle.Problem(d["G"], d["omega"], 3, 1e-2, 1e-2, 1e-2)
    st = oracle.initial_state(prob, d["X0"], d["Y0"])
    maxima = []
    for _ in range(40):
        nxt = oracle.iterate(prob, st)
        maxima.append(max(oracle.termination(st, nxt)))
        st = nxt
    # a stopping iteration with a clear margin (a few per cent) on both sides of eps
    n_stop = next(n for n in range(8, 40) if maxima[n] < 0.95 * maxima[n - 1])
    eps = (maxima[n_stop] * maxima[n_stop - 1]) ** 0.5
    assert all(m > eps for m in maxima[:n_stop])
    c = Completion(to_dev(d["G"]), to_dev(d["omega"]), 3, X0=to_dev(d["X0"]), Y0=to_dev(d["Y0"]), eps=eps)
    n, conv = c.run(200, check_every=1)
    assert conv and n == n_stop + 1, (n, n_stop + 1, eps)
    t = c.termination()
    assert t[3] == 1.0 and max(t[:3]) <= eps
    c2 = Completion(to_dev(d["G"]), to_dev(d["omega"]), 3, X0=to_dev(d["X0"]), Y0=to_dev(d["Y0"]), eps=eps)
    n2, conv2 = c2.run(n_stop, check_every=4)   # stops at the budget before the test holds
    assert not conv2 and n2 == n_stop


def test_two_row_groups_through_graph_replays():
    """n1 = 300 (two row groups of the G_X Gram) over 23 iterations: two graph replays of 10
    iterations and eager ones, against the oracle."""
    d = make_inputs(300, 14, 5, 3, p=0.4, seed=3005, weekly=True, sigma_od=1.0, noise=0.02)
    g = gpu_run(d, 3, 23)
    st, info = oracle_run(d, 3, 23, history=False)
    _compare(g, st, info, label="300x14x5 r3, 23 iterations")


@pytest.mark.parametrize("n1,n2,n3,r,p", [
    (20, 15, 17, 3, 0.4),     # odd tube length outside the generated transform lengths
    (12, 10, 144, 3, 0.5),    # 144: the OD count as the tube (slot x day x OD layout)
    (11, 11, 1008, 3, 0.5),   # 11 x 11 x 1008: the router-pair layout of the paper's Abilene tensor
    (8, 300, 128, 2, 0.4),    # a generated length whose slice is larger than the fused kernel's LDS
])
def test_three_launch_slice_path(n1, n2, n3, r, p):
    """Steps 3, 4 and 7 through the spatial buffers (direct tube transforms) against the
    oracle: W, Z, f0, and the stationarity measures (W-KKT maxima) of the same path."""
    d = make_inputs(n1, n2, n3, r, p=p, seed=n1 * n2 + n3, weekly=True, sigma_od=1.0, noise=0.02)
    g = gpu_run(d, r, 8)
    st, info = oracle_run(d, r, 8, history=True)
    _compare(g, st, info, label=f"{n1}x{n2}x{n3} r{r} (three-launch slice)")
    s = g["ctx"].stationarity()
    so = oracle.stationarity(info["problem"], st)
    assert abs(s[0] - so["factor"]) <= 1e-3 * so["factor"] + 1e-7, (s, so)
    assert s[1] < 1e-5 and s[2] == 0.0


def test_three_launch_slice_path_mixed_precision():
    """BF16 W~ (stochastic rounding) on the three-launch path: deterministic and close to FP32."""
    d = make_inputs(12, 10, 144, 3, p=0.5, seed=1234, weekly=True, sigma_od=1.0, noise=0.02)
    a = gpu_run(d, 3, 30)
    b = gpu_run(d, 3, 30, precision="mixed")
    c = gpu_run(d, 3, 30, precision="mixed")
    assert np.array_equal(b["W"], c["W"])
    assert rel(b["W"], a["W"]) < 1e-2


@pytest.mark.parametrize("layout,iters", [("slot_day_od", 20), ("origin_destination_time", 6)])
def test_paper_layouts_of_the_144x288x28_workload(layout, iters):
    """The 40 %-sampled 144 x 288 x 28 data in the paper's slot x day x OD layout (288 x 28 x
    144, section 3.1) and in the router-pair layout (12 x 12 x 8064, section 5) against the
    oracle on the same layout."""
    from synth import relayout
    w, d = make_workload("od144x288x28_r8_p40")
    e = relayout(d, layout, w.r, w.seed)
    g = gpu_run(e, w.r, iters)
    st, info = oracle_run(e, w.r, iters)
    info["f0"] = [oracle.objective(info["problem"], st)]
    _compare(g, st, info, label=f"{layout} {tuple(e['M'].shape)} ({iters} it)")


@pytest.mark.parametrize("tol,every", [(0.05, 5), (0.2, 3)])
def test_rank_adjustment_against_the_oracle(tol, every):
    """Step 5 every `every` iterations with threshold tol (singular values of Z~_k against tol
    times the largest): the rank vector equals the oracle's (FP64 SVD of every frequency's
    n1 x n2 product) and W, Z stay on the oracle's trajectory over 12 iterations.  The
    thresholds sit at least 2 % away from every singular value of this run."""
    n1, n2, n3, r = 40, 36, 12, 5
    d = make_inputs(n1, n2, n3, r, p=0.5, seed=55, weekly=True)
    g = gpu_run(d, r, 12, rank_tol=tol, rank_every=every)
    st, info = oracle.complete(d["G"], d["omega"], r, d["X0"], d["Y0"], 12, rank_tol=tol, rank_every=every)
    ranks = g["ctx"].rank_vector()
    print(f"tol {tol} every {every}: ranks {ranks} (oracle {list(info['ranks'][:n3 // 2 + 1])})", flush=True)
    assert ranks == [int(v) for v in info["ranks"][:n3 // 2 + 1]]
    assert min(ranks) < r
    _compare(g, st, None, label=f"rank adjustment tol {tol} every {every}")

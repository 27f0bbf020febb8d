"""C ABI behaviour on the GPU: error statuses, NaN detection, workspace checks, mixed precision."""
import ctypes

import numpy as np
import pytest

from tests.gpu_helpers import gpu_run, make_inputs, make_workload, oracle, oracle_run, rel, to_dev

pytestmark = pytest.mark.gpu


def _params(n1, n2, n3, r, **kw):
    from paper_2005_09838_amd import make_params
    return make_params(n1, n2, n3, r, **kw)


def test_nonfinite_observation_is_reported():
    import torch
    from paper_2005_09838_amd import binding as B
    d = make_inputs(10, 8, 4, 2, p=0.5, seed=1)
    g = d["G"].copy()
    idx = np.argwhere(d["omega"] == 1)[0]
    g[tuple(idx)] = np.nan
    p = _params(10, 8, 4, 2)
    n = B.tctf_workspace_bytes(p)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, to_dev(g), to_dev(d["omega"]), None, to_dev(d["Y0"]), 0, ws, n, None)
    assert e.value.status == B.TCTF_E_NONFINITE
    # a NaN off Omega is ignored
    g2 = d["G"].copy()
    idx = np.argwhere(d["omega"] == 0)[0]
    g2[tuple(idx)] = np.nan
    ctx = B.tctf_create(p, to_dev(g2), to_dev(d["omega"]), None, to_dev(d["Y0"]), 0, ws, n, None)
    B.tctf_step(ctx, 2)
    assert np.isfinite(B.tctf_objective(ctx))
    B.tctf_destroy(ctx)


def test_workspace_and_argument_errors():
    import torch
    from paper_2005_09838_amd import binding as B
    d = make_inputs(10, 8, 4, 2, p=0.5, seed=1)
    p = _params(10, 8, 4, 2)
    n = B.tctf_workspace_bytes(p)
    ws = torch.empty(n + 512, dtype=torch.uint8, device="cuda:0")
    G, om = to_dev(d["G"]), to_dev(d["omega"])
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, G, om, None, None, 0, ws, n - 1, None)
    assert e.value.status == B.TCTF_E_WORKSPACE
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, G, om, None, None, 0, ws.data_ptr() + 4, n, None)
    assert e.value.status == B.TCTF_E_WORKSPACE
    with pytest.raises(B.TctfError) as e:
        B.tctf_create(p, None, om, None, None, 0, ws, n, None)
    assert e.value.status == B.TCTF_E_ARG
    ctx = B.tctf_create(p, G, om, None, None, 0, ws, n, None)
    with pytest.raises(B.TctfError) as e:
        B.tctf_termination(ctx)
    assert e.value.status == B.TCTF_E_STATE
    with pytest.raises(B.TctfError) as e:
        B.tctf_step(ctx, -1)
    assert e.value.status == B.TCTF_E_ARG
    small = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(B.TctfError) as e:
        B.tctf_set_state(ctx, small, 16)
    assert e.value.status == B.TCTF_E_STATE
    B.tctf_destroy(ctx)


def test_complete_one_call():
    import torch
    from paper_2005_09838_amd import binding as B
    w, d = make_workload("od36x48x7_r3")
    p = _params(36, 48, 7, 3)
    n = B.tctf_workspace_bytes(p)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    W = torch.empty((36, 48, 7), dtype=torch.float32, device="cuda:0")
    f0 = B.tctf_complete(p, to_dev(d["G"]), to_dev(d["omega"]), to_dev(d["X0"]), to_dev(d["Y0"]), 0, 10, ws, n,
                         None, W)
    st, info = oracle_run(d, 3, 10, history=True)
    assert rel(W.cpu().numpy(), st.w) < 1e-5
    assert abs(f0 - info["f0"][-1]) / info["f0"][-1] < 1e-5


@pytest.mark.parametrize("name", ["od529x96x112_r16", "od36x48x7_r3"])
def test_mixed_precision_reaches_the_fp32_error(name):
    """W~ stored in BF16 (stochastic rounding), products accumulated in FP32: after the
    workload's whole run the completion error (RSE against the full synthetic tensor) is
    within the relative gap 5e-3 of the FP32 run's.  Runs are deterministic."""
    w, d = make_workload(name)
    iters = 200 if name.startswith("od529") else w.iters
    a = gpu_run(d, w.r, iters)
    b = gpu_run(d, w.r, iters, precision="mixed")
    b2 = gpu_run(d, w.r, iters, precision="mixed")
    rse_a = oracle.rse(a["W"], d["M"])
    rse_b = oracle.rse(b["W"], d["M"])
    print(f"{name} {iters} it: RSE fp32 {rse_a:.6f} mixed {rse_b:.6f} gap {rse_b / rse_a - 1:+.2e}", flush=True)
    assert np.all(np.isfinite(b["W"]))
    assert abs(rse_b / rse_a - 1.0) <= 5e-3
    assert np.array_equal(b["W"], b2["W"])


@pytest.mark.parametrize("name", ["od529x96x112_r16", "od144x288x28_r8_p40"])
def test_mixed_precision_first_iterations_near_the_oracle(name):
    """Mixed precision (BF16 W~ and Z~, Z~ = X~Y~ on the BF16 matrix cores from stochastically
    rounded factors) two iterations from the oracle's start: W and Z within 1e-2 (relative
    Frobenius) of the FP64 oracle.  BF16 keeps 8 significant bits, so a wrong operand
    layout, sign or rounding key in the BF16 tiles would be off by far more."""
    w, d = make_workload(name)
    g = gpu_run(d, w.r, 2, precision="mixed")
    st, _ = oracle_run(d, w.r, 2)
    ew, ez = rel(g["W"], st.w), rel(g["Z"], oracle.z_of(st))
    print(f"{name} mixed, 2 it: W {ew:.2e} Z {ez:.2e}", flush=True)
    assert ew < 1e-2 and ez < 1e-2


def test_mixed_precision_stays_near_fp32_over_long_runs():
    """Mixed precision over 4000 iterations at 529 x 96 x 112: BF16 rounding noise that is new
    every iteration must not walk the iterate along the completion's weakly determined
    directions (BF16-rounded Z~ did, by a few percent of RSE).  Every 400 iterations the RSE
    is within the relative gap 5e-3 of the FP32 run's."""
    from paper_2005_09838_amd import Completion
    w, d = make_workload("od529x96x112_r16")
    mk = lambda prec: Completion(to_dev(d["G"]), to_dev(d["omega"]), w.r, X0=to_dev(d["X0"]), Y0=to_dev(d["Y0"]),
                                 precision=prec)
    a, b = mk("fp32"), mk("mixed")
    gaps = []
    for _ in range(10):
        a.step(400)
        b.step(400)
        ra = oracle.rse(a.result()["W"].cpu().numpy(), d["M"])
        rb = oracle.rse(b.result()["W"].cpu().numpy(), d["M"])
        gaps.append(rb / ra - 1.0)
    print("mixed - fp32 RSE gaps every 400 it:", " ".join(f"{g:+.1e}" for g in gaps), flush=True)
    assert max(abs(g) for g in gaps) <= 5e-3
    a.close()
    b.close()


def test_stage_profile_records_each_launch():
    """tctf_profile brackets exactly the launches of the chosen stages; results are unchanged."""
    d = make_inputs(40, 30, 12, 4, p=0.4, seed=8)
    a = gpu_run(d, 4, 6)
    b = gpu_run(d, 4, 2)
    c = b["ctx"]
    c.profile(["slice", "bgemm"])
    c.step(4)
    rec = c.profile_read()
    assert rec["slice"][1] == 4 and rec["bgemm"][1] == 4 and rec["agemm"][1] == 0
    assert rec["slice"][0] > 0 and rec["bgemm"][0] > 0
    c.profile([])
    assert np.array_equal(c.result()["W"].cpu().numpy(), a["W"].astype(np.float32))


@pytest.mark.parametrize("xsolve", [0, 1])
def test_stage_timing_leaves_the_iterate_unchanged(xsolve):
    """tctf_time_stage recomputes stages 0-6 from the current state without advancing it:
    the iterations after it give the same bits as a context that was never timed (with the
    X-update's H_rho1^{-1} stencil, stage 2 writes the new X~ to a scratch buffer)."""
    d = make_inputs(70, 40, 12, 6, p=0.4, seed=21)
    a = gpu_run(d, 6, 9, xsolve=xsolve)
    b = gpu_run(d, 6, 4, xsolve=xsolve)
    c = b["ctx"]
    assert (c.tuning()[4] >= 0) == (xsolve == 0)
    for st in range(7):
        assert c.time_stage(st, reps=3) > 0.0
    c.step(5)
    assert np.array_equal(c.result()["W"].cpu().numpy(), a["W"].astype(np.float32))
    assert c.objective() == a["ctx"].objective()


def test_mixed_precision_stencil_and_separate_solve():
    """Mixed precision with the H_rho1^{-1} stencil in the X-update and with the separate
    tridiagonal solve: the two stay within the mixed mode's own noise of each other."""
    w, d = make_workload("od144x288x28_r8_p40")
    a = gpu_run(d, w.r, 20, precision="mixed")
    b = gpu_run(d, w.r, 20, precision="mixed", xsolve=1)
    assert a["ctx"].tuning()[4] >= 0 and b["ctx"].tuning()[4] == -1
    e = rel(a["W"], b["W"])
    print(f"mixed, stencil vs separate solve after 20 iterations: W rel {e:.2e}", flush=True)
    assert e < 1e-2


def test_graph_replays_match_eager_launches():
    """Blocks of iterations replayed from the captured graph give the same bits as eager
    launches, across several replays separated by eager work and synchronisations."""
    d = make_inputs(45, 37, 14, 5, p=0.35, seed=17)
    g = gpu_run(d, 5, 0)
    e = gpu_run(d, 5, 0)
    cg, ce = g["ctx"], e["ctx"]
    ce.profile(["slice"])   # recording stages forces eager launches
    for k in (23, 11, 30):
        cg.step(k)          # graph replays + eager remainder
        ce.step(k)
        wg = cg.result()["W"].cpu().numpy()
        we = ce.result()["W"].cpu().numpy()
        assert np.array_equal(wg, we), k
        assert cg.objective() == ce.objective()
    ce.profile([])


def test_batch_members_match_single_runs():
    """Uneven completions run as one batch give, bit for bit, what each gives alone."""
    import torch
    from paper_2005_09838_amd import Batch
    shapes = [(36, 48, 7, 3, 0.3), (20, 30, 12, 4, 0.5), (64, 24, 28, 6, 0.4), (9, 40, 5, 2, 0.6),
              (50, 17, 16, 5, 0.35), (33, 33, 9, 3, 0.45), (12, 12, 4, 1, 0.5)]
    probs, data = [], []
    for k, (n1, n2, n3, r, p) in enumerate(shapes):
        d = make_inputs(n1, n2, n3, r, p=p, seed=40 + k, weekly=True)
        data.append((d, r))
        probs.append({"G": to_dev(d["G"]), "omega": to_dev(d["omega"]), "r": r, "X0": to_dev(d["X0"]),
                      "Y0": to_dev(d["Y0"]), "mu": 0.02 * (k + 1), "rho1": 0.01, "rho2": 0.03})
    b = Batch(probs)
    assert len(b) == len(shapes)
    b.step(23)
    for k, (d, r) in enumerate(data):
        a = gpu_run(d, r, 23, mu=0.02 * (k + 1), rho1=0.01, rho2=0.03)
        wb = b[k].result()["W"].cpu().numpy()
        assert np.array_equal(wb, a["W"].astype(np.float32)), k
        assert b[k].objective() == a["f0"][-1], k
        assert b[k].iterations == 23
    b.close()
    del torch


def test_batch_member_against_oracle():
    from paper_2005_09838_amd import Batch
    d = make_inputs(30, 26, 10, 3, p=0.4, seed=77)
    d2 = make_inputs(18, 40, 6, 2, p=0.5, seed=78)
    b = Batch([{"G": to_dev(d["G"]), "omega": to_dev(d["omega"]), "r": 3, "X0": to_dev(d["X0"]), "Y0": to_dev(d["Y0"])},
               {"G": to_dev(d2["G"]), "omega": to_dev(d2["omega"]), "r": 2, "X0": to_dev(d2["X0"]),
                "Y0": to_dev(d2["Y0"])}])
    b.step(12)
    st, info = oracle_run(d, 3, 12)
    assert rel(b[0].result()["W"].cpu().numpy(), st.w) < 1e-5
    st2, _ = oracle_run(d2, 2, 12)
    assert rel(b[1].result()["W"].cpu().numpy(), st2.w) < 1e-5
    b.close()


@pytest.mark.parametrize("n1,n2,n3,r", [(36, 48, 7, 3), (40, 65, 28, 6), (30, 300, 28, 4), (20, 15, 17, 3)])
def test_autotuned_execution_shape(n1, n2, n3, r):
    """tctf_params.autotune: the chosen slice path is one the sizes allow, the result stays on
    the oracle's trajectory, and a second context of the same shape takes the cached choice
    and gives the same bits."""
    from paper_2005_09838_amd import Completion
    d = make_inputs(n1, n2, n3, r, p=0.4, seed=n1 + n2, weekly=True)
    mk = lambda: Completion(to_dev(d["G"]), to_dev(d["omega"]), r, X0=to_dev(d["X0"]), Y0=to_dev(d["Y0"]),
                            autotune=True)
    a = mk()
    ta = a.tuning()
    assert ta[0] in (1, 2, 3) and ta[1] in (16, 32) and ta[2] >= 1
    a.step(8)
    wa = a.result()["W"].cpu().numpy()
    b = mk()
    tb = b.tuning()
    assert tb[:3] == ta[:3] and tb[3] == 1
    b.step(8)
    assert np.array_equal(b.result()["W"].cpu().numpy(), wa)
    st, _ = oracle_run(d, r, 8)
    print(f"{n1}x{n2}x{n3} r{r}: tuning {ta} rel {rel(wa, st.w):.2e}", flush=True)
    assert rel(wa, st.w) < 1e-5
    a.close()
    b.close()


def test_batch_of_autotuned_members_matches_single_runs():
    """Members with autotune: the batch gives, bit for bit, what autotuned single contexts give."""
    from paper_2005_09838_amd import Batch, Completion
    shapes = [(36, 48, 7, 3, 0.3), (20, 30, 12, 4, 0.5), (64, 24, 28, 6, 0.4), (30, 300, 28, 4, 0.4)]
    probs, data = [], []
    for k, (n1, n2, n3, r, p) in enumerate(shapes):
        d = make_inputs(n1, n2, n3, r, p=p, seed=90 + k, weekly=True)
        data.append((d, r))
        probs.append({"G": to_dev(d["G"]), "omega": to_dev(d["omega"]), "r": r, "X0": to_dev(d["X0"]),
                      "Y0": to_dev(d["Y0"]), "autotune": True})
    b = Batch(probs)
    b.step(13)
    for k, (d, r) in enumerate(data):
        c = Completion(to_dev(d["G"]), to_dev(d["omega"]), r, X0=to_dev(d["X0"]), Y0=to_dev(d["Y0"]), autotune=True)
        c.step(13)
        assert c.tuning()[:3] == b[k].tuning()[:3]
        assert np.array_equal(b[k].result()["W"].cpu().numpy(), c.result()["W"].cpu().numpy()), k
        c.close()
    b.close()

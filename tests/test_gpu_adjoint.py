"""Reverse-mode derivatives on the GPU against the FP64 oracle adjoint (needs an MI355X).

The GPU forward runs in FP32 and its reverse pass in FP64; the oracle runs both in FP64 on
the same inputs.  Tolerances: one iteration's adjoints within 1e-5 (largest entry error
relative to the largest entry; weights' adjoints relative); the unrolled hypergradients
of the held-out error through 20 iterations within 2e-5 relative and the gradient with
respect to Y0 within 3e-4 (largest entry error relative to the largest entry: the FP32
forward's rounding, carried through 20 iterations, dominates), and the oracle's own
hypergradients within 1e-5 of central differences (h = 1e-4, FP64) at the same size."""
import numpy as np
import pytest

from oracle import adjoint as AD
from tests.gpu_helpers import make_workload, oracle, to_dev

pytestmark = pytest.mark.gpu


def _maxrel(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300))


def _stored(full, order):
    """Full-spectrum (.., .., m3) complex array -> stored bins in the library's layout."""
    nb = full.shape[2] // 2 + 1
    return np.ascontiguousarray(np.transpose(full[:, :, :nb], order))


def _to_complex_dev(a):
    import torch
    v = np.stack([a.real, a.imag], axis=-1).astype(np.float64)
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0").reshape(-1)


def _from_complex_dev(t, shape):
    v = t.cpu().numpy().reshape(*shape, 2)
    return v[..., 0] + 1j * v[..., 1]


@pytest.mark.parametrize("eta", [1.0, 0.8])
def test_one_iteration_adjoint_at_the_differentiation_shape(eta):
    """144 x 288 x 28, r = 8, 40 % sampled: one iteration's reverse pass from random output
    adjoints, GPU against the oracle (X~, Y~ and W adjoints, and those of mu, rho1, rho2)."""
    import torch
    from paper_2005_09838_amd import Completion, binding as B
    w, d = make_workload("od144x288x28_r8_holdout")
    n1, n2, n3, r = w.n1, w.n2, w.n3, w.r
    nb = n3 // 2 + 1
    rng = np.random.default_rng(31)
    x0 = rng.normal(size=(n1, r, n3)).astype(np.float32)
    c = Completion(to_dev(d["G"]), to_dev(d["omega"]), r, mu=w.mu, rho1=w.rho1, rho2=w.rho2, eta=eta,
                   X0=to_dev(x0), Y0=to_dev(d["Y0"]))
    s0 = c.get_state()
    c.step(1)
    s1 = c.get_state()
    xb = oracle.dft3(rng.normal(size=(n1, r, n3)))
    yb = oracle.dft3(rng.normal(size=(r, n2, n3)))
    wb = rng.normal(size=(n1, n2, n3))
    xt_bar = _to_complex_dev(_stored(xb, (2, 1, 0)))      # (n1, r, m3) -> [nb][r][n1]
    yt_bar = _to_complex_dev(_stored(yb, (2, 0, 1)))      # (r, n2, m3) -> [nb][r][n2]
    w_bar = torch.from_numpy(wb.copy()).to("cuda:0")
    th = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    ws, nbytes = c.adjoint_workspace()
    B.tctf_adjoint_step(c.ctx, s0, s1, xt_bar, yt_bar, w_bar, th, ws, nbytes)
    gx = _from_complex_dev(xt_bar, (nb, r, n1))
    gy = _from_complex_dev(yt_bar, (nb, r, n2))
    gw = w_bar.cpu().numpy()
    prob = oracle.Problem(d["G"], d["omega"], r, w.mu, w.rho1, w.rho2, eta)
    st0 = oracle.initial_state(prob, x0, d["Y0"])
    st1 = oracle.iterate(prob, st0)
    tb = AD.ThetaBar()
    ox, oy, ow = AD.iterate_adjoint(prob, st0, st1, xb, yb, wb, tb)
    ex = _maxrel(gx, _stored(ox, (2, 1, 0)))
    ey = _maxrel(gy, _stored(oy, (2, 0, 1)))
    ew = _maxrel(gw, ow)
    ot = tb.as_array()
    et = np.abs(th.cpu().numpy() - ot) / np.abs(ot)
    print(f"eta {eta}: X~ {ex:.2e} Y~ {ey:.2e} W {ew:.2e} theta {et} ({th.cpu().numpy()} vs {ot})", flush=True)
    assert ex <= 1e-5 and ey <= 1e-5 and ew <= 1e-5, (ex, ey, ew)
    assert np.all(et <= 1e-5), et
    c.close()


def test_unrolled_hypergradients_of_the_heldout_error():
    """144 x 288 x 28, r = 8, 40 % sampled + 10 % held out: d(held-out RSE after 20
    iterations) / d(mu, rho1, rho2) and d / d Y0 through the torch.autograd.Function
    (checkpoints every 5 iterations), against the FP64 oracle adjoint; the oracle against
    central differences of its forward run."""
    import torch
    from paper_2005_09838_amd.autodiff import unrolled_completion
    w, d = make_workload("od144x288x28_r8_holdout")
    iters = w.iters
    dev = "cuda:0"
    theta = torch.tensor([w.mu, w.rho1, w.rho2], dtype=torch.float64, requires_grad=True)
    X0 = torch.from_numpy(d["X0"]).to(dev).requires_grad_(True)
    Y0 = torch.from_numpy(d["Y0"]).to(dev).requires_grad_(True)
    M = torch.from_numpy(d["M"]).to(dev).double()
    H = torch.from_numpy(d["holdout"]).to(dev).bool()
    W = unrolled_completion(theta, X0, Y0, to_dev(d["G"]), to_dev(d["omega"]), w.r, iters, checkpoint_every=5)
    e = torch.where(H, W - M, torch.zeros_like(M))
    loss = torch.linalg.norm(e) / torch.linalg.norm(M[H])
    loss.backward()
    prob = oracle.Problem(d["G"], d["omega"], w.r, w.mu, w.rho1, w.rho2)
    ol, oth, ox0, oy0, _ = AD.unrolled_gradients(prob, d["X0"].astype(float), d["Y0"].astype(float), iters,
                                                 d["M"].astype(float), d["holdout"])
    gth = theta.grad.numpy()
    gy0 = Y0.grad.cpu().numpy()
    el = abs(loss.item() - ol) / ol
    eth = np.abs(gth - oth) / np.abs(oth)
    ey0 = _maxrel(gy0, oy0)
    print(f"loss {loss.item():.6f} vs {ol:.6f} ({el:.1e}); theta grad {gth} vs {oth} ({eth}); Y0 grad {ey0:.2e}",
          flush=True)
    assert el <= 1e-5
    assert np.all(eth <= 2e-5), eth
    assert ey0 <= 3e-4
    assert np.abs(X0.grad.cpu().numpy()).max() == 0.0   # eta = 1: the first X-step does not read X0
    # the oracle's hypergradients against central differences (h = 1e-4) of its forward run
    h = 1e-4
    for k in range(3):
        tp = [w.mu, w.rho1, w.rho2]
        tm = list(tp)
        tp[k] += h
        tm[k] -= h
        sp, _ = oracle.complete(d["G"], d["omega"], w.r, d["X0"], d["Y0"], iters, *tp)
        sm, _ = oracle.complete(d["G"], d["omega"], w.r, d["X0"], d["Y0"], iters, *tm)
        fd = (AD.heldout_rse(sp.w, d["M"], d["holdout"]) - AD.heldout_rse(sm.w, d["M"], d["holdout"])) / (2 * h)
        assert abs(fd - oth[k]) <= 1e-5 * abs(fd) + 1e-9, (k, fd, oth[k])


def test_objective_gradient_with_respect_to_the_factors():
    """d f0 / d X and d f0 / d Y at the iterate after 3 iterations, GPU against the oracle."""
    from paper_2005_09838_amd import Completion
    w, d = make_workload("od36x48x7_r3")
    c = Completion(to_dev(d["G"]), to_dev(d["omega"]), w.r, X0=to_dev(d["X0"]), Y0=to_dev(d["Y0"]))
    c.step(3)
    gx, gy = c.objective_gradient()
    st, info = oracle.complete(d["G"], d["omega"], w.r, d["X0"], d["Y0"], 3)
    ox, oy = AD.objective_factor_gradients(info["problem"], st)
    ex, ey = _maxrel(gx.cpu().numpy(), ox), _maxrel(gy.cpu().numpy(), oy)
    print(f"d f0 / dX {ex:.2e}, d f0 / dY {ey:.2e}", flush=True)
    assert ex <= 1e-4 and ey <= 1e-4
    c.close()


def test_adjoint_reports_a_rank_deficient_gram():
    """Y0 with a zero row: G_Y is singular in every frequency, the adjoint refuses."""
    from paper_2005_09838_amd import Completion, binding as B
    import torch
    w, d = make_workload("od36x48x7_r3")
    y0 = d["Y0"].copy()
    y0[1] = 0.0
    c = Completion(to_dev(d["G"]), to_dev(d["omega"]), w.r, X0=to_dev(d["X0"]), Y0=to_dev(y0))
    s0 = c.get_state()
    c.step(1)
    s1 = c.get_state()
    nb = 7 // 2 + 1
    xt = torch.zeros(nb * 3 * 36 * 2, dtype=torch.float64, device="cuda:0")
    yt = torch.zeros(nb * 3 * 48 * 2, dtype=torch.float64, device="cuda:0")
    wb = torch.ones((36, 48, 7), dtype=torch.float64, device="cuda:0")
    th = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    ws, nbytes = c.adjoint_workspace()
    with pytest.raises(B.TctfError) as e:
        B.tctf_adjoint_step(c.ctx, s0, s1, xt, yt, wb, th, ws, nbytes)
    assert e.value.status == B.TCTF_E_STATE
    with pytest.raises(B.TctfError) as e:   # blobs out of order
        B.tctf_adjoint_step(c.ctx, s1, s0, xt, yt, wb, th, ws, nbytes)
    assert e.value.status == B.TCTF_E_STATE
    c.close()

"""Pins of the oracle's hand-written reverse-mode derivatives (CPU only).

Each is fixed by something other than the adjoint code: central finite differences of the
forward oracle (itself pinned by the other test files), and a closed form of the W-step at
rho2 = 0."""
import numpy as np
import pytest

import oracle as O
from oracle import adjoint as AD
from synth import make_inputs


def _problem(seed=0, shape=(6, 7, 5), r=2, p=0.5, mu=0.05, rho1=0.3, rho2=0.2, eta=1.0, holdout=False):
    d = make_inputs(*shape, r, p=p, seed=seed, sigma_od=0.5, noise=0.02, weekly=True, holdout=holdout)
    return d, O.Problem(d["G"], d["omega"], r, mu, rho1, rho2, eta)


def _phi(prob, x, y, w, xb, yb, wb):
    """<adjoint of the outputs, outputs> of one iteration from the real spatial state (x, y, w)."""
    st = O.State(O.dft3(x), O.dft3(y), w, O.dft3(w))
    nxt = O.iterate(prob, st)
    return (float(np.sum(np.real(np.conj(xb) * nxt.xt))) + float(np.sum(np.real(np.conj(yb) * nxt.yt)))
            + float(np.sum(wb * nxt.w)))


@pytest.mark.parametrize("eta,seed", [(1.0, 1), (0.7, 2), (1.3, 3)])
def test_one_iteration_adjoint_matches_finite_differences(eta, seed):
    """The reverse pass of one iteration against directional central differences of the
    forward iteration, for directions in the real factors X, Y, in W and in mu, rho1, rho2."""
    d, prob = _problem(seed=seed, eta=eta)
    rng = np.random.default_rng(100 + seed)
    m1, m2, m3 = prob.shape
    r = prob.r
    x = rng.normal(size=(m1, r, m3))
    y = rng.normal(size=(r, m2, m3))
    w = np.where(prob.omega, prob.g, rng.normal(size=prob.shape))
    st = O.State(O.dft3(x), O.dft3(y), w, O.dft3(w))
    nxt = O.iterate(prob, st)
    # output adjoints of conjugate-symmetric form (they come from real spatial arrays)
    xb = O.dft3(rng.normal(size=(m1, r, m3)))
    yb = O.dft3(rng.normal(size=(r, m2, m3)))
    wb = rng.normal(size=prob.shape)
    tb = AD.ThetaBar()
    xt_bar, yt_bar, w_bar = AD.iterate_adjoint(prob, st, nxt, xb, yb, wb, tb)
    # adjoints of the real spatial inputs X, Y (X~ = dft3(X))
    x_bar = np.real(np.fft.fft(xt_bar, axis=2))
    y_bar = np.real(np.fft.fft(yt_bar, axis=2))
    h = 1e-5
    for _ in range(2):
        dx, dy, dw = rng.normal(size=x.shape), rng.normal(size=y.shape), rng.normal(size=w.shape)
        for name, fx, adj in (("X", lambda t: _phi(prob, x + t * dx, y, w, xb, yb, wb), np.sum(x_bar * dx)),
                              ("Y", lambda t: _phi(prob, x, y + t * dy, w, xb, yb, wb), np.sum(y_bar * dy)),
                              ("W", lambda t: _phi(prob, x, y, w + t * dw, xb, yb, wb), np.sum(w_bar * dw))):
            fd = (fx(h) - fx(-h)) / (2 * h)
            assert abs(fd - adj) <= 1e-6 * max(1.0, abs(fd)), (name, fd, adj)
    for k, name in enumerate(("mu", "rho1", "rho2")):
        def f(t, k=k):
            th = [prob.mu, prob.rho1, prob.rho2]
            th[k] += t
            p2 = O.Problem(prob.g, prob.omega, r, th[0], th[1], th[2], eta)
            return _phi(p2, x, y, w, xb, yb, wb)
        fd = (f(h) - f(-h)) / (2 * h)
        adj = tb.as_array()[k]
        assert abs(fd - adj) <= 1e-6 * max(1.0, abs(fd)), (name, fd, adj)


@pytest.mark.parametrize("eta", [1.0, 0.7])
def test_unrolled_hypergradients_match_central_differences(eta):
    """Held-out RSE after K = 4 iterations: gradients with respect to (mu, rho1, rho2) and to
    entries of X0, Y0 against central differences with h = 1e-4 in FP64."""
    d, prob = _problem(seed=5, shape=(8, 9, 6), r=2, p=0.45, eta=eta, holdout=True)
    rng = np.random.default_rng(7)
    x0 = rng.normal(size=(8, 2, 6)) if eta != 1.0 else d["X0"].astype(float)
    y0 = d["Y0"].astype(float)
    m, hold = d["M"].astype(float), d["holdout"]
    iters = 4
    loss, th_bar, x0_bar, y0_bar, _ = AD.unrolled_gradients(prob, x0, y0, iters, m, hold)
    h = 1e-4

    def run(th=(prob.mu, prob.rho1, prob.rho2), xx=x0, yy=y0):
        p2 = O.Problem(prob.g, prob.omega, prob.r, th[0], th[1], th[2], eta)
        st, _ = O.complete(p2.g, p2.omega, p2.r, xx, yy, iters, th[0], th[1], th[2], eta)
        return AD.heldout_rse(st.w, m, hold)

    assert abs(run() - loss) < 1e-14
    for k in range(3):
        tp = [prob.mu, prob.rho1, prob.rho2]
        tm = list(tp)
        tp[k] += h
        tm[k] -= h
        fd = (run(th=tp) - run(th=tm)) / (2 * h)
        assert abs(fd - th_bar[k]) <= 1e-6 * max(abs(fd), 1e-3), (k, fd, th_bar[k])
    for idx in [(0, 0, 0), (3, 1, 2), (7, 0, 5)]:
        e = np.zeros_like(x0)
        e[idx] = h
        fd = (run(xx=x0 + e) - run(xx=x0 - e)) / (2 * h)
        assert abs(fd - x0_bar[idx]) <= 1e-6 * max(abs(fd), 1e-3), ("X0", idx, fd, x0_bar[idx])
    for idx in [(0, 0, 0), (1, 4, 3), (1, 8, 5)]:
        e = np.zeros_like(y0)
        e[idx] = h
        fd = (run(yy=y0 + e) - run(yy=y0 - e)) / (2 * h)
        assert abs(fd - y0_bar[idx]) <= 1e-6 * max(abs(fd), 1e-3), ("Y0", idx, fd, y0_bar[idx])
    if eta == 1.0:   # at eta = 1 the first X-step does not read X0
        assert np.abs(x0_bar).max() == 0.0


def test_w_step_adjoint_without_rho2_is_a_scaling():
    """rho2 = 0: w_u = z_u / (1 + mu), so z_bar_u = w_bar_u / (1 + mu), z_bar_o = 0 and
    mu_bar = -sum_u w_bar_u w_u / (1 + mu)."""
    d, prob = _problem(seed=9, mu=0.3, rho2=0.0)
    rng = np.random.default_rng(1)
    z = rng.normal(size=prob.shape)
    w = O.w_step(z, prob.g, prob.omega, prob.mu, 0.0)
    wb = rng.normal(size=prob.shape)
    tb = AD.ThetaBar()
    zb = AD.w_step_adjoint(prob, w, wb, tb)
    un = ~prob.omega
    np.testing.assert_allclose(zb[un], wb[un] / 1.3, rtol=1e-13)
    assert np.all(zb[prob.omega] == 0.0)
    assert np.isclose(tb.mu, -np.sum(wb[un] * w[un]) / 1.3, rtol=1e-12)
    assert tb.rho2 != 0.0 or not un.any()


def test_objective_factor_gradients_match_central_differences():
    """d f0 / d X and d f0 / d Y entry by entry against central differences of the spatial
    objective eq. (TETP-optim)."""
    d, prob = _problem(seed=11, shape=(5, 4, 4), r=2)
    rng = np.random.default_rng(3)
    x, y, w = rng.normal(size=(5, 2, 4)), rng.normal(size=(2, 4, 4)), rng.normal(size=(5, 4, 4))
    st = O.State(O.dft3(x), O.dft3(y), w, O.dft3(w))
    gx, gy = AD.objective_factor_gradients(prob, st)
    f = lambda xx, yy: O.objective_spatial(O.tprod(xx, yy), w, prob.mu, prob.rho1, prob.rho2)
    h = 1e-5
    for arr, g, is_x in ((x, gx, True), (y, gy, False)):
        for idx in np.ndindex(*arr.shape):
            e = np.zeros_like(arr)
            e[idx] = h
            fd = ((f(x + e, y) - f(x - e, y)) if is_x else (f(x, y + e) - f(x, y - e))) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), (is_x, idx, fd, g[idx])

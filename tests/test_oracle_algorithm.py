"""Pins of the oracle's section-4 algorithm (CPU only)."""
import numpy as np
import pytest

import oracle as O
from oracle.algorithm import grad_x, grad_y, h_k
from synth import make_inputs

RNG = np.random.default_rng(2024)


def crandn(*shape, rng=RNG):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


# ----------------------------------------------------------------------------- pseudo-inverse

@pytest.mark.parametrize("r,rank", [(1, 1), (1, 0), (4, 4), (5, 2), (8, 7), (16, 16), (16, 3)])
def test_pinv_penrose_conditions(r, rank):
    """Moore-Penrose conditions (Penrose 1955, as cited for A^+) for Hermitian PSD Grams of any rank."""
    b = crandn(r, max(rank, 1)) if rank else np.zeros((r, 1), complex)
    a = b @ b.conj().T
    p = O.pinv_h(a)
    tol = 1e-9 * max(1.0, np.linalg.norm(a)) * max(1.0, np.linalg.norm(p))
    np.testing.assert_allclose(a @ p @ a, a, atol=tol)
    np.testing.assert_allclose(p @ a @ p, p, atol=tol)
    np.testing.assert_allclose((a @ p).conj().T, a @ p, atol=tol)
    np.testing.assert_allclose((p @ a).conj().T, p @ a, atol=tol)
    assert np.linalg.matrix_rank(p, tol=1e-8 * max(np.linalg.norm(p), 1e-300)) == rank


def test_pinv_of_zero_and_full_rank():
    assert np.array_equal(O.pinv_h(np.zeros((3, 3), complex)), np.zeros((3, 3), complex))
    b = crandn(4, 6)
    a = b @ b.conj().T
    np.testing.assert_allclose(O.pinv_h(a), np.linalg.inv(a), rtol=1e-10, atol=1e-12)


# ----------------------------------------------------------------------------- gradients

def _dir_deriv(f, x, e, h=1e-6):
    return (f(x + h * e) - f(x - h * e)) / (2 * h)


@pytest.mark.parametrize("m1,r,m2,rho1", [(5, 2, 4, 0.0), (6, 3, 5, 0.7), (1, 1, 3, 2.0), (4, 4, 4, 0.1)])
def test_gradients_match_finite_differences(m1, r, m2, rho1):
    """eq. (hkXYDer): the directional derivative of h_k along E equals Re<E, nabla>, for real
    and imaginary directions (pins signs, conjugation and transposition)."""
    x, y, w = crandn(m1, r), crandn(r, m2), crandn(m1, m2)
    h = O.toeplitz_diff(m1)
    hth = h.T @ h
    gx = grad_x(x, y, w, hth, rho1)
    gy = grad_y(x, y, w, hth, rho1)
    for _ in range(3):
        for e in (crandn(m1, r).real.astype(complex), 1j * crandn(m1, r).real):
            dd = _dir_deriv(lambda xx: h_k(xx, y, w, h, rho1), x, e)
            assert np.isclose(dd, np.real(np.sum(np.conj(gx) * e)), rtol=1e-6, atol=1e-6)
        for e in (crandn(r, m2).real.astype(complex), 1j * crandn(r, m2).real):
            dd = _dir_deriv(lambda yy: h_k(x, yy, w, h, rho1), y, e)
            assert np.isclose(dd, np.real(np.sum(np.conj(gy) * e)), rtol=1e-6, atol=1e-6)


# ----------------------------------------------------------------------------- block steps

def _kron_lstsq_x(y, w, h, rho1):
    """argmin_X ||X Y - W||^2 + rho1 ||H X Y||^2 by least squares on vec(X) (column-major)."""
    m1 = w.shape[0]
    a = np.vstack([np.kron(y.T, np.eye(m1)), np.sqrt(rho1) * np.kron(y.T, h)])
    b = np.concatenate([w.reshape(-1, order="F"), np.zeros(h.shape[0] * w.shape[1])])
    sol = np.linalg.lstsq(a, b, rcond=None)[0]
    return sol.reshape(m1, y.shape[0], order="F")


def _kron_lstsq_y(x, w, h, rho1):
    """argmin_Y ||X Y - W||^2 + rho1 ||H X Y||^2 by least squares on vec(Y)."""
    m2 = w.shape[1]
    a = np.vstack([np.kron(np.eye(m2), x), np.sqrt(rho1) * np.kron(np.eye(m2), h @ x)])
    b = np.concatenate([w.reshape(-1, order="F"), np.zeros(h.shape[0] * m2)])
    sol = np.linalg.lstsq(a, b, rcond=None)[0]
    return sol.reshape(x.shape[1], m2, order="F")


@pytest.mark.parametrize("m1,r,m2,rho1", [(6, 2, 5, 0.0), (7, 3, 6, 0.5), (5, 1, 4, 2.0), (8, 4, 9, 0.01)])
def test_unit_steps_are_exact_block_minimisers(m1, r, m2, rho1):
    """With eta = 1 and full-rank Grams, eq. (updataXYW1) lands on the minimiser of h_k over
    one block (checked by an independent Kronecker least-squares solve)."""
    g = np.zeros((m1, m2, 1))
    prob = O.Problem(g, np.ones_like(g), r, mu=0.0, rho1=rho1, rho2=0.0, eta=1.0)
    x, y, w = crandn(m1, r), crandn(r, m2), crandn(m1, m2)
    x1 = O.x_update(prob, x, y, w)
    np.testing.assert_allclose(x1, _kron_lstsq_x(y, w, prob.h, rho1), atol=1e-9)
    y1 = O.y_update(prob, x1, y, w)
    np.testing.assert_allclose(y1, _kron_lstsq_y(x1, w, prob.h, rho1), atol=1e-9)
    # KKT system eq. (KKTcondition) at the new blocks
    hr = prob.hr
    np.testing.assert_allclose(hr @ x1 @ (y @ y.conj().T), w @ y.conj().T, atol=1e-9)
    np.testing.assert_allclose((x1.conj().T @ hr @ x1) @ y1, x1.conj().T @ w, atol=1e-9)


@pytest.mark.parametrize("eta", [0.3, 1.0, 1.7])
def test_descent_inequalities(eta):
    """Propositions DirecX / DirecY: <d, nabla h> <= -||nabla h U_1||^2 / ((1 + 4 rho1) sigma_1^2)."""
    m1, r, m2, rho1 = 7, 3, 6, 0.4
    g = np.zeros((m1, m2, 1))
    prob = O.Problem(g, np.ones_like(g), r, rho1=rho1, eta=eta)
    for rank_y in (3, 2):
        x = crandn(m1, r)
        y = crandn(rank_y, m2)
        y = np.vstack([y, np.zeros((r - rank_y, m2))]) if rank_y < r else y
        w = crandn(m1, m2)
        gx = grad_x(x, y, w, prob.hth, rho1)
        dx = (O.x_update(prob, x, y, w) - x) / eta
        u, s, _ = np.linalg.svd(y)
        u1 = u[:, s > 1e-10]
        lhs = np.sum(dx * np.conj(gx))
        assert abs(lhs.imag) < 1e-9 * max(1, abs(lhs))
        assert lhs.real <= -np.linalg.norm(gx @ u1) ** 2 / ((1 + 4 * rho1) * s[0] ** 2) + 1e-9
        x1 = x + eta * dx
        gy = grad_y(x1, y, w, prob.hth, rho1)
        dy = (O.y_update(prob, x1, y, w) - y) / eta
        _, sx, vh = np.linalg.svd(x1)
        v1 = vh.conj().T[:, sx > 1e-10]
        lhs = np.sum(dy * np.conj(gy))
        assert lhs.real <= -np.linalg.norm(v1.conj().T @ gy) ** 2 / ((1 + 4 * rho1) * sx[0] ** 2) + 1e-9


# ----------------------------------------------------------------------------- whole iteration

def _small(seed=0, p=0.5, n=(7, 8, 5), r=2, **kw):
    d = make_inputs(*n, r, p=p, seed=seed, **kw)
    return d


@pytest.mark.parametrize("eta", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("n3", [1, 4, 5])
def test_objective_never_increases(eta, n3):
    """Theorem GlobConvergM with Proposition inWWk: f0 is non-increasing along the iterates."""
    d = _small(seed=n3, n=(6, 7, n3), r=2, p=0.5)
    _, info = O.complete(d["G"], d["omega"], 2, d["X0"], d["Y0"], 40, mu=0.05, rho1=0.2,
                         rho2=0.3, eta=eta, record_objective=True)
    f = info["f0"]
    assert all(f[i + 1] <= f[i] * (1 + 1e-12) + 1e-12 for i in range(len(f) - 1)), f


def test_conjugate_symmetry_is_preserved():
    """eq. (rcm_3-k+2) for the iterates X~, Y~, W~: the half spectrum determines the rest."""
    d = _small(n=(5, 6, 6), r=2)
    st, _ = O.complete(d["G"], d["omega"], 2, d["X0"], d["Y0"], 5)
    for a in (st.xt, st.yt, st.wt):
        m3 = a.shape[2]
        assert np.abs(a[:, :, 0].imag).max() < 1e-9 * np.abs(a).max()
        for k in range(1, m3):
            np.testing.assert_allclose(a[:, :, k], np.conj(a[:, :, m3 - k]), atol=1e-9 * np.abs(a).max())


def test_exact_recovery_in_one_sweep():
    """Fully observed, rho1 = 0, exact tubal rank r, generic start: Z = G after one iteration."""
    rng = np.random.default_rng(5)
    for n3 in (1, 4, 7):
        xg = rng.normal(size=(9, 3, n3))
        yg = rng.normal(size=(3, 8, n3))
        g = O.tprod(xg, yg)
        om = np.ones(g.shape, dtype=np.uint8)
        y0 = rng.normal(size=(3, 8, n3))
        st, _ = O.complete(g, om, 3, np.zeros((9, 3, n3)), y0, 1, mu=0.1, rho1=0.0, rho2=0.5)
        np.testing.assert_allclose(O.z_of(st), g, atol=1e-10 * np.abs(g).max())


def test_stationarity_residual_goes_to_zero():
    """Theorem ThKKT / eq. (AKKTstar): the factor-gradient residual tends to 0 and the W-KKT
    system holds at every iterate."""
    d = make_inputs(6, 7, 4, 2, p=0.7, seed=11, sigma_od=0.3)
    prob = O.Problem(d["G"], d["omega"], 2, 0.05, 0.1, 0.1)
    st = O.initial_state(prob, d["X0"], d["Y0"])
    res = []
    for it in range(3000):
        st = O.iterate(prob, st)
        if it in (10, 100, 2999):
            res.append(O.stationarity(prob, st))
    assert res[-1]["factor"] < 1e-8
    assert res[-1]["factor"] < res[0]["factor"]
    for s in res:
        assert s["w_kkt"] < 1e-12 and s["w_obs"] == 0.0


def test_unregularised_iteration_is_alternating_least_squares():
    """mu = rho1 = rho2 = 0, eta = 1: each frequency takes plain ALS steps and W fills the
    missing entries with Z (the TCTF special case, without rank adjustment)."""
    d = _small(seed=3, n=(6, 5, 3), r=2)
    prob = O.Problem(d["G"], d["omega"], 2, 0.0, 0.0, 0.0)
    st = O.initial_state(prob, d["X0"], d["Y0"])
    nxt = O.iterate(prob, st)
    for k in range(3):
        y, w = st.yt[:, :, k], st.wt[:, :, k]
        x1 = w @ y.conj().T @ np.linalg.inv(y @ y.conj().T)
        np.testing.assert_allclose(nxt.xt[:, :, k], x1, atol=1e-9)
        y1 = np.linalg.inv(x1.conj().T @ x1) @ x1.conj().T @ w
        np.testing.assert_allclose(nxt.yt[:, :, k], y1, atol=1e-9)
    z = O.z_of(nxt)
    np.testing.assert_allclose(nxt.w, np.where(d["omega"] == 1, d["G"], z), atol=1e-9)


def test_matrix_case_n3_equal_one():
    """n3 = 1: the transform is the identity and one iteration is regularised matrix ALS
    (checked step by step against Kronecker least squares and the W-step closed form)."""
    d = _small(seed=4, n=(7, 6, 1), r=2)
    mu, rho1, rho2 = 0.1, 0.3, 0.2
    prob = O.Problem(d["G"], d["omega"], 2, mu, rho1, rho2)
    st = O.initial_state(prob, d["X0"], d["Y0"])
    np.testing.assert_allclose(st.yt[:, :, 0], d["Y0"][:, :, 0], atol=1e-15)
    nxt = O.iterate(prob, st)
    y, w = d["Y0"][:, :, 0].astype(float), np.where(d["omega"] == 1, d["G"], 0.0)[:, :, 0]
    x1 = _kron_lstsq_x(y, w, prob.h, rho1)
    y1 = _kron_lstsq_y(x1, w, prob.h, rho1)
    np.testing.assert_allclose(nxt.xt[:, :, 0], x1, atol=1e-9)
    np.testing.assert_allclose(nxt.yt[:, :, 0], y1, atol=1e-9)
    z = (x1 @ y1).real[:, :, None]
    np.testing.assert_allclose(nxt.w, O.w_step_closed_form(z, d["G"], d["omega"], mu, rho2), atol=1e-9)


def test_termination_on_planted_differences():
    """Step 6 of the algorithm box on two hand-built states: the factor changes are measured
    in the sup norm (largest entry modulus, complex entries) and the W change in the
    Frobenius norm.  The planted entries separate those norms from the plausible slips (largest
    real part, largest |W| entry, sum of moduli)."""
    m1, m2, m3, r = 4, 5, 3, 2
    a = O.State(np.zeros((m1, r, m3), complex), np.zeros((r, m2, m3), complex), np.zeros((m1, m2, m3)),
                np.zeros((m1, m2, m3), complex))
    b = a.copy()
    b.xt[1, 0, 2] = 3.0 - 4.0j    # modulus 5
    b.xt[0, 1, 0] = -4.5          # larger real part, smaller modulus
    b.yt[1, 3, 1] = 2.0j          # modulus 2, real part 0
    b.yt[0, 0, 0] = 1.5
    b.w[0, 0, 0], b.w[3, 4, 2], b.w[2, 1, 1] = 1.0, -2.0, 2.0   # sqrt(1 + 4 + 4) = 3
    assert O.termination(a, b) == (5.0, 2.0, 3.0)
    assert O.termination(b, a) == (5.0, 2.0, 3.0)
    assert O.termination(b, b) == (0.0, 0.0, 0.0)


def test_termination_quantities():
    d = _small(seed=6)
    prob = O.Problem(d["G"], d["omega"], 2)
    a = O.initial_state(prob, d["X0"], d["Y0"])
    b = O.iterate(prob, a)
    dx, dy, dw = O.termination(a, b)
    assert dx > 0 and dy > 0 and dw > 0
    assert O.termination(b, b) == (0.0, 0.0, 0.0)


@pytest.mark.parametrize("m3", [1, 4, 5])
def test_stationarity_normalisation_against_spatial_gradient(m3):
    """The factor residual of Theorem ThKKT / eq. (AKKTstar), pinned through the spatial
    objective.  f0 of eq. (TETP-optim) depends on the real factors X, Y through the Fourier
    form eq. (fun-XYW), f0 = (1/m3) sum_k h_k(X~_k, Y~_k) + (W terms), and with eq. (bar BA-k)
    the real gradient is d f0 / d X = idft(nabla_X h), likewise for Y.  Parseval
    (sum_k ||A~_k||^2 = m3 ||A||^2) then gives

        sqrt(sum_k ||nabla_X h_k||^2 + ||nabla_Y h_k||^2) / (||W~|| (||X~|| + ||Y~||))
            = ||grad f0|| / (sqrt(m3) ||W|| (||X|| + ||Y||)),

    whose right side needs only the spatial objective (pinned term by term) and the
    t-product (pinned by its block-circulant definition); the gradient is taken by central
    differences over every entry of X and Y."""
    rng = np.random.default_rng(40 + m3)
    m1, m2, r = 4, 5, 2
    mu, rho1, rho2 = 0.2, 0.7, 0.3
    x, y, w = rng.normal(size=(m1, r, m3)), rng.normal(size=(r, m2, m3)), rng.normal(size=(m1, m2, m3))
    om = (rng.random((m1, m2, m3)) < 0.5).astype(np.uint8)
    prob = O.Problem(w, om, r, mu, rho1, rho2)
    st = O.State(O.dft3(x), O.dft3(y), w, O.dft3(w))
    f = lambda xx, yy: O.objective_spatial(O.tprod(xx, yy), w, mu, rho1, rho2)
    h = 1e-5
    g2 = 0.0
    for arr, is_x in ((x, True), (y, False)):
        for idx in np.ndindex(*arr.shape):
            e = np.zeros_like(arr)
            e[idx] = h
            fp = f(x + e, y) if is_x else f(x, y + e)
            fm = f(x - e, y) if is_x else f(x, y - e)
            g2 += ((fp - fm) / (2 * h)) ** 2
    expect = np.sqrt(g2) / (np.sqrt(m3) * np.linalg.norm(w) * (np.linalg.norm(x) + np.linalg.norm(y)))
    got = O.stationarity(prob, st)["factor"]
    assert abs(got - expect) <= 1e-7 * expect, (got, expect)


def test_metrics():
    m = np.array([[[1.0, 2.0], [3.0, 4.0]]])
    w = m.copy()
    w[0, 1, 1] = 5.0
    om = np.array([[[1, 1], [1, 0]]], dtype=np.uint8)
    assert np.isclose(O.nmae(w, m, om), 1.0 / 4.0)
    assert np.isclose(O.rse(w, m), 1.0 / np.sqrt(30.0))


# ----------------------------------------------------------------------------- step 5

def _iterated_state(seed=8, shape=(9, 8, 6), r=4, iters=3, **kw):
    d = make_inputs(*shape, r, p=0.6, seed=seed, weekly=True)
    prob = O.Problem(d["G"], d["omega"], r, **kw)
    st = O.initial_state(prob, d["X0"], d["Y0"])
    for _ in range(iters):
        st = O.iterate(prob, st)
    return prob, st


def test_rank_adjust_without_threshold_keeps_the_product():
    prob, st = _iterated_state()
    adj, ranks = O.rank_adjust(prob, st, 0.0)
    np.testing.assert_allclose(O.z_of(adj), O.z_of(st), atol=1e-10 * np.abs(O.z_of(st)).max())
    assert np.all(ranks == prob.r)


@pytest.mark.parametrize("tol", [0.05, 0.2])
def test_rank_adjust_is_the_best_approximation_of_each_frequency(tol):
    """Eckart-Young: the kept part of Z~_k has rank r_k and misses Z~_k by exactly the
    dropped singular values; the dropped ones are those below tol * (largest overall); the
    adjusted factors keep the conjugate symmetry eq. (rcm_3-k+2)."""
    prob, st = _iterated_state()
    adj, ranks = O.rank_adjust(prob, st, tol)
    m3 = prob.shape[2]
    zt = np.einsum("irk,rjk->ijk", st.xt, st.yt)
    za = np.einsum("irk,rjk->ijk", adj.xt, adj.yt)
    sv = [np.linalg.svd(zt[:, :, k], compute_uv=False) for k in range(m3)]
    smax = max(s[0] for s in sv)
    assert ranks.min() < prob.r   # the threshold bites somewhere at these settings
    for k in range(m3):
        q = ranks[k]
        assert q == int(np.sum(sv[k][:prob.r] > tol * smax))
        assert np.linalg.matrix_rank(za[:, :, k], tol=1e-9 * smax) == q
        err = np.linalg.norm(zt[:, :, k] - za[:, :, k]) ** 2
        assert np.isclose(err, np.sum(sv[k][q:] ** 2), rtol=1e-8, atol=1e-18 * smax ** 2)
        assert np.all(adj.xt[:, q:, k] == 0) and np.all(adj.yt[q:, :, k] == 0)
    for k in range(1, m3):
        np.testing.assert_allclose(adj.xt[:, :, k], np.conj(adj.xt[:, :, m3 - k]), atol=1e-12)


def test_rank_adjust_recovers_the_exact_tubal_rank():
    """A fully observed tensor of exact tubal rank 2 fitted with r = 4 (rho1 = 0: Z = G after one
    sweep): step 5 with a small threshold leaves rank 2 in every frequency and the same Z."""
    rng = np.random.default_rng(12)
    g = O.tprod(rng.normal(size=(10, 2, 5)), rng.normal(size=(2, 9, 5)))
    om = np.ones(g.shape, dtype=np.uint8)
    st, info = O.complete(g, om, 4, np.zeros((10, 4, 5)), rng.normal(size=(4, 9, 5)), 1, mu=0.1, rho1=0.0,
                          rho2=0.3, rank_tol=1e-8, rank_every=1)
    assert np.all(info["ranks"] == 2)
    assert O.tubal_rank(O.z_of(st)) == 2
    np.testing.assert_allclose(O.z_of(st), g, atol=1e-10 * np.abs(g).max())


def test_dropped_components_stay_zero_in_later_iterations():
    """After step 5 the pseudo-inverse steps of eq. (updataXYW1) never bring a dropped
    component back (its Gram rows are zero, so Lemma SVPMPI's inverse leaves it out)."""
    prob, st = _iterated_state()
    adj, ranks = O.rank_adjust(prob, st, 0.2)
    nxt = O.iterate(prob, adj)
    for k in range(prob.shape[2]):
        assert np.abs(nxt.xt[:, ranks[k]:, k]).max() == 0.0
        assert np.abs(nxt.yt[ranks[k]:, :, k]).max() == 0.0

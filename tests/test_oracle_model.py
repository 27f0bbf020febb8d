"""Pins of the oracle's section-3 model: the objective and the W-step (CPU only)."""
import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(777)


def _rand_problem(m1, m2, m3, p=0.5, seed=0):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(m1, m2, m3))
    g = rng.normal(size=(m1, m2, m3))
    om = (rng.random((m1, m2, m3)) < p).astype(np.uint8)
    return z, g, om


@pytest.mark.parametrize("m1,m2,m3,r", [(1, 1, 1, 1), (3, 4, 1, 2), (4, 3, 4, 2), (5, 4, 5, 3), (2, 6, 6, 1)])
def test_objective_parseval(m1, m2, m3, r):
    """eq. (TETP-optim) in the spatial domain equals eq. (fun-XYW) in the Fourier domain."""
    x = RNG.normal(size=(m1, r, m3))
    y = RNG.normal(size=(r, m2, m3))
    w = RNG.normal(size=(m1, m2, m3))
    mu, rho1, rho2 = 0.3, 0.7, 1.1
    fs = O.objective_spatial(O.tprod(x, y), w, mu, rho1, rho2)
    ff = O.model.fourier_objective_from_spatial(x, y, w, mu, rho1, rho2)
    assert np.isclose(fs, ff, rtol=1e-12)


def test_objective_terms_by_hand():
    """Each term of eq. (TETP-optim) on a tiny tensor with hand-countable values."""
    z = np.zeros((2, 2, 1))
    w = np.zeros((2, 2, 1))
    z[0, 0, 0] = 1.0          # one difference along mode 1 and ||Z - W||^2 = 1
    w[1, 1, 0] = 2.0          # one difference along mode 2 (of size 2), ||W||^2 = 4
    # 1/2 * 1 (fit: Z-W has entries 1 and -2 -> 1 + 4 = 5) ...
    f = O.objective_spatial(z, w, mu=0.0, rho1=0.0, rho2=0.0)
    assert np.isclose(f, 0.5 * 5.0)
    assert np.isclose(O.objective_spatial(z, w, 1.0, 0.0, 0.0) - f, 0.5 * 4.0)
    assert np.isclose(O.objective_spatial(z, w, 0.0, 1.0, 0.0) - f, 0.5 * 1.0)
    assert np.isclose(O.objective_spatial(z, w, 0.0, 0.0, 1.0) - f, 0.5 * 4.0)


@pytest.mark.parametrize("m1,m2,m3,p", [(3, 1, 2, 0.5), (3, 2, 2, 0.5), (4, 6, 3, 0.3), (5, 9, 2, 0.7),
                                        (2, 12, 3, 0.0), (2, 12, 3, 1.0)])
@pytest.mark.parametrize("mu,rho2", [(0.01, 0.01), (0.5, 2.0), (0.0, 0.3), (0.2, 0.0)])
def test_w_step_banded_kkt_equals_closed_form(m1, m2, m3, p, mu, rho2):
    """The KKT system eq. (subquKKT) (banded solve) and the closed form eq. (Wkiom) agree,
    the KKT residual vanishes and observed entries equal G exactly."""
    z, g, om = _rand_problem(m1, m2, m3, p, seed=int(100 * p) + m2)
    w1 = O.w_step(z, g, om, mu, rho2)
    w2 = O.w_step_closed_form(z, g, om, mu, rho2)
    np.testing.assert_allclose(w1, w2, atol=1e-12)
    r_un, r_ob = O.w_kkt_residual(w1, z, g, om, mu, rho2)
    assert r_un < 1e-12
    assert r_ob == 0.0


def test_w_step_rho2_zero_is_shrinkage():
    """rho2 = 0: unobserved entries are Z / (1 + mu) exactly (eq. (Wkiom) with K dropped)."""
    z, g, om = _rand_problem(4, 7, 3, 0.4, seed=3)
    mu = 0.25
    w = O.w_step(z, g, om, mu, 0.0)
    un = om == 0
    np.testing.assert_allclose(w[un], z[un] / (1 + mu), rtol=1e-15)
    np.testing.assert_array_equal(w[~un], g[~un])


def test_w_step_without_regularisation_fills_with_z():
    """mu = rho2 = 0 (the plain factorisation model, eq. (ETP-optim)): W = P_Omega(G) + P_Omega^C(Z)."""
    z, g, om = _rand_problem(3, 5, 4, 0.5, seed=4)
    w = O.w_step(z, g, om, 0.0, 0.0)
    np.testing.assert_allclose(w, np.where(om == 1, g, z), atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_w_step_minimises_g_k_by_brute_force_least_squares(seed):
    """W-step = argmin of sum_k g_k subject to P_Omega(W) = P_Omega(G) (eq. (WETP-optim20)),
    checked against a dense least-squares solve of the stacked quadratic."""
    m1, m2, m3 = 2, 5, 2
    z, g, om = _rand_problem(m1, m2, m3, 0.4, seed=seed)
    mu, rho2 = 0.3, 0.8
    w = O.w_step(z, g, om, mu, rho2)
    # unknowns: unobserved entries; g_k = 1/2(||Z_k - W_k||^2 + rho2 ||W_k K^T||^2 + mu ||W_k||^2)
    k = O.toeplitz_diff(m2)
    idx = np.argwhere(om == 0)
    n = len(idx)
    pos = {tuple(t): c for c, t in enumerate(idx)}
    rows, rhs = [], []

    def add(coefs, const):
        # residual = sum coefs[c] x_c + const  ->  row coefs, rhs -const
        row = np.zeros(n)
        for c, v in coefs:
            row[c] += v
        rows.append(row)
        rhs.append(-const)

    for i in range(m1):
        for kk in range(m3):
            for j in range(m2):
                known = om[i, j, kk] == 1
                c = pos.get((i, j, kk))
                # fit term  (W - Z)
                add([] if known else [(c, 1.0)], (g[i, j, kk] if known else 0.0) - z[i, j, kk])
                # ridge term sqrt(mu) W
                add([] if known else [(c, np.sqrt(mu))], np.sqrt(mu) * g[i, j, kk] if known else 0.0)
            for q in range(m2 - 1):
                coefs, const = [], 0.0
                for j in range(m2):
                    if k[q, j] == 0:
                        continue
                    v = np.sqrt(rho2) * k[q, j]
                    if om[i, j, kk] == 1:
                        const += v * g[i, j, kk]
                    else:
                        coefs.append((pos[(i, j, kk)], v))
                add(coefs, const)
    sol = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
    for c, t in enumerate(idx):
        assert np.isclose(w[tuple(t)], sol[c], atol=1e-10)


def test_w_minus_z_bound():
    """Bound after Proposition KKProp: sum_k ||(W_k - Z_k)_{Omega^C}|| <= (mu + 4 rho2) sum_k ||W_k||."""
    for seed in range(5):
        z, g, om = _rand_problem(5, 8, 3, 0.5, seed=seed)
        g = z + 0.1 * RNG.normal(size=z.shape)
        for mu, rho2 in [(0.01, 0.01), (0.1, 0.5), (0.0, 0.2)]:
            w = O.w_step(z, g, om, mu, rho2)
            un = om == 0
            lhs = sum(np.linalg.norm(((w - z) * un)[:, :, k]) for k in range(3))
            rhs = (mu + 4 * rho2) * sum(np.linalg.norm(w[:, :, k]) for k in range(3))
            assert lhs <= rhs + 1e-12


def test_w_step_rows_fully_observed_and_fully_missing():
    """A row with every entry observed is G; a fully missing row solves K_{mu rho2} w = z."""
    m1, m2, m3 = 2, 6, 1
    z = RNG.normal(size=(m1, m2, m3))
    g = RNG.normal(size=(m1, m2, m3))
    om = np.zeros((m1, m2, m3), dtype=np.uint8)
    om[0] = 1
    mu, rho2 = 0.1, 0.7
    w = O.w_step(z, g, om, mu, rho2)
    np.testing.assert_array_equal(w[0], g[0])
    kmr = O.k_mu_rho2(m2, mu, rho2)
    np.testing.assert_allclose(w[1, :, 0] @ kmr, z[1, :, 0], atol=1e-12)

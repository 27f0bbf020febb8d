"""The closed form of H_rho1^{-1} that the X-update's stencil uses, against the matrix of
eq. (KKTcondition) itself (CPU only).

H_rho1 = I + rho1 H^T H is tridiagonal with diagonal 1 + 2 rho1 (1 + rho1 in the two end
rows) and off-diagonal -rho1.  With lambda the root in (0, 1) of
rho1 lambda^2 - (1 + 2 rho1) lambda + rho1 = 0 and c = lambda / (rho1 (1 - lambda^2)), its
inverse is c (lambda^|i-j| + lambda^(i+j+1) + lambda^(2n-1-i-j)) up to terms of order
lambda^(2n): the direct term plus one mirror image per end row.
"""
import numpy as np
import pytest

from oracle.model import h_rho1


def lam_c(rho1):
    a = 1.0 + 2.0 * rho1
    lam = 2.0 * rho1 / (a + np.sqrt(a * a - 4.0 * rho1 * rho1))
    return lam, lam / (rho1 * (1.0 - lam * lam))


def closed_form(n, rho1, k=None):
    lam, c = lam_c(rho1)
    i, j = np.arange(n)[:, None], np.arange(n)[None, :]
    g = c * (lam ** np.abs(i - j) + lam ** (i + j + 1) + lam ** (2 * n - 1 - i - j))
    if k is not None:
        g = np.where(np.abs(i - j) <= k, g, 0.0)
    return g


def half_width(rho1):
    """Least k with lambda^(k + 1) <= 2^-40."""
    lam, _ = lam_c(rho1)
    k = 0
    while lam ** (k + 1) > 2.0 ** -40:
        k += 1
    return k


@pytest.mark.parametrize("n,rho1", [(529, 0.01), (40, 0.1), (12, 0.01), (9, 0.05), (300, 0.15), (30, 0.5)])
def test_closed_form_inverse(n, rho1):
    hinv = np.linalg.inv(h_rho1(n, rho1))
    lam, _ = lam_c(rho1)
    # the neglected images of images are of order lambda^(2 n)
    assert np.abs(closed_form(n, rho1) - hinv).max() <= 1e-13 + 4 * lam ** (2 * n)


def test_root_and_scale():
    for rho1 in (1e-4, 0.01, 0.1, 1.0):
        lam, c = lam_c(rho1)
        assert abs(rho1 * lam * lam - (1 + 2 * rho1) * lam + rho1) < 1e-15
        # interior row of H_rho1 applied to c lambda^|i - j| gives the unit vector
        assert abs((1 + 2 * rho1) * c - 2 * rho1 * c * lam - 1.0) < 1e-13


@pytest.mark.parametrize("rho1,k", [(0.01, 5), (0.1, 11), (0.0, 0)])
def test_half_width_and_truncation(rho1, k):
    """The half-width rule, and the truncated stencil's error on rows whose scales differ by
    up to 10^4: below FP32's rounding unit relative to each row."""
    if rho1 == 0.0:
        assert k == 0   # H_rho1 = I
        return
    assert half_width(rho1) == k
    n = 200
    rng = np.random.default_rng(1)
    v = rng.standard_normal((n, 4)) * 10.0 ** rng.uniform(-2, 2, size=(n, 1))
    exact = np.linalg.solve(h_rho1(n, rho1), v)
    approx = closed_form(n, rho1, k) @ v
    err = np.abs(approx - exact).max(axis=1) / np.abs(exact).max(axis=1)
    assert err.max() < 2.0 ** -24

"""Section 3 of the paper: the regularised model and its separable Fourier form, in FP64.

Part of the FP64 CPU oracle.  Test infrastructure only: nothing in the library's product
path imports this.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from .tensor_algebra import dft3, toeplitz_diff, unfold


def h_rho1(m1: int, rho1: float) -> np.ndarray:
    """H_rho1 = I + rho1 H^T H (the matrix of eq. (KKTcondition)), H = Toeplitz(0,1,-1) of size (m1-1) x m1."""
    h = toeplitz_diff(m1)
    return np.eye(m1) + rho1 * h.T @ h


def k_mu_rho2(m2: int, mu: float, rho2: float) -> np.ndarray:
    """K_{mu rho2} = (1 + mu) I + rho2 K^T K (below eq. (subquKKT)), K of size (m2-1) x m2."""
    k = toeplitz_diff(m2)
    return (1.0 + mu) * np.eye(m2) + rho2 * k.T @ k


def objective_spatial(z: np.ndarray, w: np.ndarray, mu: float, rho1: float, rho2: float) -> float:
    """f0 of eq. (TETP-optim) with Z = X * Y given:

    1/2 ||Z - W||^2 + mu/2 ||W||^2 + rho1/2 ||H unfold(Z, 1)||^2 + rho2/2 ||K unfold(W, 2)||^2.
    """
    m1, m2, _ = z.shape
    h = toeplitz_diff(m1)
    k = toeplitz_diff(m2)
    f = 0.5 * np.sum((z - w) ** 2) + 0.5 * mu * np.sum(w ** 2)
    f += 0.5 * rho1 * np.sum((h @ unfold(z, 1)) ** 2)
    f += 0.5 * rho2 * np.sum((k @ unfold(w, 2)) ** 2)
    return float(f)


def objective_fourier(xt: np.ndarray, yt: np.ndarray, wt: np.ndarray,
                      mu: float, rho1: float, rho2: float) -> float:
    """f0 in the separable form eq. (fun-XYW), from full-spectrum X~ (m1,r,m3), Y~ (r,m2,m3), W~.

    1/(2 m3) sum_k { ||X~_k Y~_k - W~_k||^2 + rho1 ||H X~_k Y~_k||^2 + rho2 ||W~_k K^T||^2 + mu ||W~_k||^2 }.
    """
    m1, _, m3 = xt.shape
    m2 = yt.shape[1]
    h = toeplitz_diff(m1)
    k = toeplitz_diff(m2)
    total = 0.0
    for kk in range(m3):
        zk = xt[:, :, kk] @ yt[:, :, kk]
        wk = wt[:, :, kk]
        total += np.sum(np.abs(zk - wk) ** 2)
        total += rho1 * np.sum(np.abs(h @ zk) ** 2)
        total += rho2 * np.sum(np.abs(wk @ k.T) ** 2)
        total += mu * np.sum(np.abs(wk) ** 2)
    return float(total / (2.0 * m3))


def w_step(z: np.ndarray, g: np.ndarray, omega_mask: np.ndarray, mu: float, rho2: float) -> np.ndarray:
    """Step 4 of the TCTF2R algorithm: the minimiser of g_k for every frontal slice k.

    Solves the KKT system eq. (subquKKT) row by row: for every (i, k) and every j,
      j in Omega_ik:      w_j = g_j
      j not in Omega_ik:  (w K_{mu rho2})_j = z_j.
    K_{mu rho2} is tridiagonal, so each row's system is tridiagonal; all rows are stacked
    into one block-diagonal banded system (no coupling between rows) and solved with a
    banded LU (LAPACK gbsv through scipy).
    """
    m1, m2, m3 = z.shape
    kmr = k_mu_rho2(m2, mu, rho2)
    if m2 > 2:
        assert np.count_nonzero(np.triu(kmr, 2)) == 0 and np.count_nonzero(np.tril(kmr, -2)) == 0
    obs = omega_mask.astype(bool)
    # rows (i, k) with j contiguous
    z_r = np.transpose(z, (0, 2, 1)).reshape(-1, m2)
    g_r = np.transpose(g, (0, 2, 1)).reshape(-1, m2)
    o_r = np.transpose(obs, (0, 2, 1)).reshape(-1, m2)
    nrow = z_r.shape[0]
    # equation j of a row: sum_l w_l K[l, j]; coefficient of w_{j-1} is K[j-1, j], of w_{j+1} is K[j+1, j]
    diag = np.where(o_r, 1.0, np.broadcast_to(np.diag(kmr), (nrow, m2)))
    lower = np.zeros((nrow, m2))   # coefficient of w_{j-1} in equation j
    upper = np.zeros((nrow, m2))   # coefficient of w_{j+1} in equation j
    if m2 > 1:
        lower[:, 1:] = np.where(o_r[:, 1:], 0.0, np.array([kmr[j - 1, j] for j in range(1, m2)])[None, :])
        upper[:, :-1] = np.where(o_r[:, :-1], 0.0, np.array([kmr[j + 1, j] for j in range(m2 - 1)])[None, :])
    rhs = np.where(o_r, g_r, z_r).reshape(-1)
    n = nrow * m2
    ab = np.zeros((3, n))
    # banded storage: ab[1 + i - j, j] = A[i, j]
    ab[1, :] = diag.reshape(-1)
    up = upper.reshape(-1)      # A[e, e+1] for equation e
    lo = lower.reshape(-1)      # A[e, e-1]
    ab[0, 1:] = up[:-1]
    ab[2, :-1] = lo[1:]
    # rows never couple: equation at j = m2-1 has no upper entry, j = 0 has no lower one
    w_r = solve_banded((1, 1), ab, rhs).reshape(nrow, m2)
    # observed entries are G itself (second line of eq. (Wkiom)); the pivoted LU can leave
    # rounding there, so they are written back exactly
    w_r = np.where(o_r, g_r, w_r)
    return np.transpose(w_r.reshape(m1, m3, m2), (0, 2, 1)).copy()


def w_step_closed_form(z: np.ndarray, g: np.ndarray, omega_mask: np.ndarray,
                       mu: float, rho2: float) -> np.ndarray:
    """Step 4 via the closed form eq. (Wkiom), one row (i, k) at a time (small tensors only).

    With K = [K1, K2] split by the observed / unobserved columns of the row:
      w_C = (z_C - rho2 g_O K1^T K2) ((1 + mu) I + rho2 K2^T K2)^{-1},   w_O = g_O.
    """
    m1, m2, m3 = z.shape
    k = toeplitz_diff(m2)
    w = np.zeros_like(z, dtype=float)
    obs = omega_mask.astype(bool)
    for i in range(m1):
        for kk in range(m3):
            o = obs[i, :, kk]
            c = ~o
            row = np.zeros(m2)
            row[o] = g[i, o, kk]
            if c.any():
                k1 = k[:, o]
                k2 = k[:, c]
                rhs = z[i, c, kk] - rho2 * (g[i, o, kk] @ k1.T @ k2)
                mat = (1.0 + mu) * np.eye(int(c.sum())) + rho2 * k2.T @ k2
                row[c] = np.linalg.solve(mat.T, rhs)   # rhs @ mat^{-1}; mat is symmetric
            w[i, :, kk] = row
    return w


def w_kkt_residual(w: np.ndarray, z: np.ndarray, g: np.ndarray, omega_mask: np.ndarray,
                   mu: float, rho2: float) -> tuple[float, float]:
    """Residuals of eq. (subquKKT): max |(W_k K_{mu rho2} - Z_k)_ij| over unobserved (i, j, k),
    and max |W - G| over observed entries."""
    m2 = z.shape[1]
    kmr = k_mu_rho2(m2, mu, rho2)
    obs = omega_mask.astype(bool)
    wk = np.einsum("ijk,jl->ilk", w, kmr)
    r_unobs = np.abs(wk - z)[~obs]
    r_obs = np.abs(w - g)[obs]
    return (float(r_unobs.max()) if r_unobs.size else 0.0,
            float(r_obs.max()) if r_obs.size else 0.0)


def fourier_objective_from_spatial(x: np.ndarray, y: np.ndarray, w: np.ndarray,
                                   mu: float, rho1: float, rho2: float) -> float:
    """eq. (fun-XYW) evaluated from real spatial X, Y, W (transforms them first)."""
    return objective_fourier(dft3(x), dft3(y), dft3(w), mu, rho1, rho2)

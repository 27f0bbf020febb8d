"""Section 4 of the paper: the TCTF2R iteration, written step by step in FP64.

Part of the FP64 CPU oracle.  Test infrastructure only: nothing in the library's product
path imports this.

Readings taken where the paper leaves a choice (each is listed in the design notes):
* step sizes alpha_kl / L_k1 and beta_kl / L_k2 of eq. (updataXYW1) are one common
  constant ``eta`` (default 1, the exact block minimiser along the direction);
* the rank vector stays r for every frequency (step 5 adjusts nothing);
* the Moore-Penrose inverse of a Hermitian Gram is formed from its eigen-decomposition
  (Lemma SVPMPI), keeping eigenvalues above r * eps64 * lambda_max;
* W^(0) = P_Omega(G) (missing entries start at 0, as P_Omega fills them);
* all m3 frequencies are updated (full spectrum), and the iterates are checked for the
  conjugate symmetry eq. (rcm_3-k+2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import lu_factor, lu_solve

from .model import h_rho1, k_mu_rho2, objective_spatial, w_step
from .tensor_algebra import dft3, idft3, toeplitz_diff

EPS64 = np.finfo(np.float64).eps


def pinv_h(gram: np.ndarray) -> np.ndarray:
    """Moore-Penrose inverse of a Hermitian PSD matrix through its eigen-decomposition
    (Lemma SVPMPI): V diag(1/lambda_i) V^*, over eigenvalues lambda_i > r eps64 lambda_max."""
    r = gram.shape[0]
    lam, v = np.linalg.eigh(gram)
    lam_max = float(lam[-1]) if lam.size else 0.0
    tau = max(r * EPS64 * lam_max, 0.0)
    keep = lam > tau
    if not keep.any():
        return np.zeros_like(gram)
    vk = v[:, keep]
    return (vk / lam[keep]) @ vk.conj().T


def grad_x(xk, yk, wk, hth, rho1):
    """nabla_{X~_k} h_k of eq. (hkXYDer): (X~Y~ - W~) Y~^* + rho1 H^T H X~ Y~ Y~^*."""
    yh = yk.conj().T
    return (xk @ yk - wk) @ yh + rho1 * hth @ xk @ yk @ yh


def grad_y(xk, yk, wk, hth, rho1):
    """nabla_{Y~_k} h_k of eq. (hkXYDer): X~^*(X~Y~ - W~) + rho1 X~^* H^T H X~ Y~."""
    xh = xk.conj().T
    return xh @ (xk @ yk - wk) + rho1 * xh @ hth @ xk @ yk


def h_k(xk, yk, wk, h, rho1):
    """h_k of eq. (kXYETP-optim20): 1/2 (||X~Y~ - W~||^2 + rho1 ||H X~ Y~||^2)."""
    zk = xk @ yk
    return 0.5 * (np.sum(np.abs(zk - wk) ** 2) + rho1 * np.sum(np.abs(h @ zk) ** 2))


@dataclass
class Problem:
    """Data and parameters of one completion (the inputs of the algorithm box)."""

    g: np.ndarray          # observed tensor (m1, m2, m3); values off Omega are ignored
    omega: np.ndarray      # 0/1 mask (m1, m2, m3)
    r: int
    mu: float = 1e-2
    rho1: float = 1e-2
    rho2: float = 1e-2
    eta: float = 1.0
    _cache: dict = field(default_factory=dict, repr=False)

    def __post_init__(self):
        self.g = np.asarray(self.g, dtype=np.float64)
        self.omega = np.asarray(self.omega).astype(bool)
        m1, m2, _ = self.g.shape
        self.h = toeplitz_diff(m1)
        self.hth = self.h.T @ self.h
        self.hr = h_rho1(m1, self.rho1)
        self.hr_lu = lu_factor(self.hr)
        self.kmr = k_mu_rho2(m2, self.mu, self.rho2)

    @property
    def shape(self):
        return self.g.shape

    def p_omega_g(self) -> np.ndarray:
        """P_Omega(G): observed entries kept, the rest 0 (section 3.1)."""
        return np.where(self.omega, self.g, 0.0)


@dataclass
class State:
    """Iterate of the algorithm: full-spectrum X~, Y~, W~ and the spatial W."""

    xt: np.ndarray   # (m1, r, m3) complex
    yt: np.ndarray   # (r, m2, m3) complex
    w: np.ndarray    # (m1, m2, m3) real
    wt: np.ndarray   # (m1, m2, m3) complex
    it: int = 0

    def copy(self) -> "State":
        return State(self.xt.copy(), self.yt.copy(), self.w.copy(), self.wt.copy(), self.it)


def initial_state(prob: Problem, x0: np.ndarray, y0: np.ndarray) -> State:
    """Initialisation of the algorithm box from real X0, Y0 (conjugate symmetry holds by
    construction) and W0 = P_Omega(G)."""
    w0 = prob.p_omega_g()
    return State(dft3(np.asarray(x0, float)), dft3(np.asarray(y0, float)), w0, dft3(w0), 0)


def x_update(prob: Problem, xk, yk, wk):
    """First line of eq. (updataXYW1) with step eta:
    X~ + eta * d_X,  d_X = -H_rho1^{-1} nabla_X h_k (Y~ Y~^*)^+."""
    gy = yk @ yk.conj().T
    gx = grad_x(xk, yk, wk, prob.hth, prob.rho1)
    d = -lu_solve(prob.hr_lu, gx) @ pinv_h(gy)
    return xk + prob.eta * d


def y_update(prob: Problem, xk_new, yk, wk):
    """Second line of eq. (updataXYW1) with step eta:
    Y~ + eta * d_Y,  d_Y = -(X~^* H_rho1 X~)^+ nabla_Y h_k(X~^(l+1), Y~^(l))."""
    gxx = xk_new.conj().T @ prob.hr @ xk_new
    gy = grad_y(xk_new, yk, wk, prob.hth, prob.rho1)
    d = -pinv_h(gxx) @ gy
    return yk + prob.eta * d


def iterate(prob: Problem, st: State, check_symmetry: bool = True) -> State:
    """One pass of steps 1-4 and 7 of the TCTF2R algorithm (step 5 is the identity, step 6
    is evaluated by :func:`termination`)."""
    m1, m2, m3 = prob.shape
    xt_new = np.empty_like(st.xt)
    yt_new = np.empty_like(st.yt)
    # step 1: X~_k for every k
    sl = lambda a, k: np.ascontiguousarray(a[:, :, k])   # frontal slice k
    for k in range(m3):
        xt_new[:, :, k] = x_update(prob, sl(st.xt, k), sl(st.yt, k), sl(st.wt, k))
    # step 2: Y~_k for every k, with the new X~_k and the old W~_k
    for k in range(m3):
        yt_new[:, :, k] = y_update(prob, sl(xt_new, k), sl(st.yt, k), sl(st.wt, k))
    # step 3: Z~_k = X~_k Y~_k, then Z by eq. (barAAk)
    zt = np.einsum("irk,rjk->ijk", xt_new, yt_new)
    z_c = idft3(zt)
    scale = max(np.abs(z_c).max(), 1e-300)
    if check_symmetry:
        assert np.abs(z_c.imag).max() <= 1e-9 * scale, "Z lost its conjugate symmetry"
    z = z_c.real
    # step 4: W-step
    w = w_step(z, prob.g, prob.omega, prob.mu, prob.rho2)
    # step 7: W~ by eq. (bar BA-k)
    wt = dft3(w)
    return State(xt_new, yt_new, w, wt, st.it + 1)


def rank_adjust(prob: Problem, st: State, tol: float):
    """Step 5 of the algorithm box (adjust the rank vector r^(l+1) and the sizes of X~_k,
    Y~_k) by the following rule (the paper leaves the rule open): in every frequency k keep the
    components of Z~_k = X~_k Y~_k whose singular values exceed tol times the largest singular
    value over all frequencies.  With the SVD Z~_k = U S V^*, the kept part is written as
    X~_k = U_q S_q, Y~_k = V_q^* in the first q = r_k columns / rows, the rest zero (the factor
    sizes stay r; the zero part is what "the size" r_k leaves out).  Frequencies past m3 / 2
    take the conjugates (eq. (rcm_3-k+2)); the real frequencies are decomposed as real
    matrices.  Returns (state, r_k for every k)."""
    m3 = prob.shape[2]
    r = prob.r
    zt = np.einsum("irk,rjk->ijk", st.xt, st.yt)
    real = lambda k: k == 0 or (m3 % 2 == 0 and k == m3 // 2)
    svd = lambda k: np.linalg.svd(zt[:, :, k].real if real(k) else zt[:, :, k], full_matrices=False)
    smax = max(float(np.linalg.svd(zt[:, :, k], compute_uv=False)[0]) for k in range(m3))
    xt = np.zeros_like(st.xt)
    yt = np.zeros_like(st.yt)
    ranks = np.zeros(m3, dtype=int)
    for k in range(m3 // 2 + 1):
        u, sv, vh = svd(k)
        q = int(np.sum(sv[:r] > tol * smax))
        xt[:, :q, k] = u[:, :q] * sv[:q]
        yt[:q, :, k] = vh[:q]
        ranks[k] = q
        kc = (m3 - k) % m3
        if kc != k:
            xt[:, :, kc] = np.conj(xt[:, :, k])
            yt[:, :, kc] = np.conj(yt[:, :, k])
            ranks[kc] = q
    return State(xt, yt, st.w, st.wt, st.it), ranks


def z_of(st: State) -> np.ndarray:
    """Z = X * Y of the state (real part of the inverse transform of X~_k Y~_k)."""
    return idft3(np.einsum("irk,rjk->ijk", st.xt, st.yt)).real


def objective(prob: Problem, st: State) -> float:
    """f0 of eq. (TETP-optim) at the state, in the spatial domain."""
    return objective_spatial(z_of(st), st.w, prob.mu, prob.rho1, prob.rho2)


def termination(prev: State, cur: State) -> tuple[float, float, float]:
    """Quantities of step 6: ||X~+ - X~||_inf, ||Y~+ - Y~||_inf, ||W+ - W||_F."""
    return (float(np.abs(cur.xt - prev.xt).max()), float(np.abs(cur.yt - prev.yt).max()),
            float(np.linalg.norm(cur.w - prev.w)))


def stationarity(prob: Problem, st: State) -> dict:
    """Stationarity measures of Theorem ThKKT / eq. (AKKTstar) at the state.

    ``factor``: sqrt(sum_k ||nabla_X h_k||^2 + ||nabla_Y h_k||^2) / (||W~|| (||X~|| + ||Y~||));
    ``w_kkt``: max over unobserved entries of |(W_k K_{mu rho2} - Z_k)_ij| / ||Z||_inf;
    ``w_obs``: max over observed entries of |W - G| (must be exactly 0).
    """
    m3 = prob.shape[2]
    s = 0.0
    for k in range(m3):
        gx = grad_x(st.xt[:, :, k], st.yt[:, :, k], st.wt[:, :, k], prob.hth, prob.rho1)
        gy = grad_y(st.xt[:, :, k], st.yt[:, :, k], st.wt[:, :, k], prob.hth, prob.rho1)
        s += np.sum(np.abs(gx) ** 2) + np.sum(np.abs(gy) ** 2)
    denom = np.linalg.norm(st.wt) * (np.linalg.norm(st.xt) + np.linalg.norm(st.yt))
    z = z_of(st)
    wk = np.einsum("ijk,jl->ilk", st.w, prob.kmr)
    un = ~prob.omega
    w_kkt = float(np.abs(wk - z)[un].max() / max(np.abs(z).max(), 1e-300)) if un.any() else 0.0
    w_obs = float(np.abs(st.w - prob.g)[prob.omega].max()) if prob.omega.any() else 0.0
    return {"factor": float(np.sqrt(s) / max(denom, 1e-300)), "w_kkt": w_kkt, "w_obs": w_obs}


def complete(g, omega_mask, r, x0, y0, iters, mu=1e-2, rho1=1e-2, rho2=1e-2, eta=1.0,
             record_objective=False, rank_tol=0.0, rank_every=0):
    """Run ``iters`` iterations of TCTF2R from (X0, Y0, W0 = P_Omega(G)).

    With rank_every > 0, step 5 (:func:`rank_adjust` with ``rank_tol``) runs after
    iterations rank_every, 2 rank_every, ...  Returns (state, info) where info holds the
    objective history if requested (f0 before the first iteration, then after each) and the
    last rank vector.
    """
    prob = Problem(g, omega_mask, r, mu, rho1, rho2, eta)
    st = initial_state(prob, x0, y0)
    hist = []
    ranks = np.full(prob.shape[2], r)
    if record_objective:
        hist.append(objective(prob, st))
    for _ in range(iters):
        st = iterate(prob, st)
        if rank_every > 0 and st.it % rank_every == 0:
            st, ranks = rank_adjust(prob, st, rank_tol)
        if record_objective:
            hist.append(objective(prob, st))
    return st, {"f0": hist, "problem": prob, "ranks": ranks}


def rse(w: np.ndarray, m: np.ndarray, mask: np.ndarray | None = None) -> float:
    """Relative squared-error norm ||W - M||_F / ||M||_F (over ``mask`` when given)."""
    if mask is not None:
        sel = mask.astype(bool)
        return float(np.linalg.norm((w - m)[sel]) / max(np.linalg.norm(m[sel]), 1e-300))
    return float(np.linalg.norm(w - m) / max(np.linalg.norm(m), 1e-300))


def nmae(w: np.ndarray, m: np.ndarray, omega_mask: np.ndarray) -> float:
    """NMAE of section 5 over the missing entries: sum |M - W| / sum |M| off Omega."""
    un = ~omega_mask.astype(bool)
    return float(np.abs(m - w)[un].sum() / max(np.abs(m)[un].sum(), 1e-300))

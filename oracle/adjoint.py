"""Reverse-mode derivatives of the TCTF2R iteration, written out by hand in FP64.

Part of the FP64 CPU oracle (test infrastructure only: nothing in the library's product
path imports this).  It differentiates the oracle's own iteration (``algorithm.iterate``)
over the full spectrum, one step of the algorithm box at a time, in reverse order.

Convention for complex variables (the real-gradient convention that section 4.1's
gradients eq. (hkXYDer) follow, cf. Theorem PDconj): the adjoint of a complex array z is
``z_bar = dL/dRe z + i dL/dIm z``, so that a first-order change of the real loss L is
``dL = Re sum conj(z_bar) dz``.  For real arrays it is the ordinary gradient.  The rules
used below follow from that definition:

* C = A B:            A_bar += C_bar B^*,   B_bar += A^* C_bar;
* C = A^*:            A_bar += C_bar^*;
* C = G^{-1}:         G_bar += -C^* C_bar C^*;
* G = Y Y^*:          Y_bar += (G_bar + G_bar^*) Y;
* A~ = dft3(A) (real A, eq. (bar BA-k), A~_k = sum_l omega^{kl} A_l):
                      A_bar = Re sum_k omega^{-kl} A~_bar_k = Re fft(A~_bar);
* A = Re idft3(A~) (eq. (barAAk)):
                      A~_bar = ifft(A_bar)  (= dft3(A_bar) / m3).

The step sizes of eq. (updataXYW1) are one common constant eta, and the Grams G_Y = Y~Y~^* and
G_X = X~^* H_rho1 X~ are taken to have full rank (then their pseudo-inverses of Lemma
SVPMPI are inverses, P = I, and the updates of eq. (updataXYW1) simplify to

    X~+ = (1 - eta) X~ + eta H_rho1^{-1} W~ Y~^* G_Y^{-1},
    Y~+ = (1 - eta) Y~ + eta G_X^{-1} X~+^* W~,

because grad_X = H_rho1 X~ G_Y - W~ Y~^* and grad_Y = G_X Y~ - X~^* W~, see eq. (KKTcondition)).
The W-step of eq. (subquKKT) keeps observed entries at G and solves
K_uu w_u = z_u - K_uo g_o on the unobserved ones of each row (i, :, k), K = K_{mu rho2} =
(1 + mu) I + rho2 K^T K symmetric, so z_bar_u = K_uu^{-1} w_bar_u and z_bar_o = 0, and
dw_u / dmu = -K_uu^{-1} w_u, dw_u / drho2 = -K_uu^{-1} (K^T K w)_u.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_banded

from .algorithm import Problem, State, initial_state, iterate
from .tensor_algebra import dft3, idft3, toeplitz_diff


def _h(a):
    """Conjugate transpose of the last two axes."""
    return np.conj(np.swapaxes(a, -1, -2))


def _slices(a):
    """Frontal slices as a leading axis: (m1, m2, m3) -> (m3, m1, m2)."""
    return np.moveaxis(a, 2, 0)


def _unslices(a):
    return np.moveaxis(a, 0, 2)


@dataclass
class ThetaBar:
    """Adjoints of the weights mu, rho1, rho2 (accumulated)."""

    mu: float = 0.0
    rho1: float = 0.0
    rho2: float = 0.0

    def as_array(self):
        return np.array([self.mu, self.rho1, self.rho2])


def w_step_adjoint(prob: Problem, w_new: np.ndarray, w_bar: np.ndarray, theta_bar: ThetaBar) -> np.ndarray:
    """Adjoint of the W-step (eq. (subquKKT) / eq. (Wkiom)) at its solution ``w_new``.

    Returns z_bar (zero on observed entries) and adds the mu and rho2 adjoints:
    mu_bar = -<lambda_u, w_u>, rho2_bar = -<lambda_u, (K^T K w)_u> with lambda_u = K_uu^{-1} w_bar_u
    (K_uu symmetric, so the adjoint solve is the same tridiagonal solve)."""
    m1, m2, m3 = w_new.shape
    obs = prob.omega
    d = toeplitz_diff(m2)
    ktk = d.T @ d
    kmr = prob.kmr
    # rows (i, k) with j contiguous
    wb = np.transpose(w_bar, (0, 2, 1)).reshape(-1, m2)
    wn = np.transpose(w_new, (0, 2, 1)).reshape(-1, m2)
    o = np.transpose(obs, (0, 2, 1)).reshape(-1, m2)
    nrow = wb.shape[0]
    # block-diagonal banded system: unobserved equations keep K's row, observed ones become
    # identity rows with a zero right-hand side (lambda_o = 0), so lambda solves K_uu lambda_u = wb_u
    diag = np.where(o, 1.0, np.broadcast_to(np.diag(kmr), (nrow, m2)))
    lower = np.zeros((nrow, m2))
    upper = np.zeros((nrow, m2))
    if m2 > 1:
        lower[:, 1:] = np.where(o[:, 1:] | o[:, :-1], 0.0, np.array([kmr[j, j - 1] for j in range(1, m2)])[None, :])
        upper[:, :-1] = np.where(o[:, :-1] | o[:, 1:], 0.0, np.array([kmr[j, j + 1] for j in range(m2 - 1)])[None, :])
    rhs = np.where(o, 0.0, wb).reshape(-1)
    n = nrow * m2
    ab = np.zeros((3, n))
    ab[1, :] = diag.reshape(-1)
    ab[0, 1:] = upper.reshape(-1)[:-1]
    ab[2, :-1] = lower.reshape(-1)[1:]
    lam = solve_banded((1, 1), ab, rhs).reshape(nrow, m2)
    lam = np.where(o, 0.0, lam)
    theta_bar.mu += -float(np.sum(lam * wn))
    theta_bar.rho2 += -float(np.sum(lam * (wn @ ktk)))
    return np.transpose(lam.reshape(m1, m3, m2), (0, 2, 1)).copy()


def iterate_adjoint(prob: Problem, st: State, nxt: State, xt_bar: np.ndarray, yt_bar: np.ndarray,
                    w_bar: np.ndarray, theta_bar: ThetaBar):
    """Reverse pass of one iteration st -> nxt (steps 1-4 and 7 of the algorithm box).

    Inputs: adjoints of the outputs X~+ (m1, r, m3), Y~+ (r, m2, m3) complex and W+ (m1, m2,
    m3) real.  Returns the adjoints of the inputs X~, Y~ (complex) and W (real: the state's W,
    through W~ = dft3(W)), and accumulates the weights' adjoints into ``theta_bar``."""
    eta = prob.eta
    x, y, wt = _slices(st.xt), _slices(st.yt), _slices(st.wt)          # (m3, m1, r) etc.
    x1, y1 = _slices(nxt.xt), _slices(nxt.yt)
    hr = prob.hr
    hth = prob.hth
    x1_bar = _slices(xt_bar).copy()
    y1_bar = _slices(yt_bar).copy()
    # step 4 (and 7 of the previous iteration is the caller's W -> W~): W-step adjoint
    z_bar = w_step_adjoint(prob, nxt.w, w_bar, theta_bar)
    # step 3: Z = Re idft3(Z~), Z~_k = X~+_k Y~+_k
    zt_bar = _slices(np.fft.ifft(z_bar, axis=2))
    x1_bar += zt_bar @ _h(y1)
    y1_bar += _h(x1) @ zt_bar
    # step 2: Y~+ = (1 - eta) Y~ + eta R,  R = G_X^{-1} B,  B = X~+^* W~,  G_X = X~+^* H_rho1 X~+
    y_bar = (1.0 - eta) * y1_bar
    r_bar = eta * y1_bar
    gx = _h(x1) @ (hr @ x1)
    gxi = np.linalg.inv(gx)
    b = _h(x1) @ wt
    gxi_bar = r_bar @ _h(b)
    b_bar = _h(gxi) @ r_bar
    gx_bar = -_h(gxi) @ gxi_bar @ _h(gxi)
    x1_bar += wt @ _h(b_bar)
    wt_bar = x1 @ b_bar
    x1_bar += (hr @ x1) @ (gx_bar + _h(gx_bar))
    theta_bar.rho1 += float(np.sum(np.real(np.conj(gx_bar) * (_h(x1) @ (hth @ x1)))))
    # step 1: X~+ = (1 - eta) X~ + eta Q,  Q = H_rho1^{-1} P,  P = A G_Y^{-1},  A = W~ Y~^*,  G_Y = Y~ Y~^*
    x_bar = (1.0 - eta) * x1_bar
    q_bar = eta * x1_bar
    gy = y @ _h(y)
    gyi = np.linalg.inv(gy)
    a = wt @ _h(y)
    p = a @ gyi
    q = np.linalg.solve(hr[None], p)
    p_bar = np.linalg.solve(hr.T[None], q_bar)           # H_rho1 is real symmetric
    theta_bar.rho1 += -float(np.sum(np.real(np.conj(p_bar) * (hth @ q))))
    a_bar = p_bar @ _h(gyi)
    gyi_bar = _h(a) @ p_bar
    gy_bar = -_h(gyi) @ gyi_bar @ _h(gyi)
    wt_bar += a_bar @ y
    y_bar += _h(a_bar) @ wt
    y_bar += (gy_bar + _h(gy_bar)) @ y
    # step 7 of the previous iteration: W~ = dft3(W)
    w_in_bar = np.real(np.fft.fft(_unslices(wt_bar), axis=2))
    return _unslices(x_bar), _unslices(y_bar), w_in_bar


def heldout_rse(w: np.ndarray, m: np.ndarray, hold: np.ndarray) -> float:
    """Relative error on the held-out entries: ||P_H(W - M)||_F / ||P_H(M)||_F."""
    h = hold.astype(bool)
    return float(np.linalg.norm((w - m)[h]) / np.linalg.norm(m[h]))


def heldout_rse_grad(w: np.ndarray, m: np.ndarray, hold: np.ndarray) -> np.ndarray:
    """d heldout_rse / d W."""
    h = hold.astype(bool)
    e = np.where(h, w - m, 0.0)
    return e / (np.linalg.norm(e) * np.linalg.norm(m[h]))


def unrolled_gradients(prob: Problem, x0: np.ndarray, y0: np.ndarray, iters: int, m: np.ndarray,
                       hold: np.ndarray):
    """Held-out RSE after ``iters`` iterations from (X0, Y0, W0 = P_Omega(G)) and its
    gradients with respect to (mu, rho1, rho2) and to the real initial factors X0, Y0.

    Every state is kept (the oracle is for small sizes); returns
    (loss, theta_bar[3], X0_bar, Y0_bar, states)."""
    states = [initial_state(prob, x0, y0)]
    for _ in range(iters):
        states.append(iterate(prob, states[-1]))
    loss = heldout_rse(states[-1].w, m, hold)
    w_bar = heldout_rse_grad(states[-1].w, m, hold)
    xt_bar = np.zeros_like(states[-1].xt)
    yt_bar = np.zeros_like(states[-1].yt)
    tb = ThetaBar()
    for l in range(iters - 1, -1, -1):
        xt_bar, yt_bar, w_bar = iterate_adjoint(prob, states[l], states[l + 1], xt_bar, yt_bar, w_bar, tb)
    # W0 = P_Omega(G) does not depend on the factors or the weights; X~0 = dft3(X0), Y~0 = dft3(Y0)
    x0_bar = np.real(np.fft.fft(xt_bar, axis=2))
    y0_bar = np.real(np.fft.fft(yt_bar, axis=2))
    return loss, tb.as_array(), x0_bar, y0_bar, states


def objective_factor_gradients(prob: Problem, st: State):
    """Gradients of f0 (eq. (TETP-optim)) with respect to the real spatial factors X, Y at the
    state: through eq. (fun-XYW) and eq. (bar BA-k), d f0 / d X = Re idft3(grad_X h) with
    grad_X h_k of eq. (hkXYDer), likewise for Y."""
    from .algorithm import grad_x, grad_y
    m3 = prob.shape[2]
    gx = np.empty_like(st.xt)
    gy = np.empty_like(st.yt)
    for k in range(m3):
        gx[:, :, k] = grad_x(st.xt[:, :, k], st.yt[:, :, k], st.wt[:, :, k], prob.hth, prob.rho1)
        gy[:, :, k] = grad_y(st.xt[:, :, k], st.yt[:, :, k], st.wt[:, :, k], prob.hth, prob.rho1)
    return np.real(idft3(gx)), np.real(idft3(gy))


__all__ = ["ThetaBar", "w_step_adjoint", "iterate_adjoint", "heldout_rse", "heldout_rse_grad",
           "unrolled_gradients", "objective_factor_gradients", "dft3"]

"""Planted mistakes in the oracle (CPU only): each plausible slip must trip at least one pin.

A mutant replaces one oracle function with a wrong variant (dropped term, wrong sign,
wrong conjugation, wrong boundary coefficient, missing preconditioner, wrong DFT root),
then the relevant pins are run; the test passes only if some pin fails.
"""
import numpy as np
import pytest

import oracle as O
import oracle.algorithm as A
import oracle.model as M
import oracle.tensor_algebra as T
import oracle.adjoint as AD
from tests import test_oracle_adjoint as PD
from tests import test_oracle_algebra as PA
from tests import test_oracle_algorithm as PG
from tests import test_oracle_model as PM


def _pins():
    return [
        lambda: PA.test_dft_is_the_written_sum_with_positive_root(5),
        lambda: PA.test_orthogonality_and_block_diagonalisation(4),
        lambda: PA.test_tproduct_fft_equals_block_circulant_definition(3, 2, 4, 5),
        lambda: PM.test_objective_parseval(4, 3, 4, 2),
        lambda: PM.test_objective_terms_by_hand(),
        lambda: PM.test_w_step_banded_kkt_equals_closed_form(4, 6, 3, 0.3, 0.5, 2.0),
        lambda: PM.test_w_step_minimises_g_k_by_brute_force_least_squares(0),
        lambda: PM.test_w_step_rho2_zero_is_shrinkage(),
        lambda: PG.test_pinv_penrose_conditions(5, 2),
        lambda: PG.test_gradients_match_finite_differences(6, 3, 5, 0.7),
        lambda: PG.test_unit_steps_are_exact_block_minimisers(7, 3, 6, 0.5),
        lambda: PG.test_objective_never_increases(1.0, 4),
        lambda: PG.test_unregularised_iteration_is_alternating_least_squares(),
        lambda: PG.test_exact_recovery_in_one_sweep(),
        lambda: PG.test_termination_on_planted_differences(),
        lambda: PG.test_stationarity_normalisation_against_spatial_gradient(4),
        lambda: PG.test_stationarity_normalisation_against_spatial_gradient(5),
        lambda: PD.test_one_iteration_adjoint_matches_finite_differences(0.7, 2),
        lambda: PD.test_unrolled_hypergradients_match_central_differences(1.0),
        lambda: PD.test_w_step_adjoint_without_rho2_is_a_scaling(),
    ]


def _some_pin_fails():
    for pin in _pins():
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError):
            return True
    return False


def _grad_x_no_rho1(xk, yk, wk, hth, rho1):
    return (xk @ yk - wk) @ yk.conj().T


def _grad_y_wrong_sign(xk, yk, wk, hth, rho1):
    xh = xk.conj().T
    return xh @ (xk @ yk + wk) + rho1 * xh @ hth @ xk @ yk


def _grad_x_no_conj(xk, yk, wk, hth, rho1):
    return (xk @ yk - wk) @ yk.T + rho1 * hth @ xk @ yk @ yk.T


def _dft_negative_root(a):
    return np.fft.fft(a, axis=2)


def _idft_negative_root(at):
    return np.fft.ifft(at, axis=2)


def _pinv_no_threshold(g):
    return np.linalg.inv(g + 0 * np.eye(g.shape[0]))


def _kmr_wrong_ends(m2, mu, rho2):
    return (1.0 + mu) * np.eye(m2) + rho2 * (2 * np.eye(m2) - np.eye(m2, k=1) - np.eye(m2, k=-1))


def _x_update_no_precond(prob, xk, yk, wk):
    gy = yk @ yk.conj().T
    gx = A.grad_x(xk, yk, wk, prob.hth, prob.rho1)
    return xk - prob.eta * gx @ A.pinv_h(gy)


def _objective_half_missing(z, w, mu, rho1, rho2):
    m1, m2, _ = z.shape
    h, k = T.toeplitz_diff(m1), T.toeplitz_diff(m2)
    return float(0.5 * np.sum((z - w) ** 2) + 0.5 * mu * np.sum(w ** 2)
                 + 0.5 * rho1 * np.sum((h @ T.unfold(z, 1)) ** 2) + rho2 * np.sum((k @ T.unfold(w, 2)) ** 2))


def _tprod_transposed(a, b):
    at, bt = T.dft3(a), T.dft3(b)
    return T.idft3(np.einsum("irk,rjk->ijk", at, bt[:, :, ::-1])).real


def _termination_real_parts(prev, cur):
    return (float(np.abs((cur.xt - prev.xt).real).max()), float(np.abs((cur.yt - prev.yt).real).max()),
            float(np.linalg.norm(cur.w - prev.w)))


def _termination_w_sup_norm(prev, cur):
    return (float(np.abs(cur.xt - prev.xt).max()), float(np.abs(cur.yt - prev.yt).max()),
            float(np.abs(cur.w - prev.w).max()))


def _stationarity_variant(half_spectrum=False, spatial_w=False):
    def stat(prob, st):
        m3 = prob.shape[2]
        s = 0.0
        for k in range(m3 // 2 + 1 if half_spectrum else m3):   # half spectrum: bin weights dropped
            gx = A.grad_x(st.xt[:, :, k], st.yt[:, :, k], st.wt[:, :, k], prob.hth, prob.rho1)
            gy = A.grad_y(st.xt[:, :, k], st.yt[:, :, k], st.wt[:, :, k], prob.hth, prob.rho1)
            s += np.sum(np.abs(gx) ** 2) + np.sum(np.abs(gy) ** 2)
        wn = np.linalg.norm(st.w) if spatial_w else np.linalg.norm(st.wt)
        denom = wn * (np.linalg.norm(st.xt) + np.linalg.norm(st.yt))
        return {"factor": float(np.sqrt(s) / denom), "w_kkt": 0.0, "w_obs": 0.0}
    return stat


def _transpose_without_conjugate(a):
    return np.swapaxes(a, -1, -2)


def _w_step_adjoint_no_rho2(prob, w_new, w_bar, theta_bar):
    saved = theta_bar.rho2
    out = _W_STEP_ADJOINT(prob, w_new, w_bar, theta_bar)
    theta_bar.rho2 = saved
    return out


def _heldout_grad_unnormalised(w, m, hold):
    h = hold.astype(bool)
    e = np.where(h, w - m, 0.0)
    return e / np.linalg.norm(e)


_W_STEP_ADJOINT = AD.w_step_adjoint

MUTANTS = {
    "grad_x drops the rho1 term": [(A, "grad_x", _grad_x_no_rho1)],
    "grad_y sign of W flipped": [(A, "grad_y", _grad_y_wrong_sign)],
    "grad_x missing conjugate": [(A, "grad_x", _grad_x_no_conj)],
    "DFT with the negative root": [(T, "dft3", _dft_negative_root), (T, "idft3", _idft_negative_root),
                                   (O, "dft3", _dft_negative_root), (O, "idft3", _idft_negative_root)],
    "pseudo-inverse without threshold": [(A, "pinv_h", _pinv_no_threshold), (O, "pinv_h", _pinv_no_threshold)],
    "K_mu_rho2 with interior coefficient at the ends": [(M, "k_mu_rho2", _kmr_wrong_ends)],
    "X-step without H_rho1^-1": [(A, "x_update", _x_update_no_precond), (O, "x_update", _x_update_no_precond)],
    "objective rho2 term without 1/2": [(M, "objective_spatial", _objective_half_missing),
                                        (O, "objective_spatial", _objective_half_missing),
                                        (A, "objective_spatial", _objective_half_missing)],
    "t-product with reversed bins": [(T, "tprod", _tprod_transposed), (O, "tprod", _tprod_transposed)],
    "termination takes the largest real part": [(A, "termination", _termination_real_parts),
                                                (O, "termination", _termination_real_parts)],
    "termination measures W in the sup norm": [(A, "termination", _termination_w_sup_norm),
                                               (O, "termination", _termination_w_sup_norm)],
    "stationarity over the half spectrum without bin weights": [
        (A, "stationarity", _stationarity_variant(half_spectrum=True)),
        (O, "stationarity", _stationarity_variant(half_spectrum=True))],
    "adjoint products without the conjugate": [(AD, "_h", _transpose_without_conjugate)],
    "W-step adjoint drops the rho2 weight's term": [(AD, "w_step_adjoint", _w_step_adjoint_no_rho2)],
    "held-out error gradient without 1 / ||P_H(M)||": [(AD, "heldout_rse_grad", _heldout_grad_unnormalised)],
    "stationarity normalised by the spatial ||W||": [
        (A, "stationarity", _stationarity_variant(spatial_w=True)),
        (O, "stationarity", _stationarity_variant(spatial_w=True))],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    assert not _some_pin_fails(), "pins must pass on the unmodified oracle"
    for mod, attr, fn in MUTANTS[name]:
        monkeypatch.setattr(mod, attr, fn)
    assert _some_pin_fails(), f"no pin caught: {name}"

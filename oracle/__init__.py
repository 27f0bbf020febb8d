"""FP64 CPU oracle of the TCTF2R iteration (Ling, Yu, Qi, Xu, arXiv:2005.09838).

TEST INFRASTRUCTURE.  A plain, slow, FP64 NumPy/SciPy implementation written from the
paper, used only by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg
of ``bench.py``.  It shares no code with the HIP library and the library never imports it.

Modules follow the paper's sections:
* ``tensor_algebra``: section 2 (unfold, bcirc, t-product, the tube DFT and its inverse);
* ``model``: section 3 (objective f0, its Fourier form, the W-step KKT system and closed form);
* ``algorithm``: section 4 (gradients, pseudo-inverse, X/Y updates, one iteration,
  termination and stationarity measures), plus the RSE / NMAE metrics;
* ``adjoint``: hand-written reverse-mode derivatives of one iteration and of K unrolled
  iterations (hypergradients of a held-out error with respect to mu, rho1, rho2 and
  gradients with respect to the initial factors), and the gradient of f0 with respect to
  the spatial factors.

Every function is pinned by ``tests/test_oracle_*.py`` against definitions, closed forms,
invariants and brute force; see the design notes for the list of pins.
"""
from . import adjoint, algorithm, model, tensor_algebra
from .algorithm import (Problem, State, complete, initial_state, iterate, nmae, objective,
                        pinv_h, rank_adjust, rse, stationarity, termination, x_update, y_update, z_of)
from .model import (h_rho1, k_mu_rho2, objective_fourier, objective_spatial, w_kkt_residual,
                    w_step, w_step_closed_form)
from .tensor_algebra import (bcirc, bvec, bvfold, dft3, dft3_by_sum, fold, idft3, toeplitz_diff,
                             tprod, tprod_definition, tubal_rank, unfold, unfold_by_index_map)

__all__ = [
    "adjoint", "algorithm", "model", "tensor_algebra", "Problem", "State", "complete", "initial_state",
    "iterate", "nmae", "objective", "pinv_h", "rank_adjust", "rse", "stationarity", "termination", "x_update",
    "y_update", "z_of", "h_rho1", "k_mu_rho2", "objective_fourier", "objective_spatial",
    "w_kkt_residual", "w_step", "w_step_closed_form", "bcirc", "bvec", "bvfold", "dft3",
    "dft3_by_sum", "fold", "idft3", "toeplitz_diff", "tprod", "tprod_definition", "tubal_rank",
    "unfold", "unfold_by_index_map",
]

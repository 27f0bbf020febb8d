"""Pins of the oracle's section-2 algebra against the paper's definitions (CPU only)."""
import numpy as np
import pytest

import oracle as O
from oracle.tensor_algebra import dft_matrix_normalised, omega

RNG = np.random.default_rng(12345)
SHAPES = [(1, 1, 1), (2, 3, 1), (3, 2, 2), (2, 4, 5), (4, 3, 6), (3, 3, 7)]


@pytest.mark.parametrize("shape", SHAPES)
def test_unfold_index_map_and_block_forms(shape):
    """Section 2.1: the index map, and unfold(A,1) = [A_1..A_m3], unfold(A,2) = [A_1^T..A_m3^T]."""
    a = RNG.normal(size=shape)
    for mode in (1, 2, 3):
        np.testing.assert_array_equal(O.unfold(a, mode), O.unfold_by_index_map(a, mode))
        np.testing.assert_array_equal(O.fold(O.unfold(a, mode), mode, shape), a)
    m3 = shape[2]
    np.testing.assert_array_equal(O.unfold(a, 1), np.concatenate([a[:, :, k] for k in range(m3)], axis=1))
    np.testing.assert_array_equal(O.unfold(a, 2), np.concatenate([a[:, :, k].T for k in range(m3)], axis=1))


@pytest.mark.parametrize("m3", [1, 2, 3, 4, 7, 8])
def test_dft_is_the_written_sum_with_positive_root(m3):
    """eq. (bar BA-k) with omega = exp(+2 pi i/m3), and eq. (barAAk) inverts it."""
    a = RNG.normal(size=(3, 2, m3))
    at = O.dft3(a)
    np.testing.assert_allclose(at, O.dft3_by_sum(a), atol=1e-12)
    # first bin by hand: sum of the slices; second bin (when present) with omega^l
    np.testing.assert_allclose(at[:, :, 0], a.sum(axis=2), atol=1e-12)
    if m3 > 1:
        w = omega(m3)
        np.testing.assert_allclose(at[:, :, 1], sum(w ** l * a[:, :, l] for l in range(m3)), atol=1e-12)
    np.testing.assert_allclose(O.idft3(at), a, atol=1e-12)


@pytest.mark.parametrize("m3", [1, 2, 5, 6])
def test_conjugate_symmetry_of_real_tensors(m3):
    """eq. (rcm_3-k+2): A~_1 real and A~_k = conj(A~_{m3-k+2}); the inverse of such a set is real."""
    a = RNG.normal(size=(2, 3, m3))
    at = O.dft3(a)
    assert np.abs(at[:, :, 0].imag).max() < 1e-12
    for k in range(1, m3):
        np.testing.assert_allclose(at[:, :, k], np.conj(at[:, :, m3 - k]), atol=1e-12)
    assert np.abs(O.idft3(at).imag).max() < 1e-12


@pytest.mark.parametrize("m3", [1, 3, 4, 7])
def test_orthogonality_and_block_diagonalisation(m3):
    """eq. (lsm3) (F_m3 is unitary) and eq. (BDFT): (F (x) I) bcirc(A) (F^* (x) I) = diag(A~_k)."""
    f = dft_matrix_normalised(m3)
    np.testing.assert_allclose(f @ f.conj().T, np.eye(m3), atol=1e-12)
    m1, m2 = 2, 3
    a = RNG.normal(size=(m1, m2, m3))
    lhs = np.kron(f, np.eye(m1)) @ O.bcirc(a) @ np.kron(f.conj().T, np.eye(m2))
    at = O.dft3(a)
    bd = np.zeros_like(lhs)
    for k in range(m3):
        bd[k * m1:(k + 1) * m1, k * m2:(k + 1) * m2] = at[:, :, k]
    np.testing.assert_allclose(lhs, bd, atol=1e-12)
    # ||bcirc(A)||_F = ||A~||_F
    assert np.isclose(np.linalg.norm(O.bcirc(a)), np.linalg.norm(at))


@pytest.mark.parametrize("m1,t,m2,m3", [(1, 1, 1, 1), (2, 3, 2, 4), (3, 2, 4, 5), (4, 1, 3, 7), (2, 2, 2, 2)])
def test_tproduct_fft_equals_block_circulant_definition(m1, t, m2, m3):
    """Definition 2.1 by brute force equals the Fourier-domain product (the t-product pin)."""
    a = RNG.normal(size=(m1, t, m3))
    b = RNG.normal(size=(t, m2, m3))
    np.testing.assert_allclose(O.tprod(a, b), O.tprod_definition(a, b), atol=1e-12)


def test_tproduct_is_circular_convolution_along_the_tube():
    """Definition 2.1 written as sums: C_k = sum_l A_{(k-l) mod m3} B_l."""
    a = RNG.normal(size=(3, 2, 5))
    b = RNG.normal(size=(2, 4, 5))
    c = np.zeros((3, 4, 5))
    for k in range(5):
        for l in range(5):
            c[:, :, k] += a[:, :, (k - l) % 5] @ b[:, :, l]
    np.testing.assert_allclose(O.tprod_definition(a, b), c, atol=1e-12)


def test_tubal_rank_of_products():
    """Proposition 2.3(2): rank_t(A*B) <= min(rank_t(A), rank_t(B))."""
    a = RNG.normal(size=(6, 2, 5))
    b = RNG.normal(size=(2, 7, 5))
    c = O.tprod(a, b)
    assert O.tubal_rank(c) <= 2
    assert O.tubal_rank(RNG.normal(size=(6, 7, 5))) == 6


@pytest.mark.parametrize("m", [1, 2, 3, 5, 10, 40])
def test_difference_matrix_spectrum(m):
    """eq. (Toeplitz) and Proposition KKProp: D^T D is the path Laplacian, lambda_min = 0, lambda_max <= 4."""
    d = O.toeplitz_diff(m)
    assert d.shape == (max(m - 1, 0), m)
    dtd = d.T @ d
    lap = np.zeros((m, m))
    for i in range(m - 1):
        lap[i, i] += 1
        lap[i + 1, i + 1] += 1
        lap[i, i + 1] -= 1
        lap[i + 1, i] -= 1
    np.testing.assert_array_equal(dtd, lap)
    lam = np.linalg.eigvalsh(dtd)
    assert abs(lam[0]) < 1e-12
    assert lam[-1] <= 4 + 1e-12


def test_difference_norm_is_sum_of_adjacent_differences():
    """Below eq. (Toeplitz): ||H unfold(Z,1)||^2 = sum (Z_{i1 i2 i3} - Z_{i1+1, i2, i3})^2."""
    z = RNG.normal(size=(4, 3, 5))
    h = O.toeplitz_diff(4)
    brute = 0.0
    for i1 in range(3):
        for i2 in range(3):
            for i3 in range(5):
                brute += (z[i1, i2, i3] - z[i1 + 1, i2, i3]) ** 2
    assert np.isclose(np.sum((h @ O.unfold(z, 1)) ** 2), brute)
    k = O.toeplitz_diff(3)
    brute2 = sum((z[i1, i2, i3] - z[i1, i2 + 1, i3]) ** 2 for i1 in range(4) for i2 in range(2) for i3 in range(5))
    assert np.isclose(np.sum((k @ O.unfold(z, 2)) ** 2), brute2)

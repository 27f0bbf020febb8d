"""Section 2 of the paper (notation and t-product), written out plainly in FP64.

Part of the FP64 CPU oracle.  Test infrastructure only: nothing in the library's product
path imports this.

Conventions follow section 2: a third-order tensor A has shape (m1, m2, m3); its k-th
frontal slice is A[:, :, k] (paper index k+1); the DFT runs along mode 3 (the tube).
"""
from __future__ import annotations

import numpy as np


def unfold(a: np.ndarray, mode: int) -> np.ndarray:
    """Mode-``mode`` matricisation (section 2.1, 1-based ``mode``).

    Entry (i_1, ..., i_d) goes to row i_k and column j = sum_{l != k} i_l J_l (0-based),
    with J_l the product of the sizes m_t, t < l, t != k.  That is a column-major
    flattening of the remaining indices.
    """
    k = mode - 1
    return np.moveaxis(a, k, 0).reshape(a.shape[k], -1, order="F")


def unfold_by_index_map(a: np.ndarray, mode: int) -> np.ndarray:
    """The same map evaluated entry by entry from the index formula (for tiny tensors)."""
    k = mode - 1
    shape = a.shape
    out = np.zeros((shape[k], a.size // shape[k]), dtype=a.dtype)
    for idx in np.ndindex(*shape):
        j = 0
        for l in range(len(shape)):
            if l == k:
                continue
            jl = 1
            for t in range(l):
                if t != k:
                    jl *= shape[t]
            j += idx[l] * jl
        out[idx[k], j] = a[idx]
    return out


def fold(mat: np.ndarray, mode: int, shape: tuple) -> np.ndarray:
    """Inverse of :func:`unfold`."""
    k = mode - 1
    rest = [shape[l] for l in range(len(shape)) if l != k]
    return np.moveaxis(mat.reshape([shape[k]] + rest, order="F"), 0, k)


def bcirc(a: np.ndarray) -> np.ndarray:
    """Block-circulant matrix of the frontal slices (section 2.2): block (p, q) = A_{(p-q) mod m3}."""
    m1, m2, m3 = a.shape
    out = np.zeros((m1 * m3, m2 * m3), dtype=a.dtype)
    for p in range(m3):
        for q in range(m3):
            out[p * m1:(p + 1) * m1, q * m2:(q + 1) * m2] = a[:, :, (p - q) % m3]
    return out


def bvec(a: np.ndarray) -> np.ndarray:
    """Frontal slices stacked vertically: [A_1; A_2; ...; A_m3] (section 2.2)."""
    m1, m2, m3 = a.shape
    return np.concatenate([a[:, :, k] for k in range(m3)], axis=0)


def bvfold(mat: np.ndarray, m3: int) -> np.ndarray:
    """Inverse of :func:`bvec`."""
    m1 = mat.shape[0] // m3
    return np.stack([mat[k * m1:(k + 1) * m1, :] for k in range(m3)], axis=2)


def tprod_definition(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """t-product by Definition 2.1: bvfold(bcirc(A) . bvec(B))."""
    return bvfold(bcirc(a) @ bvec(b), a.shape[2])


def omega(m3: int) -> complex:
    """The root of unity of section 2.2: exp(+2 pi i / m3)."""
    return np.exp(2j * np.pi / m3)


def dft_matrix_normalised(m3: int) -> np.ndarray:
    """F_{m3}: entries omega^{(p)(q)} / sqrt(m3) (section 2.2)."""
    w = omega(m3)
    idx = np.arange(m3)
    return w ** np.outer(idx, idx) / np.sqrt(m3)


def dft3(a: np.ndarray) -> np.ndarray:
    """Transform of eq. (bar BA-k): A~_k = sum_l omega^{(k-1)(l-1)} A_l, along mode 3.

    With omega = exp(+2 pi i / m3) this is m3 times numpy's inverse FFT.
    """
    return np.fft.ifft(a, axis=2) * a.shape[2]


def idft3(at: np.ndarray) -> np.ndarray:
    """Inverse of eq. (barAAk): A_k = (1/m3) sum_l conj(omega)^{(k-1)(l-1)} A~_l."""
    return np.fft.fft(at, axis=2) / at.shape[2]


def dft3_by_sum(a: np.ndarray) -> np.ndarray:
    """eq. (bar BA-k) evaluated as the written sum (for tiny tensors)."""
    m3 = a.shape[2]
    w = omega(m3)
    out = np.zeros(a.shape, dtype=complex)
    for k in range(m3):
        for l in range(m3):
            out[:, :, k] += w ** (k * l) * a[:, :, l]
    return out


def tprod(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """t-product through the block diagonalisation eq. (BDFT): C~_k = A~_k B~_k.

    Returns the real part after the inverse transform (the result of a t-product of real
    tensors is real, Remark 2.1).
    """
    at, bt = dft3(a), dft3(b)
    ct = np.einsum("irk,rjk->ijk", at, bt)
    c = idft3(ct)
    return c.real


def tubal_rank(a: np.ndarray, rtol: float = 1e-10) -> int:
    """max_k rank(A~_k) (section 2.2, after Definition 2.2)."""
    at = dft3(a)
    ranks = []
    for k in range(a.shape[2]):
        s = np.linalg.svd(at[:, :, k], compute_uv=False)
        ranks.append(int(np.sum(s > rtol * max(s[0], 1e-300))) if s.size else 0)
    return max(ranks) if ranks else 0


def toeplitz_diff(m: int) -> np.ndarray:
    """(m-1) x m matrix Toeplitz(0, 1, -1) of eq. (Toeplitz): ones on the diagonal, -1 above."""
    d = np.zeros((max(m - 1, 0), m))
    for i in range(m - 1):
        d[i, i] = 1.0
        d[i, i + 1] = -1.0
    return d

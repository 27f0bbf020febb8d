"""The oracle against matrices the paper prints (tests/golden/printed_matrices.json)."""
import json
import os

import numpy as np

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_matrices.json")))


def test_difference_matrix_as_printed():
    np.testing.assert_array_equal(O.toeplitz_diff(5), np.array(GOLD["toeplitz_H_m1_5"]["value"]))
    d = O.toeplitz_diff(6)
    np.testing.assert_array_equal(d.T @ d, np.array(GOLD["DtD_m_6"]["value"]))


def test_block_circulant_layout_as_printed():
    m3 = 6
    # slice s (1-based) is the constant matrix s, so each block reveals its slice index
    a = np.stack([np.full((1, 1), float(s + 1)) for s in range(m3)], axis=2)
    np.testing.assert_array_equal(O.bcirc(a), np.array(GOLD["bcirc_slice_index_m3_6"]["value"], dtype=float))

"""CPU pin of the identity behind plans with levels above 2048: a Toeplitz
level of size n = f_1 ... f_m, with its index taken in C order
(i = sum_k i_k w_k, w_k = f_{k+1} ... f_m), is an m-level Toeplitz operator
whose generator at offsets (r_1, ..., r_m) is t(sum_k r_k w_k) (the
multilevel block-Toeplitz structure of the introduction). Brute force on the
oracle's dense operators: the two matrices are equal entry for entry."""

import itertools

import numpy as np
import pytest

import oracle
import workloads as wl


def _gather(coeffs, factors_per_level):
    """Generator of the levels that carry each level's factors (C order)."""
    b = coeffs.shape[0]
    n = oracle.grid_of(coeffs)
    out_n = [f for fs in factors_per_level for f in fs]
    out = np.zeros((b, b) + tuple(2 * f - 1 for f in out_n), dtype=coeffs.dtype)
    for idx in itertools.product(*[range(2 * f - 1) for f in out_n]):
        src = []
        q = 0
        for e, fs in enumerate(factors_per_level):
            r = 0
            for f in fs:
                r = r * f + (idx[q] - (f - 1))  # sum_k r_k w_k, Horner form
                q += 1
            src.append(r + n[e] - 1)
        out[(slice(None), slice(None)) + idx] = coeffs[(slice(None), slice(None)) + tuple(src)]
    return out


@pytest.mark.parametrize("n, factors, b", [
    ((12,), [(3, 4)], 1),
    ((12,), [(4, 3)], 2),
    ((24,), [(2, 3, 4)], 1),
    ((6, 5), [(2, 3), (5,)], 2),
    ((4, 10), [(4,), (5, 2)], 1),
])
def test_long_level_is_a_multilevel_toeplitz_operator(n, factors, b):
    coeffs = wl.iid_coeffs(7, n, b)
    split = _gather(coeffs, factors)
    assert oracle.grid_of(split) == tuple(f for fs in factors for f in fs)
    np.testing.assert_array_equal(oracle.dense_operator(split), oracle.dense_operator(coeffs))


def test_wrong_offset_weight_is_caught():
    # r_1 + r_2 f_1 (the factors' weights swapped) is not the operator
    coeffs = wl.iid_coeffs(8, (12,), 1)
    good = _gather(coeffs, [(3, 4)])
    bad = np.zeros_like(good)
    for i1 in range(5):
        for i2 in range(7):
            r = (i1 - 2) + 3 * (i2 - 3)
            bad[0, 0, i1, i2] = coeffs[0, 0, r + 11]
    assert not np.allclose(oracle.dense_operator(bad), oracle.dense_operator(coeffs))
    np.testing.assert_array_equal(oracle.dense_operator(good), oracle.dense_operator(coeffs))

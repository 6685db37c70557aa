"""Pins of the reference's Gauss-Lobatto tables (closed forms and exactness)."""
import numpy as np
import pytest

import oracle as O


def test_closed_form_nodes_weights():
    x, w, _, _ = O.tables(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w, _, _ = O.tables(3)
    s = 1 / np.sqrt(5)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w, _, _ = O.tables(4)
    s = np.sqrt(3 / 7)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_exactness_and_sbp(k):
    x, w, D, Dh = O.tables(k)
    # quadrature exact to degree 2k-1
    for p in range(2 * k):
        exact = (1 - (-1) ** (p + 1)) / (p + 1)
        assert abs(np.dot(w, x ** p) - exact) < 1e-13
    # and not to degree 2k (Lobatto's defect) for k >= 1
    p = 2 * k
    assert abs(np.dot(w, x ** p) - 2 / (p + 1)) > 1e-6
    # D differentiates polynomials up to degree k exactly
    for p in range(k + 1):
        dp = p * x ** (p - 1) if p > 0 else 0 * x
        assert np.allclose(D @ x ** p, dp, atol=1e-12 * max(1, k ** 2))
    # summation by parts: W D + D^T W = diag(-1, 0, ..., 0, 1)
    W = np.diag(w)
    B = np.zeros((k + 1, k + 1))
    B[0, 0], B[-1, -1] = -1, 1
    assert np.allclose(W @ D + D.T @ W, B, atol=1e-13)
    # weak-form derivative matrix W^-1 D^T W
    assert np.allclose(Dh, np.linalg.inv(W) @ D.T @ W, atol=1e-13)

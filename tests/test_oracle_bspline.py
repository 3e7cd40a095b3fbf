"""Pins of the oracle's B-spline evaluation (Section 2.1) against facts fixed
by the mathematics: partition of unity, derivatives against central finite
differences, the closed-form p=1 hat functions, and the Remark 3.6 matrices."""
import numpy as np
import pytest

from oracle import bspline as bs
from oracle.spacetime import time_matrices


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("n_el", [1, 3, 7])
def test_partition_of_unity_and_nonnegativity(p, n_el):
    kn = bs.open_uniform_knots(0.0, 1.0, n_el, p)
    x = np.linspace(0.0, 1.0, 101)
    N = bs.basis_all(kn, p, x)
    assert N.shape == (101, n_el + p)
    assert np.allclose(N.sum(axis=1), 1.0, atol=1e-14)
    assert N.min() >= -1e-15
    # open knot vector: interpolatory at both ends
    assert N[0, 0] == 1.0 and N[-1, -1] == 1.0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_derivative_matches_finite_differences(p):
    kn = bs.open_uniform_knots(-0.5, 1.5, 5, p)
    x = np.array([-0.31, 0.02, 0.44, 0.97, 1.33])   # away from knots
    h = 1e-6
    fd = (bs.basis_all(kn, p, x + h) - bs.basis_all(kn, p, x - h)) / (2 * h)
    assert np.allclose(bs.basis_all(kn, p, x, 1), fd, atol=1e-7)


def test_degree_one_hat_functions():
    kn = bs.open_uniform_knots(0.0, 1.0, 4, 1)
    x = np.array([0.1, 0.3, 0.55, 0.8])
    N = bs.basis_all(kn, 1, x)
    hat = lambda c, xx: np.maximum(0.0, 1.0 - np.abs(xx - c) / 0.25)
    for i in range(5):
        assert np.allclose(N[:, i], hat(0.25 * i, x), atol=1e-15)


def test_remark_3_6_closed_forms():
    """Remark 3.6: for p=1, theta=0 and a uniform mesh, 2 K_t is the
    tridiagonal (-1, 0, 1) matrix with corners 1, and M_t is a multiple of
    tridiag(1, 4, 1) with corner entries 2 (the multiple is h/6)."""
    n = 6
    K, M = time_matrices(0.0, 1.0, n, 1, 0.0)
    N = n + 1
    K2 = np.zeros((N, N))
    for i in range(N):
        if i > 0:
            K2[i, i - 1] = -1
        if i < N - 1:
            K2[i, i + 1] = 1
    K2[0, 0] = 1
    K2[-1, -1] = 1
    assert np.allclose(2 * K, K2, atol=1e-14)
    T = np.diag([2.0] + [4.0] * (N - 2) + [2.0]) + np.diag(np.ones(N - 1), 1) + np.diag(np.ones(N - 1), -1)
    assert np.allclose(M, T / (6 * n), atol=1e-15)

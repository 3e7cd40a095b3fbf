"""Pins of the oracle's MinRes slab inverse (Section 3.3, Theorems 3.8 and
3.10, Table 3, Section 4.4).

Fixed by the paper or the mathematics, not by the oracle's own formulas:
  * Theorem 3.10 (and 3.8 as the case |beta_1| = |beta_2|): every
    generalised eigenvalue of (A_bar, P) has 1/sqrt(2) <= |lambda| <= 1
    (dense eigenvalues of the assembled matrices);
  * MinRes: the residual estimates decrease monotonically, equal the true
    P^{-1}-norm of the residual, obey the two-interval bound
    2 q^floor(k/2) that follows from the theorem, and reach the direct
    solution;
  * Table 3: the iteration counts to a 1e-10 reduction stay bounded in the
    degree and the mesh (at most 28, the count the bound gives);
  * the temporal block form reconstructs the pencil, K_t X = M_t X Z;
  * the MinRes slab inverse reaches the exact slab inverse (sparse LU of the
    assembled slab matrix), and with the 1e-4 accuracy of Section 4.4 the
    multigrid keeps the cycle count of the exact smoother.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle.mg import MultigridOracle
from oracle.minres import (Q_RATE, MinresSlabInverse, iterations_for, pair_system, pminres,
                           temporal_blocks)
from oracle.solve import SlabSystem
from oracle.spacetime import Problem, assemble_rhs, space_matrices, time_matrices


def _space(dim, ne, p):
    M, K = space_matrices(Problem(dim, ne, p, 1, 1))
    return K, M


@pytest.mark.parametrize("alpha,b1,b2", [(3.0, 2.0, -2.0), (0.5, 7.0, -7.0), (12.0, 0.3, -5.0),
                                         (1.0, -4.0, 0.25), (40.0, 90.0, -1.0)])
def test_theorem_preconditioned_spectrum(alpha, b1, b2):
    K, M = _space(2, 6, 2)
    A, P = pair_system(K, M, alpha, b1, b2)
    lam = sl.eigvals(A.toarray(), P.toarray())
    mod = np.abs(lam)
    assert mod.min() >= 1 / np.sqrt(2) - 1e-10 and mod.max() <= 1 + 1e-10
    assert np.abs(lam.imag).max() <= 1e-8 * mod.max()          # symmetric A_bar, SPD P: real spectrum


def test_iteration_counts_from_the_bound():
    assert iterations_for(1e-4) == 12 and iterations_for(1e-10) == 28
    assert 2 * Q_RATE ** 6 <= 1e-4 < 2 * Q_RATE ** 5


@pytest.mark.parametrize("alpha,b1,b2", [(3.0, 2.0, -2.0), (12.0, 0.3, -5.0)])
def test_minres_history_bound_and_solution(alpha, b1, b2):
    K, M = _space(2, 8, 3)
    A, P = pair_system(K, M, alpha, b1, b2)
    Ad, Pd = A.toarray(), P.toarray()
    b = W.random_vector(3, A.shape[0])
    Pinv = lambda v: np.linalg.solve(Pd, v)
    x, hist = pminres(lambda v: Ad @ v, Pinv, b, 60)
    hist = np.array(hist)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])                        # monotone
    for k in range(1, 40):
        assert hist[k] <= 2 * Q_RATE ** (k // 2) * hist[0] * (1 + 1e-9), k
    for k in (3, 8, 15):
        xk, hk = pminres(lambda v: Ad @ v, Pinv, b, k)
        r = b - Ad @ xk
        assert abs(np.sqrt(r @ Pinv(r)) - hk[-1]) <= 1e-8 * hk[0]          # estimate = true P^-1 norm
    assert np.linalg.norm(x - np.linalg.solve(Ad, b)) <= 1e-10 * np.linalg.norm(x)


def test_table3_counts_bounded_in_degree_and_mesh():
    """MinRes iterations to a 1e-10 reduction for every pair of the temporal
    pencil, theta = 0.1, slab length 0.1, refined uniformly in x and t."""
    counts = {}
    for p in (2, 3, 4):
        for r in range(3):
            ne, net = 2 ** (r + 2), 2 ** r
            K, M = _space(2, ne, p)
            Kt, Mt = time_matrices(0.0, 0.1, net, p, 0.1 * 0.1 / net)
            _, _, blocks = temporal_blocks(Kt, Mt)
            worst = 0
            for blk in blocks:
                if blk[0] != "pair":
                    continue
                A, P = pair_system(K, M, *blk[2:])
                Pd = P.toarray()
                b = W.random_vector(p * 10 + r, A.shape[0])
                _, hist = pminres(lambda v: A @ v, lambda v: np.linalg.solve(Pd, v), b, 60)
                worst = max(worst, next(k for k, h in enumerate(hist) if h <= 1e-10 * hist[0]))
            counts[(p, r)] = worst
    print("max MinRes iterations (p, refinement):", counts)
    vals = [v for v in counts.values() if v > 0]
    assert max(vals) <= 28 and max(vals) - min(vals) <= 10


@pytest.mark.parametrize("p,net", [(2, 2), (3, 2), (2, 1)])
def test_temporal_block_form_reconstructs_pencil(p, net):
    Kt, Mt = time_matrices(0.0, 1 / 16, net, p, 0.01 / 16 / net)
    X, Wm, blocks = temporal_blocks(Kt, Mt)
    Z = np.zeros_like(Kt)
    for blk in blocks:
        c = blk[1]
        if blk[0] == "real":
            Z[c, c] = blk[2]
        else:
            _, _, a, b1, b2 = blk
            Z[c:c + 2, c:c + 2] = [[a, b1], [b2, a]]
    assert np.abs(Kt @ X - Mt @ X @ Z).max() <= 1e-11 * np.abs(Kt).max()
    assert np.abs(Wm @ Mt @ X - np.eye(len(Kt))).max() <= 1e-11


@pytest.mark.parametrize("dim,ne,p,net", [(2, 8, 2, 2), (2, 6, 3, 2), (3, 4, 2, 1)])
def test_minres_slab_inverse_reaches_exact_inverse(dim, ne, p, net):
    prob = Problem(dim, ne, p, 2, net)
    sysm = SlabSystem.assemble(prob)
    M, K = space_matrices(prob)
    Kt, Mt = time_matrices(0.0, prob.tau, net, p, prob.sigma)
    r = W.random_vector(7, sysm.m)
    exact = sysm.lu.solve(r)
    z = MinresSlabInverse(Kt, Mt, K, M, 40).apply(r)
    assert np.linalg.norm(z - exact) <= 1e-10 * np.linalg.norm(exact)
    z12 = MinresSlabInverse(Kt, Mt, K, M, 12).apply(r)
    err = np.linalg.norm(z12 - exact) / np.linalg.norm(exact)
    print(f"12 iterations: relative error {err:.2e}")
    assert err <= 1e-3


@pytest.mark.parametrize("dim,ne,p,S,net", [(2, 8, 2, 8, 2), (2, 10, 3, 16, 2), (3, 4, 2, 4, 2)])
def test_multigrid_with_minres_smoother_keeps_cycle_count(dim, ne, p, S, net):
    prob = Problem(dim, ne, p, S, net)
    f = assemble_rhs(prob, W.random_modes(4, dim))
    exact = MultigridOracle(prob, coarse_slabs=1)
    mg = MultigridOracle(prob, coarse_slabs=1, minres_iters=iterations_for(1e-4))
    ud = exact.levels[0].forward_substitution(f)
    _, it_e, _ = exact.solve(f, rtol=1e-10)
    u, it, _ = mg.solve(f, rtol=1e-10)
    print(f"cycles: exact smoother {it_e}, MinRes smoother {it}")
    assert it <= it_e + 1
    assert np.linalg.norm(u - ud) <= 1e-8 * np.linalg.norm(ud)

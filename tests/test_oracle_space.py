"""Pins of the oracle's coarsening in space (Section 4.4: the multigrid
coarsens in space as well as in time).

Each property is fixed by the mathematics, not by the oracle's own formulas:
  * the interior columns of the spatial prolongation P_x are the two-scale
    coefficients of uniform B-splines, 2^-p binom(p+1, k) (subdivision of
    cardinal B-splines), at fine index 2i - p;
  * P_x reproduces every coarse function pointwise from the fine ones
    (brute force at random points, through the B-spline evaluation only);
  * the Galerkin products P_x^T M_f P_x and P_x^T K_f P_x equal the 1-D mass
    and stiffness matrices assembled by quadrature on the coarse mesh
    (nested spaces, exact quadrature);
  * the space-time Galerkin slab operators of a space-time step equal the
    slab matrices assembled by quadrature for the problem on the halved
    mesh with twice the slab length and the same sigma (theta halved);
  * the schedule follows the stated ratio rule (tau/h^2 halves on a
    space-time step and doubles on a time step);
  * the multigrid with coarsening in space converges to the direct solution
    with cycle counts that stay flat in the mesh size and close to those of
    time-only coarsening (exact counts: parity unpinned, the paper prints
    none for this variant).
"""
from math import comb

import numpy as np
import pytest

import workloads as W
from oracle import bspline as bs
from oracle.mg import MultigridOracle, coarsening_schedule, space_prolongation
from oracle.solve import SlabSystem
from oracle.spacetime import Problem, assemble_rhs, space_matrices_1d

RATIO = 2.0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_space_prolongation_two_scale_coefficients(p):
    nec = 9
    P = space_prolongation(nec, p)
    Nc = nec + p                          # full coarse basis
    for I in range(p, Nc - p):            # coarse functions with simple knots only
        col = np.zeros(P.shape[0])
        for k in range(p + 2):
            col[2 * I - p + k - 1] = comb(p + 1, k) / 2.0 ** p
        assert np.abs(P[:, I - 1] - col).max() <= 1e-13, I


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("nec", [2, 3, 6])
def test_space_prolongation_reproduces_coarse_functions(p, nec):
    if nec + p - 2 < 1:
        pytest.skip("no interior function")
    P = space_prolongation(nec, p)
    x = np.random.default_rng(7).uniform(0.0, 1.0, 200)
    coarse = bs.basis_all(bs.open_uniform_knots(0.0, 1.0, nec, p), p, x)[:, 1:-1]
    fine = bs.basis_all(bs.open_uniform_knots(0.0, 1.0, 2 * nec, p), p, x)
    # the full fine basis: boundary functions must carry no weight
    assert np.abs(fine[:, 1:-1] @ P - coarse).max() <= 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("nec", [2, 5, 8])
def test_space_galerkin_equals_rediscretisation(p, nec):
    if nec + p - 2 < 1:
        pytest.skip("no interior function")
    P = space_prolongation(nec, p)
    Mf, Kf = space_matrices_1d(2 * nec, p)
    Mc, Kc = space_matrices_1d(nec, p)
    assert np.abs(P.T @ Mf @ P - Mc).max() <= 1e-13 * np.abs(Mc).max()
    assert np.abs(P.T @ Kf @ P - Kc).max() <= 1e-12 * np.abs(Kc).max()


@pytest.mark.parametrize("dim,ne,p,S,net", [(2, 8, 2, 4, 2), (2, 6, 3, 2, 1), (3, 4, 2, 2, 2)])
def test_space_time_galerkin_equals_rediscretisation(dim, ne, p, S, net):
    prob = Problem(dim, ne, p, S, net)
    mg = MultigridOracle(prob, coarse_slabs=1, lam_crit=1e-9)
    assert mg.kinds[0] == "xt"
    # halved mesh, slabs twice as long, the same sigma = theta tau / n_et
    coarse = Problem(dim, ne // 2, p, S // 2, net, T=prob.T, theta=prob.theta / 2)
    assert abs(coarse.sigma - prob.sigma) <= 1e-18
    ref = SlabSystem.assemble(coarse)
    A = mg.levels[1].A.toarray()
    assert np.abs(A - ref.A.toarray()).max() <= 1e-12 * np.abs(A).max()
    if S // 2 > 1:
        B = mg.levels[1].B.toarray()
        assert np.abs(B - ref.B.toarray()).max() <= 1e-12 * np.abs(B).max()


def test_schedule_follows_the_ratio_rule():
    # tau/h^2 = 32: space-time steps down to 2 elements (16 -> 8 -> 4 -> 2)
    assert coarsening_schedule(Problem(2, 16, 2, 8, 1), 1, RATIO) == ["xt", "xt", "xt"]
    # tau/h^2 = 1/4: time steps double it to 2, then one space-time step
    assert coarsening_schedule(Problem(2, 8, 2, 16, 1, T=1 / 16), 1, RATIO) == ["t", "t", "t", "xt"]
    # an odd element count stops coarsening in space
    assert coarsening_schedule(Problem(2, 12, 3, 8, 2), 1, RATIO) == ["xt", "xt", "t"]
    # without a ratio: time only; coarse_slabs bounds the depth
    assert coarsening_schedule(Problem(2, 16, 2, 8, 1), 1, None) == ["t", "t", "t"]
    assert coarsening_schedule(Problem(2, 16, 2, 8, 1), 2, RATIO) == ["xt", "xt"]


def test_space_time_multigrid_converges_with_flat_counts():
    counts = []
    for ne in (8, 16, 32):
        for T in (1.0, 1 / 16):
            prob = Problem(2, ne, 2, 16, 1, T=T)
            f = assemble_rhs(prob, W.random_modes(3, 2))
            mg = MultigridOracle(prob, coarse_slabs=1, lam_crit=RATIO)
            u, it, _ = mg.solve(f, rtol=1e-10, maxit=60)
            ud = mg.levels[0].forward_substitution(f)
            assert np.linalg.norm(u - ud) <= 1e-8 * np.linalg.norm(ud)
            _, it_t, _ = MultigridOracle(prob, coarse_slabs=1).solve(f, rtol=1e-10, maxit=60)
            assert it <= it_t + 3, (ne, T, it, it_t)
            counts.append(it)
    assert max(counts) - min(counts) <= 3, counts

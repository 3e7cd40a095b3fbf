"""Pins of the oracle's space-time assembly.

* Kronecker structure (eq. structureAn and the B_n factorisation): the slab
  matrix assembled by (d+1)-D quadrature equals K_t (x) M_x + M_t (x) K_x built
  from 1-D matrices, and B_n = (e_1 e_{N_t}^T) (x) M_x, on tiny grids.
* Lemma 3.1: the quadratic forms of K_t and M_t equal their integral
  expressions for random coefficient vectors.
* Energy identity behind Lemma 2.1: a_h(v,v) = ||v||_dG^2 + the SUPG face
  term, for random v; with theta small this implies coercivity.
* The coarse operator of two-slab coarsening (Galerkin product with the exact
  embedding) equals the rediscretisation on the double-length slab with the
  fine SUPG parameter.
"""
import numpy as np
import pytest

from oracle import bspline as bs
from oracle.spacetime import (Problem, assemble_slab_matrix, assemble_coupling, time_matrices,
                              space_matrices, space_matrices_1d)
from oracle.solve import SlabSystem
from oracle.mg import time_prolongation
from oracle.norms import dg_norm_sq_discrete


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_kronecker_identity(dim, p):
    prob = Problem(dim=dim, n_elem=3, degree=p, n_slabs=3, n_elem_t=2, theta=0.05)
    A = assemble_slab_matrix(prob, 0).toarray()
    Kt, Mt = time_matrices(0.0, prob.tau, prob.n_elem_t, p, prob.sigma)
    Mx, Kx = space_matrices(prob)
    assert np.abs(A - (np.kron(Kt, Mx) + np.kron(Mt, Kx))).max() <= 1e-13 * np.abs(A).max()
    B = assemble_coupling(prob, 1).toarray()
    Nt = np.zeros((prob.N_t, prob.N_t))
    Nt[0, -1] = 1.0
    assert np.abs(B - np.kron(Nt, Mx)).max() <= 1e-14 * np.abs(B).max()
    # every slab of a uniform mesh has the same matrix
    A2 = assemble_slab_matrix(prob, 2).toarray()
    assert np.abs(A2 - A).max() <= 1e-13 * np.abs(A).max()


def test_space_matrices_are_spd_and_banded():
    for p in (2, 3, 4):
        M1, K1 = space_matrices_1d(12, p)
        for X in (M1, K1):
            assert np.allclose(X, X.T, atol=1e-15)
            assert np.linalg.eigvalsh(X).min() > 0
            i, j = np.nonzero(np.abs(X) > 0)
            assert np.abs(i - j).max() == p
        # smallest eigenvalue of the 1-D pencil approximates pi^2
        lam = np.linalg.eigvals(np.linalg.solve(M1, K1)).real.min()
        assert abs(lam - np.pi ** 2) < 2e-2


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("theta", [0.0, 0.01, 0.5])
def test_lemma_3_1_quadratic_forms(p, theta):
    a, b, n_el = 0.3, 0.7, 3
    h = (b - a) / n_el
    sig = theta * h
    K, M = time_matrices(a, b, n_el, p, sig)
    kn = bs.open_uniform_knots(a, b, n_el, p)
    rng = np.random.default_rng(7 + p)
    xs, ws, _ = bs.element_quadrature(kn, p + 4)
    for _ in range(5):
        v = rng.standard_normal(n_el + p)
        val = bs.spline_eval(kn, p, v, xs)
        der = bs.spline_eval(kn, p, v, xs, 1)
        va, vb = bs.spline_eval(kn, p, v, [a])[0], bs.spline_eval(kn, p, v, [b])[0]
        kform = sig * np.sum(ws * der ** 2) + 0.5 * (vb ** 2 + va ** 2)
        mform = np.sum(ws * val ** 2) + 0.5 * sig * (vb ** 2 - va ** 2)
        assert np.isclose(v @ K @ v, kform, rtol=1e-12)
        assert np.isclose(v @ M @ v, mform, rtol=1e-12)


@pytest.mark.parametrize("dim,p", [(1, 2), (2, 1), (2, 2)])
def test_energy_identity_and_coercivity(dim, p):
    prob = Problem(dim=dim, n_elem=3, degree=p, n_slabs=3, n_elem_t=2, theta=0.01)
    sysm = SlabSystem.assemble(prob)
    L = sysm.dense()
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(prob.n_dof)
        dg, supg = dg_norm_sq_discrete(prob, v)
        assert np.isclose(v @ L @ v, dg + supg, rtol=1e-11)
        assert v @ L @ v >= 0.5 * dg          # Lemma 2.1 (theta small)


@pytest.mark.parametrize("p,n_el", [(1, 2), (2, 2), (3, 2), (2, 1), (4, 2), (2, 3)])
def test_galerkin_coarse_operator_is_rediscretisation(p, n_el):
    tau, theta = 0.125, 0.01
    sig = theta * tau / n_el
    K, M = time_matrices(0.0, tau, n_el, p, sig)
    Nt = np.zeros_like(K)
    Nt[0, -1] = 1.0
    P = time_prolongation(tau, n_el, p)
    Z = np.zeros_like(K)
    Kc = P.T @ np.block([[K, Z], [-Nt, K]]) @ P
    Mc = P.T @ np.block([[M, Z], [Z, M]]) @ P
    Ec = P.T @ np.block([[Z, Nt], [Z, Z]]) @ P
    Kr, Mr = time_matrices(0.0, 2 * tau, n_el, p, sig)      # fine sigma kept
    assert np.allclose(Kc, Kr, atol=1e-13)
    assert np.allclose(Mc, Mr, atol=1e-14)
    assert np.allclose(Ec, Nt, atol=1e-14)


def test_prolongation_reproduces_coarse_functions():
    tau, n_el, p = 0.2, 3, 3
    P = time_prolongation(tau, n_el, p)
    coarse = bs.open_uniform_knots(0.0, 2 * tau, n_el, p)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(n_el + p)
    for k, (a, b) in enumerate([(0.0, tau), (tau, 2 * tau)]):
        fine = bs.open_uniform_knots(a, b, n_el, p)
        x = np.linspace(a + 1e-3, b - 1e-3, 17)
        cf = (P @ c)[k * (n_el + p):(k + 1) * (n_el + p)]
        assert np.allclose(bs.spline_eval(fine, p, cf, x), bs.spline_eval(coarse, p, c, x), atol=1e-13)

"""Pins of the oracle's direct solve and multigrid.

* Slab-wise forward substitution (eq. equ_linear_system) equals a dense solve
  of the whole L_h on tiny problems.
* Manufactured solution u = prod sin(pi x_a) sin(pi t): the dG-norm error
  decreases with order p when h_x = 2 h_t is halved (Theorem 2.3 and
  Remark 2.4); the L2 order (p+1 observed) is reported only.
* Multigrid (Section 3.1): the iterates converge to the direct solution and
  the iteration count to 1e-8 is flat in the spatial mesh and in the number
  of slabs (the paper's Table 4 shows a constant count; the exact count with
  time-only coarsening is not pinned by the paper).
"""
import numpy as np
import pytest

from oracle.spacetime import Problem, assemble_rhs
from oracle.solve import SlabSystem
from oracle.mg import MultigridOracle
from oracle.norms import errors, ExactSolution
import workloads as W


@pytest.mark.parametrize("dim,p,S", [(1, 2, 3), (2, 1, 2), (2, 2, 3), (3, 1, 2)])
def test_forward_substitution_equals_dense_solve(dim, p, S):
    prob = Problem(dim=dim, n_elem=3, degree=p, n_slabs=S, n_elem_t=2, theta=0.01)
    sysm = SlabSystem.assemble(prob)
    f = assemble_rhs(prob, W.random_modes(5, dim))
    u = sysm.forward_substitution(f)
    ud = np.linalg.solve(sysm.dense(), f)
    assert np.linalg.norm(u - ud) <= 1e-12 * np.linalg.norm(ud)
    assert np.linalg.norm(sysm.apply(u) - f) <= 1e-12 * np.linalg.norm(f)


def test_separable_rhs_matches_tensor_quadrature():
    """The load vector of a separable f equals the product of 1-D load
    vectors (time and each axis), computed here independently."""
    from oracle import bspline as bs
    prob = Problem(dim=2, n_elem=4, degree=2, n_slabs=2, n_elem_t=2)
    modes = W.random_modes(11, 2, n_modes=2)
    f = assemble_rhs(prob, modes)
    amp, k, om, ph = modes.arrays()
    q = prob.degree + 3
    kx = bs.open_uniform_knots(0, 1, prob.n_elem, prob.degree)
    xs, wx, _ = bs.element_quadrature(kx, q)
    Nx = bs.basis_all(kx, prob.degree, xs)[:, 1:-1]
    out = []
    for s in range(prob.n_slabs):
        kt = bs.open_uniform_knots(s * prob.tau, (s + 1) * prob.tau, prob.n_elem_t, prob.degree)
        ts, wt, _ = bs.element_quadrature(kt, q)
        test = bs.basis_all(kt, prob.degree, ts) + prob.sigma * bs.basis_all(kt, prob.degree, ts, 1)
        vec = 0
        for m in range(len(amp)):
            lt = (wt * np.cos(om[m] * np.pi * ts + ph[m])) @ test
            lx = (wx * np.sin(k[m, 0] * np.pi * xs)) @ Nx
            ly = (wx * np.sin(k[m, 1] * np.pi * xs)) @ Nx
            vec = vec + amp[m] * np.einsum("t,y,x->tyx", lt, ly, lx).ravel()
        out.append(vec)
    assert np.allclose(f, np.concatenate(out), rtol=1e-12, atol=1e-15)


def _dg_error(dim, p, ne):
    prob = Problem(dim=dim, n_elem=ne, degree=p, n_slabs=ne, n_elem_t=2, theta=0.01)
    f = assemble_rhs(prob, W.manufactured_modes(dim))
    u = SlabSystem.assemble(prob).forward_substitution(f)
    return errors(prob, u, ExactSolution(*W.manufactured_exact(dim)))


@pytest.mark.parametrize("dim,p,levels", [(1, 1, (8, 16, 32)), (1, 2, (8, 16, 32)), (1, 3, (4, 8, 16)),
                                          (2, 1, (4, 8, 16)), (2, 2, (4, 8, 16))])
def test_manufactured_dg_convergence_order(dim, p, levels):
    errs = [_dg_error(dim, p, ne) for ne in levels]
    rate_dg = np.log2(errs[-2]["dG"] / errs[-1]["dG"])
    rate_l2 = np.log2(errs[-2]["L2"] / errs[-1]["L2"])
    print(f"dim={dim} p={p} dG order {rate_dg:.3f} L2 order {rate_l2:.3f}")
    assert rate_dg >= p - 0.15
    assert errs[-1]["dG"] < errs[0]["dG"]


def test_mg_converges_to_direct_solution():
    prob = Problem(dim=2, n_elem=8, degree=2, n_slabs=8, n_elem_t=2)
    f = assemble_rhs(prob, W.random_modes(3, 2))
    mg = MultigridOracle(prob)
    u, it, hist = mg.solve(f, rtol=1e-13, maxit=60)
    ud = mg.levels[0].forward_substitution(f)
    assert hist[-1] <= 1e-13
    assert np.linalg.norm(u - ud) <= 1e-11 * np.linalg.norm(ud)
    # geometric convergence
    assert all(h1 < 0.5 * h0 for h0, h1 in zip(hist[:-1], hist[1:]))


def test_mg_iteration_counts_flat_in_h_and_slabs():
    counts = {}
    for ne in (8, 16):
        for S in (8, 16, 32):
            prob = Problem(dim=2, n_elem=ne, degree=2, n_slabs=S, n_elem_t=2)
            f = assemble_rhs(prob, W.random_modes(1, 2))
            _, it, _ = MultigridOracle(prob).solve(f, rtol=1e-8)
            counts[(ne, S)] = it
    print(counts)
    assert max(counts.values()) - min(counts.values()) <= 2
    assert max(counts.values()) <= 15


def test_mg_iteration_counts_flat_down_to_small_tau_over_h2():
    """Time-only coarsening keeps its count where the slab width is small next
    to the squared mesh size: tau/h^2 from 8 down to 1/16 (the serving mix
    reaches 2).  The space-time multigrid of Section 3.1 also coarsens in
    space; these counts show that the time-only hierarchy does not need it
    on these shapes (Section 4.4, Table 4: counts independent of the number of
    slabs)."""
    counts = {}
    for ne, S in ((8, 8), (8, 64), (8, 128), (4, 64), (4, 256)):
        prob = Problem(dim=2, n_elem=ne, degree=2, n_slabs=S, n_elem_t=2)
        f = assemble_rhs(prob, W.random_modes(1, 2))
        _, it, _ = MultigridOracle(prob).solve(f, rtol=1e-8)
        counts[ne * ne / S] = it
    print(counts)
    assert max(counts.values()) - min(counts.values()) <= 2
    assert max(counts.values()) <= 15

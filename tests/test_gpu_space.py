"""GPU parity of the multigrid with coarsening in space (Section 4.4) against
the FP64 oracle, through the C ABI.

The library stops the levels of a spatial mesh at the first space-time
step and hands the levels below to the problem on the halved mesh; the
oracle forms every coarse operator as a Galerkin product.  Compared, at the
same ratio rule (space_ratio 2):
  * the schedule (spatial elements and slabs per level);
  * the space-time transfers at every space-time step, 1e-13;
  * V-cycle iterates, 1e-10 relative to the largest entry;
  * solves to rtol 1e-12 against the direct solution, 1e-10, with the
    oracle's cycle count (+-1);
  * FGMRES with the space-time cycle as preconditioner, 1e-10.
Shapes: all space-time steps down to two elements, time steps first, a
space-time step between time steps, an odd element count that stops the
coarsening in space, and 3-D.
"""
import functools
import sys

import numpy as np
import pytest

import workloads as W
from oracle.mg import MultigridOracle
from oracle.spacetime import Problem as OProblem, assemble_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RATIO = 2.0
SHAPES = {
    "2d_XXX": dict(dim=2, n_elem=16, degree=2, n_slabs=8, n_elem_t=1, T=1.0, coarse_slabs=1),
    "2d_tttX": dict(dim=2, n_elem=8, degree=2, n_slabs=16, n_elem_t=1, T=1 / 16, coarse_slabs=1),
    "2d_tXt": dict(dim=2, n_elem=8, degree=2, n_slabs=8, n_elem_t=2, T=1 / 8, coarse_slabs=1),
    "2d_ttXt": dict(dim=2, n_elem=16, degree=2, n_slabs=16, n_elem_t=1, T=1 / 32, coarse_slabs=1),
    "2d_p3_XXt": dict(dim=2, n_elem=12, degree=3, n_slabs=8, n_elem_t=2, T=1.0, coarse_slabs=1),
    "3d_XXt": dict(dim=3, n_elem=8, degree=2, n_slabs=8, n_elem_t=1, T=1.0, coarse_slabs=1),
    "3d_Xt": dict(dim=3, n_elem=8, degree=2, n_slabs=8, n_elem_t=2, T=0.3, coarse_slabs=2),
}


def _oshape(name):
    return {k: v for k, v in SHAPES[name].items() if k != "coarse_slabs"}


@functools.lru_cache(maxsize=None)
def oracle_for(name):
    prob = OProblem(**_oshape(name))
    return prob, MultigridOracle(prob, coarse_slabs=SHAPES[name]["coarse_slabs"], lam_crit=RATIO)


@functools.lru_cache(maxsize=None)
def solver_for(name):
    import paper_1802_09277_amd as sth
    return sth.Solver(**SHAPES[name], space_ratio=RATIO)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def banner(name, what):
    print(f"[gpu-space] {what} shape={name} {SHAPES[name]}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(SHAPES))
def test_schedule_matches_oracle(name):
    banner(name, "schedule")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    assert s.num_levels == len(mg.levels)
    for lvl, lev in enumerate(mg.levels):
        assert s.level_elems(lvl) == mg.n_elem[lvl], lvl
        assert s.level_len(lvl) == lev.S * lev.m, lvl
    assert "xt" in mg.kinds


@pytest.mark.parametrize("name", list(SHAPES))
def test_space_time_transfers(name):
    banner(name, "transfers")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    for lvl, kind in enumerate(mg.kinds):
        r = W.random_vector(30 + lvl, s.level_len(lvl))
        rc = s.new_vector(lvl + 1)
        s.restrict(lvl, dev(r), rc)
        assert rel_max(host(rc), mg.restrict(lvl, r)) <= 1e-13, (lvl, kind)
        e = W.random_vector(40 + lvl, s.level_len(lvl + 1))
        u0 = W.random_vector(50 + lvl, s.level_len(lvl))
        u = dev(u0)
        s.prolong_add(lvl, dev(e), u)
        assert rel_max(host(u), u0 + mg.prolong(lvl, e)) <= 1e-13, (lvl, kind)


@pytest.mark.parametrize("name", list(SHAPES))
def test_space_time_vcycle_iterates(name):
    banner(name, "vcycle")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    f = assemble_rhs(prob, W.random_modes(3, prob.dim))
    u = s.new_vector()
    fd = dev(f)
    uo = np.zeros_like(f)
    for k in range(3):
        s.vcycle(fd, u)
        uo = mg.vcycle(f, uo)
        assert rel_max(host(u), uo) <= 1e-10, k


@pytest.mark.parametrize("name", list(SHAPES))
def test_space_time_solve_matches_direct(name):
    banner(name, "solve")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    f = assemble_rhs(prob, W.random_modes(5, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    u = s.new_vector()
    it, rr, _ = s.solve(dev(f), u, rtol=1e-12, maxit=80)
    print(f"  iterations {it} relres {rr:.3e} schedule {mg.kinds}")
    assert rr <= 1e-12
    assert np.linalg.norm(host(u) - ud) <= 1e-10 * np.linalg.norm(ud)
    _, it_o, _ = mg.solve(f, rtol=1e-12, maxit=80)
    assert abs(it - it_o) <= 1


@pytest.mark.parametrize("name", ["2d_ttXt", "3d_XXt"])
def test_space_time_fgmres(name):
    banner(name, "fgmres")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    f = assemble_rhs(prob, W.random_modes(6, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    u = s.new_vector()
    it, rr, _ = s.solve_fgmres(dev(f), u, rtol=1e-12, maxit=60, restart=20)
    print(f"  FGMRES iterations {it} relres {rr:.3e}")
    assert rr <= 1e-12
    assert np.linalg.norm(host(u) - ud) <= 1e-10 * np.linalg.norm(ud)

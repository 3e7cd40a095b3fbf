"""Multigrid as a preconditioner: flexible GMRES(m) right-preconditioned by
one V-cycle (sth_solve_fgmres), in both iteration bases.  The solution must
match the oracle's direct solve; with the V-cycle as preconditioner the
Krylov loop needs no more iterations than the stationary multigrid itself
(the exact counts are not pinned by the paper)."""
import numpy as np
import pytest

import workloads as W
from oracle.spacetime import Problem as OProblem, assemble_rhs
from oracle.mg import MultigridOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = {
    "2d_p2": dict(dim=2, n_elem=6, degree=2, n_slabs=4, n_elem_t=2, coarse_slabs=1),
    "2d_ragged_p3": dict(dim=2, n_elem=37, degree=3, n_slabs=6, n_elem_t=2, coarse_slabs=1),
    "2d_16slabs": dict(dim=2, n_elem=12, degree=2, n_slabs=16, n_elem_t=2, coarse_slabs=4),
    "3d_8slabs": dict(dim=3, n_elem=7, degree=2, n_slabs=8, n_elem_t=2, coarse_slabs=2),
    "2d_n98_axiswise": dict(dim=2, n_elem=98, degree=2, n_slabs=2, n_elem_t=2, coarse_slabs=1),
}
_ORACLES = {}


def oracle_for(name):
    if name not in _ORACLES:
        kw = {k: v for k, v in SHAPES[name].items() if k != "coarse_slabs"}
        prob = OProblem(**kw)
        _ORACLES[name] = (prob, MultigridOracle(prob, coarse_slabs=SHAPES[name]["coarse_slabs"]))
    return _ORACLES[name]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("basis", ["nodal", "eigen"])
def test_fgmres_matches_direct(name, basis):
    import paper_1802_09277_amd as sth
    print(f"[gpu-krylov] fgmres {basis} shape={name} {SHAPES[name]}", flush=True)
    prob, mg = oracle_for(name)
    f = assemble_rhs(prob, W.random_modes(9, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    s = sth.Solver(**SHAPES[name], basis=basis)
    fd = dev(f)
    u = s.new_vector()
    it, rr, _ = s.solve_fgmres(fd, u, rtol=1e-12, maxit=60, restart=20)
    u_mg = s.new_vector()
    it_mg, _, _ = s.solve(fd, u_mg, rtol=1e-12, maxit=60)
    torch.cuda.synchronize()
    err = np.linalg.norm(u.cpu().numpy() - ud) / np.linalg.norm(ud)
    print(f"  fgmres {it} iterations (multigrid {it_mg}), relres {rr:.2e}, error vs direct {err:.2e}")
    assert rr <= 1e-12 and err <= 1e-10
    assert it <= it_mg
    s.close()


def test_fgmres_short_restart_and_nonconvergence():
    import paper_1802_09277_amd as sth
    print("[gpu-krylov] restart 2 / maxit", flush=True)
    prob, mg = oracle_for("2d_16slabs")
    f = assemble_rhs(prob, W.random_modes(10, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    s = sth.Solver(**SHAPES["2d_16slabs"], basis="eigen")
    u = s.new_vector()
    it, rr, _ = s.solve_fgmres(dev(f), u, rtol=1e-11, maxit=80, restart=2)
    torch.cuda.synchronize()
    assert rr <= 1e-11
    assert np.linalg.norm(u.cpu().numpy() - ud) <= 1e-9 * np.linalg.norm(ud)
    u = s.new_vector()
    it, rr, code = s.solve_fgmres(dev(f), u, rtol=1e-14, maxit=2, restart=5, check=False)
    assert code == -6 and it == 2
    with pytest.raises(sth.StatusError):
        s.solve_fgmres(dev(f), u, restart=40)
    s.close()

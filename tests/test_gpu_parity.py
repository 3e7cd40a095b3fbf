"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Element-wise comparisons on seeded inputs.  Tolerances (relative to the
largest entry of the oracle result unless noted):
  load vector 1e-13, L_h u and residual 1e-12, one slab inverse D^{-1} r
  1e-11, smoothing steps 1e-11, transfers 1e-13, V-cycle iterates 1e-10,
  solve to rtol 1e-12 against the direct solution 1e-10.
The shapes span several residual and MFMA tiles with ragged tails, an odd
coarsest level (forward substitution), N_t from 3 to 6 and d = 2, 3.
"""
import functools
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle.spacetime import Problem as OProblem, assemble_rhs
from oracle.solve import SlabSystem
from oracle.mg import MultigridOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = {
    "2d_p2": dict(dim=2, n_elem=6, degree=2, n_slabs=4, n_elem_t=2, coarse_slabs=1),
    "2d_ragged_p3": dict(dim=2, n_elem=37, degree=3, n_slabs=6, n_elem_t=2, coarse_slabs=1),
    "2d_p1_net3": dict(dim=2, n_elem=20, degree=1, n_slabs=8, n_elem_t=3, coarse_slabs=2),
    "2d_p4": dict(dim=2, n_elem=14, degree=4, n_slabs=2, n_elem_t=2, coarse_slabs=1),
    "2d_16slabs": dict(dim=2, n_elem=12, degree=2, n_slabs=16, n_elem_t=2, coarse_slabs=4),
    "3d_p2": dict(dim=3, n_elem=9, degree=2, n_slabs=4, n_elem_t=2, coarse_slabs=4),
    "3d_p3": dict(dim=3, n_elem=6, degree=3, n_slabs=2, n_elem_t=1, coarse_slabs=1),
    "3d_8slabs": dict(dim=3, n_elem=7, degree=2, n_slabs=8, n_elem_t=2, coarse_slabs=2),
    # n = 98 > 96: the two-kernel (per-axis) transform path of large images
    "2d_n98_axiswise": dict(dim=2, n_elem=98, degree=2, n_slabs=2, n_elem_t=2, coarse_slabs=1),
    # five levels (32 -> 16 -> 8 -> 4 -> 2 slabs; 100 modes padded to 112 per
    # time row): the coarse-level descent and post-smoothing passes of levels
    # 1 and 2 and the two-level coarse pass, as the large workloads run them
    "2d_5lev": dict(dim=2, n_elem=10, degree=2, n_slabs=32, n_elem_t=1, coarse_slabs=2),
    # five levels in 3-D down to a single slab (16 -> 8 -> 4 -> 2 -> 1)
    "3d_5lev": dict(dim=3, n_elem=6, degree=2, n_slabs=16, n_elem_t=2, coarse_slabs=1),
    # n = 113 (np = 128): the per-axis transforms with the transform matrix in
    # LDS (two 64-column panels in FP64), a ragged last tile of k and rows
    "2d_n113_panel": dict(dim=2, n_elem=113, degree=2, n_slabs=2, n_elem_t=1, coarse_slabs=1),
    # 1024 -> 512 -> 256 slabs, N_t = 3: the two coarsest levels in one pass
    # with 64 slab groups of 8 level-a slabs (1024-thread blocks)
    "2d_wide_tail": dict(dim=2, n_elem=4, degree=1, n_slabs=1024, n_elem_t=2, coarse_slabs=256),
    # 1024 -> 512 -> 256 -> 128 slabs, N_t = 3 (the level structure of the
    # large 2-D workload): the three coarsest levels in one pass, 64 groups
    "2d_wide_tail3": dict(dim=2, n_elem=4, degree=1, n_slabs=1024, n_elem_t=2, coarse_slabs=128),
    # 64 -> 32 -> 16 -> 8 slabs, N_t = 5: the three-level pass with 8 groups
    # of 4 level-a slabs
    "2d_p3_tail3": dict(dim=2, n_elem=6, degree=3, n_slabs=64, n_elem_t=2, coarse_slabs=8),
}


def _shape(name):
    return {k: v for k, v in SHAPES[name].items() if k != "coarse_slabs"}


@functools.lru_cache(maxsize=None)
def oracle_for(name):
    prob = OProblem(**_shape(name))
    mg = MultigridOracle(prob, coarse_slabs=SHAPES[name]["coarse_slabs"])
    return prob, mg


@functools.lru_cache(maxsize=None)
def solver_for(name):
    import paper_1802_09277_amd as sth
    return sth.Solver(**SHAPES[name])


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def last_error():
    import paper_1802_09277_amd as sth
    msg = sth.load_library().sth_last_error()
    return msg.decode() if msg else ""


def banner(name, what):
    print(f"[gpu-parity] {what} shape={name} {SHAPES[name]}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(SHAPES))
def test_rhs_load(name):
    banner(name, "rhs")
    prob, _ = oracle_for(name)
    s = solver_for(name)
    modes = W.random_modes(2, prob.dim)
    f = s.new_vector()
    s.load_rhs(modes, f)
    assert rel_max(host(f), assemble_rhs(prob, modes)) <= 1e-13


@pytest.mark.parametrize("name", list(SHAPES))
def test_apply_and_residual(name):
    banner(name, "apply/residual")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    u = W.random_vector(10, prob.n_dof)
    f = W.random_vector(11, prob.n_dof)
    y = s.new_vector()
    s.apply(dev(u), y)
    ref = mg.levels[0].apply(u)
    assert rel_max(host(y), ref) <= 1e-12
    r = s.new_vector()
    s.residual(dev(f), dev(u), r)
    assert rel_max(host(r), f - ref) <= 1e-12


@pytest.mark.parametrize("name", list(SHAPES))
def test_block_solve(name):
    banner(name, "block_solve")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    r = W.random_vector(12, prob.n_dof)
    z = s.new_vector()
    s.block_solve(dev(r), z)
    assert rel_max(host(z), mg.levels[0].slab_solve(r)) <= 1e-11


@pytest.mark.parametrize("name", list(SHAPES))
def test_smoothing_steps(name):
    banner(name, "smooth")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    f = W.random_vector(13, prob.n_dof)
    u0 = W.random_vector(14, prob.n_dof)
    u = dev(u0)
    s.smooth(dev(f), u, steps=2)
    assert rel_max(host(u), mg.smooth(0, f, u0, 2)) <= 1e-11


@pytest.mark.parametrize("name", [n for n in SHAPES if SHAPES[n]["n_slabs"] > SHAPES[n]["coarse_slabs"]])
def test_transfers(name):
    banner(name, "transfers")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    r = W.random_vector(15, prob.n_dof)
    rc = s.new_vector(1)
    s.restrict(0, dev(r), rc)
    assert rel_max(host(rc), mg.restrict(0, r)) <= 1e-13
    e = W.random_vector(16, s.level_len(1))
    u0 = W.random_vector(17, prob.n_dof)
    u = dev(u0)
    s.prolong_add(0, dev(e), u)
    assert rel_max(host(u), u0 + mg.prolong(0, e)) <= 1e-13


@pytest.mark.parametrize("name", list(SHAPES))
def test_vcycle_iterates(name):
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
def test_solve_matches_direct(name):
    banner(name, "solve")
    prob, mg = oracle_for(name)
    s = solver_for(name)
    f = assemble_rhs(prob, W.random_modes(5, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    u = s.new_vector()
    it, rr, _ = s.solve(dev(f), u, rtol=1e-12, maxit=60)
    print(f"  iterations {it} relres {rr:.3e}")
    assert rr <= 1e-12
    err = np.linalg.norm(host(u) - ud) / np.linalg.norm(ud)
    assert err <= 1e-10
    # iteration count equals the oracle multigrid's
    _, it_o, _ = mg.solve(f, rtol=1e-12, maxit=60)
    assert abs(it - it_o) <= 1


def test_solve_reports_nonconvergence():
    import paper_1802_09277_amd as sth
    name = "2d_p2"
    banner(name, "enoconv")
    prob, _ = oracle_for(name)
    s = solver_for(name)
    f = W.random_vector(20, prob.n_dof)
    u = s.new_vector()
    it, rr, code = s.solve(dev(f), u, rtol=1e-30, maxit=2, check=False)
    assert code == -6 and it == 2
    f[7] = np.nan
    u = s.new_vector()
    it, rr, code = s.solve(dev(f), u, rtol=1e-8, maxit=5, check=False)
    assert code == -6 and it <= 1


@pytest.mark.parametrize("basis", ["nodal", "eigen"])
def test_graph_replay_matches_eager_solve(basis):
    """Solve on a non-default stream (graph replay of the iterations) gives
    bit-identical iterates to the eager launches.  In the eigenbasis the
    fused cycle close alternates its finest-level buffers, so the replays
    cycle through two cached graphs."""
    name = "2d_16slabs"
    banner(name, f"graph {basis}")
    prob, mg = oracle_for(name)
    s = solver_for(name) if basis == "nodal" else eigen_solver_for(name)
    f = dev(assemble_rhs(prob, W.random_modes(8, prob.dim)))
    stream = torch.cuda.Stream()
    results = []
    for graphs in (False, True, True):
        s.use_graphs(graphs)
        with torch.cuda.stream(stream):
            u = s.new_vector()
            it, rr, _ = s.solve(f, u, rtol=1e-11, maxit=60, stream=stream)
        stream.synchronize()
        results.append((it, rr, host(u)))
    s.use_graphs(False)
    assert results[0][0] == results[1][0] == results[2][0]
    assert np.array_equal(results[0][2], results[1][2])
    assert np.array_equal(results[1][2], results[2][2])


@functools.lru_cache(maxsize=None)
def eigen_solver_for(name):
    import paper_1802_09277_amd as sth
    return sth.Solver(**SHAPES[name], basis="eigen")


@pytest.mark.parametrize("name", list(SHAPES))
def test_eigenbasis_iterates_match_oracle_cycles(name):
    """Iterating in the spatial eigenbasis gives the multigrid iterates of the
    oracle (k cycles from zero, mapped back to B-spline coefficients), both on
    the default stream and with graph replay on a side stream."""
    banner(name, "eigenbasis")
    prob, mg = oracle_for(name)
    s = eigen_solver_for(name)
    f = assemble_rhs(prob, W.random_modes(3, prob.dim))
    fd = dev(f)
    uo = np.zeros_like(f)
    for k in range(1, 4):
        uo = mg.vcycle(f, uo)
        u = s.new_vector()
        it, rr, code = s.solve(fd, u, rtol=0.0, maxit=k, check=False)
        assert (it, code) == (k, -6), last_error()
        assert rel_max(host(u), uo) <= 1e-10, k
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        u = s.new_vector()
        it, rr, code = s.solve(fd, u, rtol=0.0, maxit=3, check=False, stream=stream)
    stream.synchronize()
    assert (it, code) == (3, -6), last_error()
    assert rel_max(host(u), uo) <= 1e-10


@pytest.mark.parametrize("name", list(SHAPES))
def test_eigenbasis_solve_matches_direct(name):
    banner(name, "eigenbasis solve")
    prob, mg = oracle_for(name)
    s = eigen_solver_for(name)
    f = assemble_rhs(prob, W.random_modes(5, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    u = s.new_vector()
    it, rr, _ = s.solve(dev(f), u, rtol=1e-12, maxit=60)
    _, it_o, _ = mg.solve(f, rtol=1e-12, maxit=60)
    print(f"  eigenbasis: {it} cycles (oracle {it_o}), relres {rr:.2e}")
    assert rr <= 1e-12 and abs(it - it_o) <= 1
    assert np.linalg.norm(host(u) - ud) <= 1e-10 * np.linalg.norm(ud)


# ---------------------------------------------------------------------------
# Real Schur form of the temporal pencil (orthogonal temporal transforms and a
# block back substitution per spatial mode, the Schur alternative of Section
# 3.3): the same slab inverse and the same solution as the oracle.
# ---------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def schur_solver_for(name, basis):
    import paper_1802_09277_amd as sth
    return sth.Solver(**SHAPES[name], temporal="schur", basis=basis)


@pytest.mark.parametrize("name", list(SHAPES))
def test_schur_block_solve(name):
    banner(name, "schur block_solve")
    prob, mg = oracle_for(name)
    s = schur_solver_for(name, "nodal")
    r = W.random_vector(41, prob.n_dof)
    z = s.new_vector()
    s.block_solve(dev(r), z)
    assert rel_max(host(z), mg.levels[0].slab_solve(r)) <= 1e-10


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("basis", ["nodal", "eigen"])
def test_schur_solve_matches_direct(name, basis):
    banner(name, f"schur solve ({basis})")
    prob, mg = oracle_for(name)
    s = schur_solver_for(name, basis)
    f = assemble_rhs(prob, W.random_modes(7, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    u = s.new_vector()
    it, rr, _ = s.solve(dev(f), u, rtol=1e-12, maxit=60)
    _, it_o, _ = mg.solve(f, rtol=1e-12, maxit=60)
    print(f"  schur/{basis}: {it} cycles (oracle {it_o}), relres {rr:.2e}")
    assert rr <= 1e-12 and abs(it - it_o) <= 1
    assert np.linalg.norm(host(u) - ud) <= 1e-10 * np.linalg.norm(ud)


# ---------------------------------------------------------------------------
# Image sizes at the tile boundaries of the LDS-resident 2-D transforms and
# of the Gram-matrix residual norm: n = 33 and 50 (rows and columns past the
# last whole MFMA tile done as dot products), 64 and 80 (whole tiles), 82
# (six tiles per axis, no dot products).  One slab inverse in both bases and
# an eigenbasis solve against the direct solution.
# ---------------------------------------------------------------------------
TILE_SHAPES = {f"2d_n{ne + p - 2}": dict(dim=2, n_elem=ne, degree=p, n_slabs=2, n_elem_t=1)
               for ne, p in ((33, 2), (50, 2), (64, 2), (80, 2), (82, 2))}


@functools.lru_cache(maxsize=None)
def tile_oracle(name):
    prob = OProblem(**TILE_SHAPES[name])
    return prob, MultigridOracle(prob, coarse_slabs=1)


@pytest.mark.parametrize("name", list(TILE_SHAPES))
def test_transform_tile_boundaries(name):
    import paper_1802_09277_amd as sth
    print(f"[gpu-parity] tile boundaries shape={name} {TILE_SHAPES[name]}", flush=True)
    prob, mg = tile_oracle(name)
    r = W.random_vector(22, prob.n_dof)
    zo = mg.levels[0].slab_solve(r)
    f = assemble_rhs(prob, W.random_modes(21, prob.dim))
    ud = mg.levels[0].forward_substitution(f)
    for basis in ("nodal", "eigen"):
        s = sth.Solver(**TILE_SHAPES[name], basis=basis, coarse_slabs=1)
        z = s.new_vector()
        s.block_solve(dev(r), z)
        assert rel_max(host(z), zo) <= 1e-11, basis
        u = s.new_vector()
        it, rr, _ = s.solve(dev(f), u, rtol=1e-12, maxit=60)
        print(f"  {basis}: {it} cycles, relres {rr:.2e}")
        assert rr <= 1e-12
        assert np.linalg.norm(host(u) - ud) <= 1e-10 * np.linalg.norm(ud), basis
        s.close()


# ---------------------------------------------------------------------------
# Speculative cycles (eigenbasis, fused cycle close): each cycle is enqueued
# before its predecessor's norm has reached the host and is skipped on the
# device when the predecessor may have converged.  The iterates, counts and
# results must be those of the plain loop, eager or replayed, and the NaN and
# maxit exits must behave as there.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["2d_16slabs", "2d_p1_net3", "3d_8slabs", "2d_ragged_p3", "3d_p3"])
def test_speculative_cycles_match_plain_loop(name):
    banner(name, "speculation")
    prob, mg = oracle_for(name)
    s = eigen_solver_for(name)
    f = dev(assemble_rhs(prob, W.random_modes(13, prob.dim)))
    ud = mg.levels[0].forward_substitution(host(f))
    stream = torch.cuda.Stream()
    results = []
    for spec, graphs in ((False, False), (True, False), (True, True), (True, True), (False, True)):
        s.speculate(spec)
        s.use_graphs(graphs)
        with torch.cuda.stream(stream):
            u = s.new_vector()
            it, rr, _ = s.solve(f, u, rtol=1e-11, maxit=60, stream=stream)
        stream.synchronize()
        results.append((it, rr, host(u)))
        print(f"  speculate={spec} graphs={graphs}: {it} cycles, relres {rr:.3e}")
    s.speculate(True)
    s.use_graphs(False)
    for it, rr, u in results[1:]:
        assert it == results[0][0] and rr == results[0][1]
        assert np.array_equal(u, results[0][2])
    assert results[0][1] <= 1e-11
    assert np.linalg.norm(results[0][2] - ud) <= 1e-9 * np.linalg.norm(ud)
    # exits: maxit (no cycle beyond it) and a non-finite right-hand side
    for maxit in (1, 2, 3):
        u = s.new_vector()
        it, rr, code = s.solve(f, u, rtol=1e-30, maxit=maxit, check=False)
        assert code == -6 and it == maxit
    g = host(f).copy()
    g[5] = np.nan
    u = s.new_vector()
    it, rr, code = s.solve(dev(g), u, rtol=1e-8, maxit=5, check=False)
    assert code == -6 and it <= 1
    # a start that already meets the tolerance: the flag of the initial pass
    # skips the cycles enqueued behind it, and the result is the plain loop's
    outs = []
    for spec in (False, True):
        s.speculate(spec)
        u = dev(ud)
        it, rr, code = s.solve(f, u, rtol=1e-6, maxit=10, check=False)
        outs.append((it, rr, code, host(u)))
    s.speculate(True)
    assert outs[0][:3] == outs[1][:3] and outs[0][0] == 0 and outs[0][2] == 0
    assert np.array_equal(outs[0][3], outs[1][3])
    # a tolerance between the lower bound and the exact norm after k cycles:
    # the exact norm says "go on" (so the mapping into u enqueued behind it is
    # skipped on the device) and the solve continues as in the plain loop
    k = 2
    s.speculate(True)
    _, rb, _ = s.solve(f, s.new_vector(), rtol=0.0, maxit=k, check=False)    # bound / ||f||
    s.speculate(False)
    _, re_, _ = s.solve(f, s.new_vector(), rtol=0.0, maxit=k, check=False)   # exact / ||f||
    assert rb < re_
    rt = float(np.sqrt(rb * re_))
    outs = []
    for spec in (False, True):
        s.speculate(spec)
        u = s.new_vector()
        it, rr, code = s.solve(f, u, rtol=rt, maxit=60, check=False)
        outs.append((it, rr, code, host(u)))
    s.speculate(True)
    assert outs[0][:3] == outs[1][:3] and outs[0][0] > k and outs[0][2] == 0
    assert np.array_equal(outs[0][3], outs[1][3])


@pytest.mark.parametrize("spec", [False, True])
def test_zero_guess_start_without_cycles(spec):
    """A zero initial guess is not written to the eigenbasis buffer (the
    initial pass reads its device flag); a solve that ends before any cycle
    must still return exactly the zero guess, also after an earlier solve
    has left other values in that buffer: maxit = 0, and f = 0 (converged at
    the start)."""
    name = "2d_16slabs"
    banner(name, f"zero guess, no cycles, speculate={spec}")
    prob, _ = oracle_for(name)
    s = eigen_solver_for(name)
    s.speculate(spec)
    f = dev(assemble_rhs(prob, W.random_modes(8, prob.dim)))
    u = s.new_vector()
    it, rr, _ = s.solve(f, u, rtol=1e-10, maxit=60)        # leaves the eigenbasis buffers nonzero
    assert it > 0 and np.abs(host(u)).max() > 0
    u = s.new_vector()
    it, rr, code = s.solve(f, u, rtol=1e-10, maxit=0, check=False)
    assert it == 0 and not host(u).any(), (it, code)
    u = s.new_vector()
    it, rr, code = s.solve(s.new_vector(), u, rtol=1e-8, maxit=10, check=False)
    assert (it, code) == (0, 0) and not host(u).any()
    s.speculate(True)


# ---------------------------------------------------------------------------
# Cycle shapes other than V(1,1) in the eigenbasis iteration (the fused
# passes are V(1,1) only; these run the general level loop, including the
# prolongation alone when there is no post-smoothing step) on a padded
# four-level shape, cycle by cycle against the oracle's multigrid with the
# same nu1, nu2.
# ---------------------------------------------------------------------------
CYCLE_SHAPE = dict(dim=2, n_elem=6, degree=2, n_slabs=8, n_elem_t=2)   # 36 modes padded to 48


@pytest.mark.parametrize("nu", [(1, 0), (0, 1), (2, 1), (1, 2)])
@pytest.mark.parametrize("basis", ["nodal", "eigen"])
def test_cycle_shapes_match_oracle(nu, basis):
    import paper_1802_09277_amd as sth
    print(f"[gpu-parity] cycle shape V{nu} basis={basis} {CYCLE_SHAPE}", flush=True)
    prob = OProblem(**CYCLE_SHAPE)
    mg = MultigridOracle(prob, nu1=nu[0], nu2=nu[1], coarse_slabs=1)
    s = sth.Solver(**CYCLE_SHAPE, nu_pre=nu[0], nu_post=nu[1], coarse_slabs=1, basis=basis)
    assert s.num_levels == len(mg.levels) == 4
    f = assemble_rhs(prob, W.random_modes(9, prob.dim))
    fd = dev(f)
    uo = np.zeros_like(f)
    for k in range(1, 4):
        uo = mg.vcycle(f, uo)
        u = s.new_vector()
        it, rr, code = s.solve(fd, u, rtol=0.0, maxit=k, check=False)
        assert (it, code) == (k, -6), last_error()
        assert rel_max(host(u), uo) <= 1e-10, k
    s.close()


# ---------------------------------------------------------------------------
# A five-level 2-D shape wide enough for the widest slab chains of the
# finest-level cycle pass (91 x 91 elements, p = 2, 64 slabs; the bench
# workloads run the same chains): the eigenbasis iterates after 1, 2 and 3
# cycles and a solve to 1e-12 against the oracle's multigrid iterates and
# direct solution, sampled at 3000 indices (tests/golden/deep_cycle_samples.txt,
# written by make_deep_cycle_samples.py from the oracle alone).
# ---------------------------------------------------------------------------
DEEP = os.path.join(os.path.dirname(__file__), "golden", "deep_cycle_samples.txt")
DEEP_SHAPE = dict(dim=2, n_elem=91, degree=2, n_slabs=64, n_elem_t=1)


@pytest.mark.parametrize("temporal", ["eigen", "schur"])
def test_deep_wide_shape_cycles(temporal):
    import paper_1802_09277_amd as sth
    if not os.path.exists(DEEP):
        pytest.skip("golden samples not generated")
    print(f"[gpu-parity] deep wide shape temporal={temporal} {DEEP_SHAPE}", flush=True)
    data = np.loadtxt(DEEP)
    idx = data[:, 0].astype(np.int64)
    s = sth.Solver(**DEEP_SHAPE, coarse_slabs=4, basis="eigen", temporal=temporal)
    assert s.num_levels == 5
    f = s.new_vector()
    s.load_rhs(W.random_modes(3, 2), f)
    assert rel_max(host(f)[idx], data[:, 1]) <= 1e-13
    for k in range(1, 4):
        u = s.new_vector()
        it, rr, code = s.solve(f, u, rtol=0.0, maxit=k, check=False)
        assert (it, code) == (k, -6), last_error()
        err = rel_max(host(u)[idx], data[:, 1 + k])
        print(f"  cycle {k}: sampled max rel error {err:.2e}")
        assert err <= 1e-10, k
    u = s.new_vector()
    it, rr, _ = s.solve(f, u, rtol=1e-12, maxit=60)
    err = rel_max(host(u)[idx], data[:, 5])
    print(f"  solve: {it} cycles, relres {rr:.2e}, sampled max rel error vs direct {err:.2e}")
    assert rr <= 1e-12 and err <= 1e-10
    s.close()


# ---------------------------------------------------------------------------
# The residual kernel of large 2-D images (n >= 128: one wave per column
# range and row range, marching along y; overlapping column chunks) on
# ragged shapes, element-wise against the oracle's assembled L_h.
# ---------------------------------------------------------------------------
MARCH_SHAPES = {
    "2d_n128_p1": dict(dim=2, n_elem=129, degree=1, n_slabs=3, n_elem_t=2),
    "2d_n130_p2": dict(dim=2, n_elem=130, degree=2, n_slabs=3, n_elem_t=2),
    # N_t = 3, p = 2: the instantiation of the 2-D p = 2 one-time-element workloads
    "2d_n128_p2_nt3": dict(dim=2, n_elem=128, degree=2, n_slabs=3, n_elem_t=1),
    "2d_n181_p3": dict(dim=2, n_elem=180, degree=3, n_slabs=2, n_elem_t=1),
}


@pytest.mark.parametrize("name", list(MARCH_SHAPES))
def test_residual_large_images(name):
    import paper_1802_09277_amd as sth
    from oracle.solve import SlabSystem
    shape = MARCH_SHAPES[name]
    print(f"[gpu-parity] large-image residual shape={name} {shape}", flush=True)
    prob = OProblem(**shape)
    sysm = SlabSystem.assemble(prob)
    s = sth.Solver(**shape)
    u = W.random_vector(40, prob.n_dof)
    f = W.random_vector(41, prob.n_dof)
    y = s.new_vector()
    s.apply(dev(u), y)
    ref = sysm.apply(u)
    assert rel_max(host(y), ref) <= 1e-12
    r = s.new_vector()
    s.residual(dev(f), dev(u), r)
    assert rel_max(host(r), f - ref) <= 1e-12
    s.close()

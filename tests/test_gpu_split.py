"""GPU parity of the even/odd split spatial transforms (n = 128 and 256).

On a uniform mesh the 1-D pencil (K_x, M_x) commutes with the reflection
i -> n-1-i, so every eigenvector of the fast diagonalisation (Section 3.3)
is even or odd.  The library orders the modes [even | odd]; for n = 128 and
256 its per-axis transforms fold each line (x_k + x_{n-1-k} for the even
modes, x_k - x_{n-1-k} for the odd ones) before the forward products and
unfold the two half sums after the inverse ones, with half the multiply-adds.

Checked, on the x axis and the strided axes, forward and inverse:
  * 2-D, n = 128, two slabs, against the oracle (which uses neither the split
    nor the eigenvectors): one slab inverse in FP64 (1e-11), FP32 (1e-4) and
    BF16x3 (1e-3), the MinRes slab inverse after 12 iterations (1e-10), and
    eigenbasis V-cycle iterates (1e-10);
  * one slab of 2-D n = 256 and of 3-D n = 128 (6.3M unknowns, beyond the
    oracle's direct solver): the FP64 round trip z = A^{-1} (A z0) through
    the library's nodal operator (banded, no transforms) recovers z0 to 1e-9
    (an indexing fault in a fold or an unfold gives errors of order one), and
    the FP32 and BF16x3 slab inverses agree with that FP64 one to 1e-4 and
    1e-3.
"""
import functools
import sys

import numpy as np
import pytest

import workloads as W
from oracle.mg import MultigridOracle
from oracle.minres import MinresSlabInverse
from oracle.spacetime import Problem as OProblem, assemble_rhs, space_matrices, time_matrices

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N128 = dict(dim=2, n_elem=128, degree=2, n_slabs=2, n_elem_t=1)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def banner(what, shape):
    print(f"[gpu-split] {what} {shape}", flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def oracle128():
    prob = OProblem(**N128)
    return prob, MultigridOracle(prob, coarse_slabs=1)


@functools.lru_cache(maxsize=None)
def solver(prec="fp64", basis="nodal", minres_iters=0, **shape):
    import paper_1802_09277_amd as sth
    return sth.Solver(**shape, coarse_slabs=1, prec=prec, basis=basis, minres_iters=minres_iters)


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-11), ("fp32", 1e-4), ("bf16x3", 1e-3)])
def test_split_slab_inverse_matches_oracle(prec, bound):
    banner(f"{prec} block_solve", N128)
    prob, mg = oracle128()
    s = solver(prec, **N128)
    r = W.random_vector(51, prob.n_dof)
    z = s.new_vector()
    s.block_solve(dev(r), z)
    err = rel_max(host(z), mg.levels[0].slab_solve(r))
    print(f"  max relative difference {err:.2e}")
    assert err <= bound


def test_split_minres_slab_inverse_matches_oracle():
    banner("MinRes block_solve (12 iterations)", N128)
    prob, _ = oracle128()
    M, K = space_matrices(prob)
    Kt, Mt = time_matrices(0.0, prob.tau, prob.n_elem_t, prob.degree, prob.sigma)
    mi = MinresSlabInverse(Kt, Mt, K, M, 12)
    s = solver(minres_iters=12, **N128)
    r = W.random_vector(52, prob.n_dof)
    z = s.new_vector()
    s.block_solve(dev(r), z)
    R = r.reshape(prob.n_slabs, prob.slab_size)
    ref = np.concatenate([mi.apply(R[i]) for i in range(prob.n_slabs)])
    err = rel_max(host(z), ref)
    print(f"  max relative difference {err:.2e}")
    assert err <= 1e-10


def test_split_eigenbasis_iterates_match_oracle():
    banner("eigenbasis cycles", N128)
    prob, mg = oracle128()
    s = solver(basis="eigen", **N128)
    f = assemble_rhs(prob, W.random_modes(3, prob.dim))
    fd = dev(f)
    uo = np.zeros_like(f)
    for k in range(1, 3):
        uo = mg.vcycle(f, uo)
        u = s.new_vector()
        it, _, code = s.solve(fd, u, rtol=0.0, maxit=k, check=False)
        assert (it, code) == (k, -6)
        err = rel_max(host(u), uo)
        print(f"  {k} cycles: max relative difference {err:.2e}")
        assert err <= 1e-10


ROUND_TRIP = {
    "2d_n256": dict(dim=2, n_elem=256, degree=2, n_slabs=1, n_elem_t=1),
    "3d_n128": dict(dim=3, n_elem=128, degree=2, n_slabs=1, n_elem_t=1),
}


@pytest.mark.parametrize("name", list(ROUND_TRIP))
def test_split_slab_inverse_round_trip(name):
    shape = ROUND_TRIP[name]
    banner("fp64 round trip", shape)
    s = solver(**shape)
    z0 = dev(W.random_vector(53, s.vector_len))
    r = s.new_vector()
    s.apply(z0, r)                       # one slab: L_h = A_1
    z = s.new_vector()
    s.block_solve(r, z)
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(z - z0) / torch.linalg.vector_norm(z0))
    print(f"  |A^-1 A z0 - z0| / |z0| = {err:.2e}")
    assert err <= 1e-9


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-4), ("bf16x3", 1e-3)])
@pytest.mark.parametrize("name", list(ROUND_TRIP))
def test_split_reduced_precision_matches_fp64(name, prec, bound):
    """The reduced-precision split transforms against the FP64 slab inverse
    the round trip above checks (the bounds of the oracle comparison)."""
    shape = ROUND_TRIP[name]
    banner(f"{prec} block_solve against fp64", shape)
    s64, sp = solver(**shape), solver(prec, **shape)
    r = dev(W.random_vector(54, s64.vector_len))
    z64, zp = s64.new_vector(), sp.new_vector()
    s64.block_solve(r, z64)
    sp.block_solve(r, zp)
    err = rel_max(host(zp), host(z64))
    print(f"  max relative difference {err:.2e}")
    assert err <= bound
    sp.close()

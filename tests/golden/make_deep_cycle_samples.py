"""Writes sampled oracle multigrid iterates of a deep, wide 2-D shape.  Calls
only the oracle.

    python tests/golden/make_deep_cycle_samples.py          # ~2 min

Shape: unit square, p = 2, 91 x 91 elements (n = 91 interior functions per
axis, 8281 spatial modes), 64 slabs x 1 time element, theta 0.01, V(1,1)
cycles with omega 1/2, time coarsening down to 4 slabs (levels 64, 32, 16,
8, 4: five levels), right-hand side of 8 random modes (seed 3).  This is the
smallest 2-D shape on which the finest level of the eigenbasis iteration runs
its widest slab chains, so the tests compare that configuration cycle by
cycle.  Stored at 3000 seeded indices: the load vector, the oracle's
V-cycle iterates after 1, 2 and 3 cycles from zero (Section 3.1, with the
readings of the oracle's multigrid module) and the direct solution
(slab-wise forward substitution of eq. equ_linear_system), with the
Euclidean norms of the full vectors.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W                                   # noqa: E402
from oracle.spacetime import Problem, assemble_rhs       # noqa: E402
from oracle.mg import MultigridOracle                    # noqa: E402

SHAPE = dict(dim=2, n_elem=91, degree=2, n_slabs=64, n_elem_t=1)
COARSE_SLABS = 4
RHS_SEED = 3
CYCLES = 3


def main(n_samples=3000, seed=777):
    t0 = time.time()
    prob = Problem(**SHAPE)
    mg = MultigridOracle(prob, coarse_slabs=COARSE_SLABS)
    f = assemble_rhs(prob, W.random_modes(RHS_SEED, prob.dim))
    print(f"setup {time.time() - t0:.1f} s, {len(mg.levels)} levels", flush=True)
    iters = []
    u = np.zeros_like(f)
    for _ in range(CYCLES):
        u = mg.vcycle(f, u)
        iters.append(u)
        print(f"cycle {len(iters)}: {time.time() - t0:.1f} s", flush=True)
    ud = mg.levels[0].forward_substitution(f)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(prob.n_dof, size=n_samples, replace=False))
    path = os.path.join(HERE, "deep_cycle_samples.txt")
    with open(path, "w") as fh:
        fh.write("# oracle multigrid iterates of a five-level 2-D shape (unit square, p = 2, 91 x 91 elements,\n")
        fh.write("# 64 slabs x 1 time element, coarsest level 4 slabs, V(1,1), omega 1/2, random modes seed 3)\n")
        fh.write("# written by tests/golden/make_deep_cycle_samples.py (oracle only)\n")
        fh.write(f"# unknowns {prob.n_dof} levels {len(mg.levels)}\n")
        fh.write("# norms f u1 u2 u3 u_direct " + " ".join(f"{np.linalg.norm(v):.17e}" for v in [f] + iters + [ud])
                 + "\n")
        fh.write("# columns: index f u1 u2 u3 u_direct\n")
        for i in idx:
            fh.write(f"{i} " + " ".join(f"{v[i]:.17e}" for v in [f] + iters + [ud]) + "\n")
    print(f"wrote {path} ({time.time() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    main()

"""Writes sampled oracle values for the full-size workloads.  Calls only the
oracle.

    python tests/golden/make_fullsize_samples.py            # C2, ~15 min
    python tests/golden/make_fullsize_samples.py C3 rhs     # load vector only
    python tests/golden/make_fullsize_samples.py C4 rhs

C2 (unit square, p = 3, 64 x 64 elements, 256 slabs x 2 time elements, 8
random modes, seed 2): the load vector and the direct solution (slab-wise
SuperLU forward substitution of eq. equ_linear_system) at 4000 seeded
indices, plus their Euclidean norms.

"rhs" (C3: unit cube, p = 2, 32^3 elements, 128 slabs; C4: unit square,
p = 2, 256 x 256 elements, 1024 slabs x 1 time element): the load vector by
the oracle's space-time quadrature on the first, a middle and the last slab,
at 3000 seeded indices per slab, and the Euclidean norm of those slabs.  A
direct solve is out of reach for the oracle at these sizes; the tests check
the GPU solution with the oracle's slab operators instead.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W                                   # noqa: E402
from oracle.spacetime import Problem, assemble_rhs       # noqa: E402
from oracle.solve import SlabSystem                      # noqa: E402


def main(name="C2", n_samples=4000, seed=12345):
    cfg = W.CONFIGS[name]
    prob = Problem(cfg.dim, cfg.n_elem, cfg.degree, cfg.n_slabs, cfg.n_elem_t, cfg.T, cfg.theta)
    t0 = time.time()
    sysm = SlabSystem.assemble(prob)
    print(f"assembly {time.time() - t0:.1f} s", flush=True)
    f = assemble_rhs(prob, cfg.modes())
    print(f"load vector {time.time() - t0:.1f} s", flush=True)
    u = sysm.forward_substitution(f)
    print(f"direct solve {time.time() - t0:.1f} s", flush=True)
    rel = np.linalg.norm(sysm.apply(u) - f) / np.linalg.norm(f)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(prob.n_dof, size=n_samples, replace=False))
    path = os.path.join(HERE, f"{name.lower()}_direct_samples.txt")
    with open(path, "w") as fh:
        fh.write(f"# oracle direct solution of the full-size workload {name}: {cfg.note}\n")
        fh.write("# written by tests/golden/make_fullsize_samples.py (oracle only)\n")
        fh.write(f"# unknowns {prob.n_dof} relres_of_direct_solution {rel:.3e}\n")
        fh.write(f"# norm_f {np.linalg.norm(f):.17e} norm_u {np.linalg.norm(u):.17e}\n")
        fh.write("# columns: index f[index] u[index]\n")
        for i in idx:
            fh.write(f"{i} {f[i]:.17e} {u[i]:.17e}\n")
    print(f"wrote {path}", flush=True)


def rhs_samples(name, n_per_slab=3000, seed=54321):
    cfg = W.CONFIGS[name]
    prob = Problem(cfg.dim, cfg.n_elem, cfg.degree, cfg.n_slabs, cfg.n_elem_t, cfg.T, cfg.theta)
    slabs = [0, prob.n_slabs // 2, prob.n_slabs - 1]
    rng = np.random.default_rng(seed)
    path = os.path.join(HERE, f"{name.lower()}_rhs_samples.txt")
    t0 = time.time()
    with open(path, "w") as fh:
        fh.write(f"# oracle load vector of the full-size workload {name}: {cfg.note}\n")
        fh.write("# written by tests/golden/make_fullsize_samples.py (oracle only)\n")
        rows = []
        for s in slabs:
            f = assemble_rhs(prob, cfg.modes(), slabs=[s])
            print(f"slab {s}: {time.time() - t0:.1f} s", flush=True)
            fh.write(f"# slab {s} norm_f_slab {np.linalg.norm(f):.17e}\n")
            idx = np.sort(rng.choice(prob.slab_size, size=min(n_per_slab, prob.slab_size), replace=False))
            rows += [(s * prob.slab_size + i, f[i]) for i in idx]
        fh.write("# columns: global index, f[index]\n")
        for i, v in rows:
            fh.write(f"{i} {v:.17e}\n")
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[2] == "rhs":
        rhs_samples(sys.argv[1])
    else:
        main(*sys.argv[1:2])

"""Full-size parity for the benchmark workload (unit square, p = 3, 64 x 64
elements, 256 slabs x 2 time elements, 8 random modes seed 2; 5,408,000
unknowns), in the launch configuration bench.py times (non-default stream,
graph replay of the solve iterations, default coarsest level).

Checked against oracle values sampled at 4000 seeded indices
(tests/golden/c2_direct_samples.txt, written by make_fullsize_samples.py
from the oracle's SuperLU forward substitution):
  * load vector: 1e-13 relative to the largest sampled entry;
  * FP64 solve to relative residual 1e-12: 1e-9 relative;
  * solves to relative residual 1e-8 (FP64, FP32 and BF16x3 transforms):
    1e-6 relative (the accuracy a 1e-8 residual allows here), and the
    relative residual itself.
"""
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c2_direct_samples.txt")


def _samples():
    if not os.path.exists(GOLD):
        pytest.skip("golden samples not generated")
    meta = {}
    with open(GOLD) as fh:
        for line in fh:
            if line.startswith("# norm_f"):
                parts = line.split()
                meta["norm_f"], meta["norm_u"] = float(parts[2]), float(parts[4])
    data = np.loadtxt(GOLD)
    return data[:, 0].astype(np.int64), data[:, 1], data[:, 2], meta


def _run(prec, rtol, basis="nodal"):
    import paper_1802_09277_amd as sth
    cfg = W.CONFIGS["C2"]
    print(f"[gpu-fullsize] C2 prec={prec} rtol={rtol} basis={basis}", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = sth.Solver(cfg.dim, cfg.n_elem, cfg.degree, cfg.n_slabs, cfg.n_elem_t, cfg.T, cfg.theta, prec=prec,
                       basis=basis, stream=stream)
        f = s.new_vector()
        s.load_rhs(cfg.modes(), f, stream=stream)
        u = s.new_vector()
        it, rr, _ = s.solve(f, u, rtol=rtol, maxit=100, stream=stream)
        nf = s.norm(f, stream=stream)
    stream.synchronize()
    out = (it, rr, f.cpu().numpy(), u.cpu().numpy(), nf)
    s.close()
    return out


def test_fullsize_fp64_tight():
    idx, fs, us, meta = _samples()
    it, rr, f, u, nf = _run("fp64", 1e-12)
    print(f"  {it} cycles, relres {rr:.2e}")
    assert np.abs(f[idx] - fs).max() <= 1e-13 * np.abs(fs).max()
    assert abs(nf - meta["norm_f"]) <= 1e-12 * meta["norm_f"]
    err = np.abs(u[idx] - us).max() / np.abs(us).max()
    print(f"  sampled max rel error vs direct {err:.2e}")
    assert rr <= 1e-12 and err <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_fullsize_bench_tolerance(prec):
    idx, fs, us, meta = _samples()
    it, rr, f, u, nf = _run(prec, 1e-8)
    err = np.abs(u[idx] - us).max() / np.abs(us).max()
    print(f"  {prec}: {it} cycles, relres {rr:.2e}, sampled max rel error vs direct {err:.2e}")
    assert rr <= 1e-8 and err <= 1e-6


def test_fullsize_eigenbasis():
    idx, fs, us, meta = _samples()
    it, rr, f, u, nf = _run("fp64", 1e-12, basis="eigen")
    err = np.abs(u[idx] - us).max() / np.abs(us).max()
    print(f"  eigenbasis: {it} cycles, relres {rr:.2e}, sampled max rel error vs direct {err:.2e}")
    assert rr <= 1e-12 and err <= 1e-9

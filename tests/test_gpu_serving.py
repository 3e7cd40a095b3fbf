"""Serving loop (sth_server_*): continuous batching of independent solves.

A request's result must not depend on what else runs beside it: the same
request alone and inside a mix of other shapes gives the same vector (the
kernels are deterministic; graph replays and eager launches agree bitwise),
and it matches the oracle's direct solve.  Admission keeps the resident
setups within the device budget, setups are reused per problem shape, and
invalid or oversized requests are refused at submission.
"""
import numpy as np
import pytest

import workloads as W
from oracle.spacetime import Problem as OProblem, assemble_rhs
from oracle.solve import SlabSystem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (problem, rhs seed): 2-D and 3-D, multilevel and single-level (exact)
# solves, both iteration bases, reduced precision
MIX = [
    (dict(dim=2, n_elem=12, degree=2, n_slabs=8, n_elem_t=2, basis="eigen"), 11),
    (dict(dim=2, n_elem=20, degree=3, n_slabs=16, n_elem_t=2, basis="eigen", coarse_slabs=2), 12),
    (dict(dim=2, n_elem=16, degree=2, n_slabs=4, n_elem_t=2, basis="nodal", coarse_slabs=1), 13),
    (dict(dim=2, n_elem=24, degree=4, n_slabs=8, n_elem_t=2, basis="nodal", prec="fp32"), 14),
    (dict(dim=3, n_elem=6, degree=2, n_slabs=4, n_elem_t=2, basis="eigen", coarse_slabs=1), 15),
    (dict(dim=2, n_elem=12, degree=2, n_slabs=8, n_elem_t=2, basis="eigen"), 16),
    (dict(dim=2, n_elem=40, degree=2, n_slabs=32, n_elem_t=1, basis="eigen", coarse_slabs=2), 17),
    (dict(dim=3, n_elem=5, degree=3, n_slabs=8, n_elem_t=2, basis="nodal", coarse_slabs=2), 18),
]
RTOL = 1e-11


def _server(budget=8 << 30, max_active=4):
    import paper_1802_09277_amd as sth
    return sth.Server(budget, max_active)


def _out(problem):
    import paper_1802_09277_amd as sth
    shape = {k: v for k, v in problem.items() if k in ("dim", "n_elem", "degree", "n_slabs", "n_elem_t")}
    return torch.zeros(sth.problem_vector_len(**shape), dtype=torch.float64, device="cuda")


def _oracle_direct(problem, seed):
    prob = OProblem(problem["dim"], problem["n_elem"], problem["degree"], problem["n_slabs"], problem["n_elem_t"])
    f = assemble_rhs(prob, W.random_modes(seed, prob.dim))
    return SlabSystem.assemble(prob).forward_substitution(f)


def _run_all(server, items):
    tickets, outs = [], []
    for problem, seed in items:
        u = _out(problem)
        outs.append(u)
        tickets.append(server.submit(W.random_modes(seed, problem["dim"]), u, rtol=RTOL, maxit=100, **problem))
    stats = [server.wait(t) for t in tickets]
    torch.cuda.synchronize()
    return [u.cpu().numpy() for u in outs], stats


def test_result_alone_equals_result_in_mix_and_oracle():
    print("[gpu-serving] alone vs mix", flush=True)
    target = MIX[1]
    srv = _server()
    (alone,), (st_alone,) = _run_all(srv, [target])
    srv.close()
    assert st_alone["status"] == 0, st_alone["message"]
    srv = _server()
    outs, stats = _run_all(srv, MIX[:1] + [target] + MIX[2:])
    srv.close()
    for (problem, _), st in zip(MIX, stats):
        assert st["status"] == 0 and st["relres"] <= RTOL, (problem, st)
    assert np.array_equal(outs[1], alone)
    ud = _oracle_direct(*target)
    assert np.linalg.norm(alone - ud) <= 1e-8 * np.linalg.norm(ud)


@pytest.mark.parametrize("k", range(len(MIX)))
def test_every_mix_member_matches_oracle(k):
    print(f"[gpu-serving] oracle parity of mix member {k}: {MIX[k]}", flush=True)
    srv = _server()
    outs, stats = _run_all(srv, MIX)
    srv.close()
    ud = _oracle_direct(*MIX[k])
    st = stats[k]
    assert st["status"] == 0, st["message"]
    err = np.linalg.norm(outs[k] - ud) / np.linalg.norm(ud)
    print(f"  cycles {st['iters']}, relres {st['relres']:.2e}, error vs direct {err:.2e}, "
          f"latency {st['latency_ms']:.1f} ms")
    assert err <= 1e-8


def test_graph_replay_serving_matches_eager():
    """Setups made with graph replay on (sth_server_use_graphs) give the
    vectors of eager launches bitwise, also when a cached setup replays its
    captured iterations for a later request; a mixed-precision eigenbasis
    request (FP64 defect correction, FP32 storage) is in the mix."""
    print("[gpu-serving] graph replay vs eager", flush=True)
    mixed = (dict(dim=2, n_elem=40, degree=2, n_slabs=32, n_elem_t=1, basis="eigen", prec="fp32", coarse_slabs=2), 19)
    items = MIX + [mixed]
    srv = _server()
    eager, st_e = _run_all(srv, items)
    srv.close()
    srv = _server()
    srv.use_graphs(True)
    first, st_1 = _run_all(srv, items)
    again, st_2 = _run_all(srv, items)
    srv.close()
    for a, b, c, s1, s2 in zip(eager, first, again, st_1, st_2):
        assert s1["status"] == 0 and s2["status"] == 0, (s1["message"], s2["message"])
        assert s2["setup_reused"]
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_same_shape_reuses_setup_and_results_are_repeatable():
    print("[gpu-serving] setup cache", flush=True)
    srv = _server()
    outs, stats = _run_all(srv, [MIX[0]])
    outs2, stats2 = _run_all(srv, [MIX[0], MIX[5]])
    srv.close()
    assert not stats[0]["setup_reused"] and stats2[0]["setup_reused"]
    assert np.array_equal(outs[0], outs2[0])
    # MIX[5] has the shape of MIX[0] with another right-hand side
    assert not np.array_equal(outs2[0], outs2[1])


def test_admission_within_budget_and_eviction():
    import paper_1802_09277_amd as sth
    print("[gpu-serving] budget", flush=True)
    sizes = []
    for problem, _ in MIX[:3]:
        kw = {k: v for k, v in problem.items() if k != "prec"}
        shape = {k: v for k, v in kw.items() if k in ("dim", "n_elem", "degree", "n_slabs", "n_elem_t")}
        sizes.append(sth.workspace_bytes(**kw) + 16 * sth.problem_vector_len(**shape))
    budget = max(sizes) + 1024          # room for one setup at a time
    srv = _server(budget=budget, max_active=3)
    outs, stats = _run_all(srv, MIX[:3] * 2)
    resident, setups = srv.resident()
    srv.close()
    assert all(st["status"] == 0 for st in stats), [st["message"] for st in stats]
    assert resident <= budget and setups <= 1
    for a, b in zip(outs[:3], outs[3:]):
        assert np.array_equal(a, b)


def test_refusals_at_submit():
    import paper_1802_09277_amd as sth
    print("[gpu-serving] refusals", flush=True)
    srv = _server(budget=1 << 20)
    u = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(sth.StatusError) as e:
        srv.submit(W.random_modes(1, 2), u, **dict(dim=2, n_elem=64, degree=3, n_slabs=256, n_elem_t=2))
    assert e.value.name == "STH_ENOMEM"
    with pytest.raises(sth.StatusError) as e:
        srv.submit(W.random_modes(1, 2), u, **dict(dim=4, n_elem=8, degree=2, n_slabs=4, n_elem_t=2))
    assert e.value.name == "STH_EINVAL"
    srv.close()

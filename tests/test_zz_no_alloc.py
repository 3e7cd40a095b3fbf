"""The load-vector entry point that allocates nothing (sth_load_rhs_noalloc,
mode tables staged in the library's fixed device scratch) against the
allocating sth_load_rhs, through the C ABI: two calls in a row, the second
with a smaller input (fewer modes, a smaller problem), then a 3-D problem;
the same kernel reads the same tables, so the vectors must be identical.
A mode table larger than the scratch is refused on the host before any copy
or launch."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    (dict(dim=2, n_elem=20, degree=3, n_slabs=16, n_elem_t=2), 8, 31),
    (dict(dim=2, n_elem=8, degree=2, n_slabs=4, n_elem_t=2), 3, 32),     # smaller than the first
    (dict(dim=3, n_elem=7, degree=2, n_slabs=4, n_elem_t=1), 5, 33),
]


def _both(shape, n_modes, seed):
    import paper_1802_09277_amd as sth
    print(f"[gpu-noalloc] {shape} modes={n_modes} seed={seed}", flush=True)
    s = sth.Solver(**shape, basis="eigen")
    modes = W.random_modes(seed, shape["dim"], n_modes=n_modes)
    fa = s.new_vector()
    s.load_rhs(modes, fa)
    fb = torch.full_like(fa, float("nan"))
    assert s.load_rhs_noalloc(modes, fb) == 0
    torch.cuda.synchronize()
    out = fa.cpu().numpy(), fb.cpu().numpy()
    s.close()
    return out


def test_noalloc_load_rhs_matches_allocating_entry_point():
    for shape, n_modes, seed in CASES:
        a, b = _both(shape, n_modes, seed)
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), shape


def test_noalloc_load_rhs_refuses_oversized_tables():
    import paper_1802_09277_amd as sth
    shape = dict(dim=2, n_elem=8, degree=2, n_slabs=64, n_elem_t=2)
    s = sth.Solver(**shape)
    # 64 slabs x 4 time functions + 3 x 8 spatial entries = 280 doubles per
    # mode: 2000 modes need 560000 doubles, more than the 524288 of the scratch
    modes = W.random_modes(5, 2, n_modes=2000)
    f = s.new_vector()
    f.fill_(7.0)
    code = s.load_rhs_noalloc(modes, f, check=False)
    torch.cuda.synchronize()
    assert code == -1
    assert "scratch" in sth.load_library().sth_last_error().decode()
    assert bool((f == 7.0).all())
    # and a small request afterwards still works
    ok = W.random_modes(6, 2, n_modes=2)
    fa = s.new_vector()
    s.load_rhs(ok, fa)
    assert s.load_rhs_noalloc(ok, f) == 0
    torch.cuda.synchronize()
    assert torch.equal(fa, f)
    s.close()

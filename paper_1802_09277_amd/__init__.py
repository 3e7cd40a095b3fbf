"""MI355X-native space-time heat-equation slab solver (Python binding).

Thin ctypes binding of the C ABI in include/sth.h: argument marshalling
only.  Every step of the solver runs in the HIP library libsth.so (built
in-tree by `paper_1802_09277_amd.build`); PyTorch supplies device memory and
streams.  There is no fallback: if the library is missing or no GPU is
present, the GPU entry points raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsth.so")

STATUS = {0: "STH_OK", -1: "STH_EINVAL", -2: "STH_ENOMEM", -3: "STH_EHIP", -4: "STH_ENOTPOS",
          -5: "STH_ECOND", -6: "STH_ENOCONV", -7: "STH_ENODEV", -8: "STH_EAGAIN"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
KCLASS = {"residual": 0, "xform_x": 1, "xform_s": 2, "timemix": 3, "restrict": 4, "prolong": 5,
          "norm": 6, "other": 7, "xform_2d": 8, "eig_smooth": 9, "eig_resid": 10, "resnorm": 11,
          "eig_cycle_end": 12, "eig_cycle_close": 13, "eig_coarse": 14, "minres": 15}


class StatusError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_elem", ctypes.c_int), ("degree", ctypes.c_int),
                ("n_slabs", ctypes.c_int), ("n_elem_t", ctypes.c_int), ("T", ctypes.c_double),
                ("theta", ctypes.c_double), ("omega", ctypes.c_double), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("transform_prec", ctypes.c_int), ("coarse_slabs", ctypes.c_int),
                ("iterate_basis", ctypes.c_int), ("temporal_form", ctypes.c_int), ("space_ratio", ctypes.c_double),
                ("minres_iters", ctypes.c_int)]


class RhsModes(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int), ("amp", ctypes.POINTER(ctypes.c_double)),
                ("k", ctypes.POINTER(ctypes.c_int)), ("omega", ctypes.POINTER(ctypes.c_double)),
                ("phase", ctypes.POINTER(ctypes.c_double))]


class RequestStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("relres", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("footprint_bytes", ctypes.c_size_t),
                ("setup_reused", ctypes.c_int), ("message", ctypes.c_char * 160)]


_DP = ctypes.POINTER(ctypes.c_double)


class Factors(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("N_t", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("cond_V", ctypes.c_double)] + [(nm, _DP) for nm in
                                                ("M1", "K1", "U", "mu", "Kt", "Mt", "Pt", "V", "W",
                                                 "eig_re", "eig_im")] + [("schur", ctypes.c_int), ("R", _DP),
                                                                         ("mode_weights", _DP)]


_lib = None


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_09277_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sigs = {
        "sth_problem_default": (None, [P(Problem)]),
        "sth_workspace_bytes": (i, [P(Problem), P(sz)]),
        "sth_setup": (i, [P(Problem), vp, P(vp)]),
        "sth_vector_len": (sz, [vp]),
        "sth_num_levels": (i, [vp]),
        "sth_level_len": (sz, [vp, i]),
        "sth_level_elems": (i, [vp, i]),
        "sth_load_rhs": (i, [vp, P(RhsModes), vp, vp]),
        "sth_load_rhs_noalloc": (i, [vp, P(RhsModes), vp, vp]),
        "sth_apply": (i, [vp, vp, vp, vp]),
        "sth_residual": (i, [vp, vp, vp, vp, vp]),
        "sth_block_solve": (i, [vp, vp, vp, vp]),
        "sth_smooth": (i, [vp, vp, vp, i, vp]),
        "sth_vcycle": (i, [vp, vp, vp, vp]),
        "sth_solve": (i, [vp, vp, vp, d, i, P(i), P(d), vp]),
        "sth_solve_fgmres": (i, [vp, vp, vp, d, i, i, P(i), P(d), vp]),
        "sth_restrict": (i, [vp, i, vp, vp, vp]),
        "sth_prolong_add": (i, [vp, i, vp, vp, vp]),
        "sth_norm": (i, [vp, vp, P(d), vp]),
        "sth_destroy": (i, [vp]),
        "sth_last_error": (ctypes.c_char_p, []),
        "sth_host_factors": (i, [P(Problem), i, P(Factors)]),
        "sth_host_load_1d": (i, [P(Problem), d, d, i, _DP, _DP]),
        "sth_host_space_prolongation": (i, [i, i, _DP]),
        "sth_timing": (i, [vp, ctypes.c_uint]),
        "sth_timing_level": (i, [vp, i]),
        "sth_use_graphs": (i, [vp, i]),
        "sth_speculate": (i, [vp, i]),
        "sth_timing_report": (i, [vp, i, P(i), P(d), P(d), P(d)]),
        "sth_problem_vector_len": (sz, [P(Problem)]),
        "sth_server_create": (i, [sz, i, P(vp)]),
        "sth_server_submit": (i, [vp, P(Problem), P(RhsModes), d, i, vp, P(ctypes.c_longlong)]),
        "sth_server_poll": (i, [vp, ctypes.c_longlong, P(RequestStats)]),
        "sth_server_wait": (i, [vp, ctypes.c_longlong, P(RequestStats)]),
        "sth_server_resident": (i, [vp, P(sz), P(i)]),
        "sth_server_use_graphs": (i, [vp, i]),
        "sth_server_destroy": (i, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        msg = load_library().sth_last_error()
        raise StatusError(code, msg.decode() if msg else "")


BASIS = {"nodal": 0, "eigen": 1}


TEMPORAL = {"eigen": 0, "schur": 1, "auto": 2}


def make_problem(dim, n_elem, degree, n_slabs, n_elem_t, T=1.0, theta=0.01, omega=0.5, nu_pre=1,
                 nu_post=1, prec="fp64", coarse_slabs=None, basis="nodal", temporal="auto", space_ratio=0.0,
                 minres_iters=0):
    p = Problem()
    load_library().sth_problem_default(ctypes.byref(p))
    p.dim, p.n_elem, p.degree, p.n_slabs, p.n_elem_t = dim, n_elem, degree, n_slabs, n_elem_t
    p.T, p.theta, p.omega, p.nu_pre, p.nu_post = T, theta, omega, nu_pre, nu_post
    p.transform_prec = PREC[prec] if isinstance(prec, str) else int(prec)
    if coarse_slabs is not None:
        p.coarse_slabs = int(coarse_slabs)
    p.iterate_basis = BASIS[basis] if isinstance(basis, str) else int(basis)
    p.temporal_form = TEMPORAL[temporal] if isinstance(temporal, str) else int(temporal)
    p.space_ratio = float(space_ratio)
    p.minres_iters = int(minres_iters)
    return p


def workspace_bytes(**kw):
    out = ctypes.c_size_t()
    _check(load_library().sth_workspace_bytes(ctypes.byref(make_problem(**kw)), ctypes.byref(out)))
    return out.value


def host_factors(level=0, **kw):
    """Setup quantities of one level as numpy arrays (host only, no GPU)."""
    lib = load_library()
    p = make_problem(**kw)
    n = kw["n_elem"] + kw["degree"] - 2
    Nt = kw["n_elem_t"] + kw["degree"]
    arrs = {"M1": (n, n), "K1": (n, n), "U": (n, n), "mu": (n,), "Kt": (Nt, Nt), "Mt": (Nt, Nt),
            "Pt": (2 * Nt, Nt), "V": (Nt, Nt), "W": (Nt, Nt), "eig_re": (Nt,), "eig_im": (Nt,), "R": (Nt, Nt),
            "mode_weights": (n, 2)}
    buf = {k: np.zeros(s) for k, s in arrs.items()}
    f = Factors()
    for k, a in buf.items():
        setattr(f, k, a.ctypes.data_as(_DP))
    _check(lib.sth_host_factors(ctypes.byref(p), level, ctypes.byref(f)))
    buf["cond_V"] = f.cond_V
    buf["n_levels"] = f.n_levels
    buf["schur"] = bool(f.schur)
    return buf


def host_space_prolongation(n_elem_c, degree):
    """The library's P_x (n_f x n_c) from n_elem_c to 2 n_elem_c elements."""
    import numpy as np
    nf, nc = 2 * n_elem_c + degree - 2, n_elem_c + degree - 2
    out = np.zeros((nf, nc))
    _check(load_library().sth_host_space_prolongation(int(n_elem_c), int(degree), out.ctypes.data_as(_DP)))
    return out


def host_load_1d(omega, phase, k, **kw):
    p = make_problem(**kw)
    n = kw["n_elem"] + kw["degree"] - 2
    Nt = kw["n_elem_t"] + kw["degree"]
    tp = np.zeros(kw["n_slabs"] * Nt)
    sp_ = np.zeros(n)
    _check(load_library().sth_host_load_1d(ctypes.byref(p), omega, phase, int(k), tp.ctypes.data_as(_DP),
                                           sp_.ctypes.data_as(_DP)))
    return tp, sp_


def problem_vector_len(**kw):
    """Unknowns of a problem (n_slabs * N_t * n^dim) without a setup."""
    n = load_library().sth_problem_vector_len(ctypes.byref(make_problem(**kw)))
    if n == 0:
        raise StatusError(-1, "invalid problem")
    return n


def _modes(modes):
    amp, k, om, ph = modes.arrays()
    arrs = (np.ascontiguousarray(amp, dtype=np.float64), np.ascontiguousarray(k, dtype=np.int32).ravel(),
            np.ascontiguousarray(om, dtype=np.float64), np.ascontiguousarray(ph, dtype=np.float64))
    m = RhsModes(len(arrs[0]), arrs[0].ctypes.data_as(_DP), arrs[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                 arrs[2].ctypes.data_as(_DP), arrs[3].ctypes.data_as(_DP))
    return m, arrs          # keep the arrays alive while m is in use


def _ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One discrete problem on the GPU (setup factors and workspaces)."""

    def __init__(self, dim, n_elem, degree, n_slabs, n_elem_t, T=1.0, theta=0.01, omega=0.5, nu_pre=1,
                 nu_post=1, prec="fp64", coarse_slabs=None, basis="nodal", temporal="auto", space_ratio=0.0,
                 minres_iters=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP slab solver needs a gfx950 device")
        self.lib = load_library()
        self.problem = make_problem(dim, n_elem, degree, n_slabs, n_elem_t, T, theta, omega, nu_pre,
                                    nu_post, prec, coarse_slabs, basis, temporal, space_ratio, minres_iters)
        self.shape = dict(dim=dim, n_elem=n_elem, degree=degree, n_slabs=n_slabs, n_elem_t=n_elem_t)
        self.coarse_slabs = self.problem.coarse_slabs
        h = ctypes.c_void_p()
        _check(self.lib.sth_setup(ctypes.byref(self.problem), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.n = n_elem + degree - 2
        self.N_t = n_elem_t + degree
        self.dim = dim

    # sizes ---------------------------------------------------------------
    @property
    def vector_len(self):
        return self.lib.sth_vector_len(self.h)

    @property
    def num_levels(self):
        return self.lib.sth_num_levels(self.h)

    def level_len(self, level):
        return self.lib.sth_level_len(self.h, level)

    def level_elems(self, level):
        """spatial elements per axis on a level (halved by each space-time coarsening)"""
        return self.lib.sth_level_elems(self.h, level)

    def new_vector(self, level=0):
        import torch
        return torch.zeros(self.level_len(level), dtype=torch.float64, device="cuda")

    # operations ----------------------------------------------------------
    def load_rhs(self, modes, f, stream=None):
        m, _keep = _modes(modes)
        _check(self.lib.sth_load_rhs(self.h, ctypes.byref(m), _ptr(f), _stream(stream)))
        return f

    def load_rhs_noalloc(self, modes, f, stream=None, check=True):
        """The same load vector staged through the library's fixed device
        scratch (no device allocation); returns the status code."""
        m, _keep = _modes(modes)
        code = self.lib.sth_load_rhs_noalloc(self.h, ctypes.byref(m), _ptr(f), _stream(stream))
        if check:
            _check(code)
        return code

    def apply(self, u, y, stream=None):
        _check(self.lib.sth_apply(self.h, _ptr(u), _ptr(y), _stream(stream)))
        return y

    def residual(self, f, u, r, stream=None):
        _check(self.lib.sth_residual(self.h, _ptr(f), _ptr(u), _ptr(r), _stream(stream)))
        return r

    def block_solve(self, r, z, stream=None):
        _check(self.lib.sth_block_solve(self.h, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def smooth(self, f, u, steps=1, stream=None):
        _check(self.lib.sth_smooth(self.h, _ptr(f), _ptr(u), int(steps), _stream(stream)))
        return u

    def vcycle(self, f, u, stream=None):
        _check(self.lib.sth_vcycle(self.h, _ptr(f), _ptr(u), _stream(stream)))
        return u

    def solve(self, f, u, rtol=1e-8, maxit=100, stream=None, check=True):
        it = ctypes.c_int()
        rr = ctypes.c_double()
        code = self.lib.sth_solve(self.h, _ptr(f), _ptr(u), float(rtol), int(maxit), ctypes.byref(it),
                                  ctypes.byref(rr), _stream(stream))
        if check:
            _check(code)
        return it.value, rr.value, code

    def solve_fgmres(self, f, u, rtol=1e-8, maxit=100, restart=20, stream=None, check=True):
        """Flexible GMRES(restart) preconditioned by one V-cycle; returns (iterations, relres, code)."""
        it = ctypes.c_int()
        rr = ctypes.c_double()
        code = self.lib.sth_solve_fgmres(self.h, _ptr(f), _ptr(u), float(rtol), int(maxit), int(restart),
                                         ctypes.byref(it), ctypes.byref(rr), _stream(stream))
        if check:
            _check(code)
        return it.value, rr.value, code

    def restrict(self, level, r, rc, stream=None):
        _check(self.lib.sth_restrict(self.h, level, _ptr(r), _ptr(rc), _stream(stream)))
        return rc

    def prolong_add(self, level, ec, u, stream=None):
        _check(self.lib.sth_prolong_add(self.h, level, _ptr(ec), _ptr(u), _stream(stream)))
        return u

    def use_graphs(self, enable):
        """Graph replay of solve iterations on non-default streams (default off)."""
        _check(self.lib.sth_use_graphs(self.h, int(enable)))

    def speculate(self, enable):
        """Cycles enqueued ahead of their predecessor's norm (default on)."""
        _check(self.lib.sth_speculate(self.h, int(enable)))

    def norm(self, v, stream=None):
        out = ctypes.c_double()
        _check(self.lib.sth_norm(self.h, _ptr(v), ctypes.byref(out), _stream(stream)))
        return out.value

    def timing(self, class_mask, level=-1):
        """Event timing of the kernel classes in class_mask (bit per class, 0 = off),
        on one multigrid level (0 = finest) or on all (-1)."""
        _check(self.lib.sth_timing_level(self.h, int(level)))
        _check(self.lib.sth_timing(self.h, int(class_mask)))

    def timing_report(self, kclass):
        c = ctypes.c_int()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self.lib.sth_timing_report(self.h, KCLASS[kclass] if isinstance(kclass, str) else kclass,
                                          ctypes.byref(c), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)))
        return {"launches": c.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.sth_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop of the library (sth_server_*): requests are admitted by
    device footprint, run concurrently on their own streams and write their
    solution into a caller-owned device tensor."""

    def __init__(self, hbm_budget_bytes, max_active=4):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP slab solver needs a gfx950 device")
        self.lib = load_library()
        h = ctypes.c_void_p()
        _check(self.lib.sth_server_create(int(hbm_budget_bytes), int(max_active), ctypes.byref(h)))
        self.h = h

    def submit(self, modes, u_out, rtol=1e-8, maxit=100, **problem):
        """problem: the keyword arguments of make_problem; u_out: float64 CUDA
        tensor of problem_vector_len(**problem) elements (kept alive by the
        caller until the request has finished).  Returns the ticket."""
        p = make_problem(**problem)
        m, _keep = _modes(modes)
        t = ctypes.c_longlong()
        _check(self.lib.sth_server_submit(self.h, ctypes.byref(p), ctypes.byref(m), float(rtol), int(maxit),
                                          _ptr(u_out), ctypes.byref(t)))
        return t.value

    @staticmethod
    def _stats(st):
        return {"status": st.status, "iters": st.iters, "relres": st.relres, "queue_ms": st.queue_ms,
                "setup_ms": st.setup_ms, "solve_ms": st.solve_ms, "latency_ms": st.latency_ms,
                "footprint_bytes": st.footprint_bytes, "setup_reused": bool(st.setup_reused),
                "message": st.message.decode(errors="replace")}

    def poll(self, ticket):
        """None while pending, else the request's statistics."""
        st = RequestStats()
        code = self.lib.sth_server_poll(self.h, ticket, ctypes.byref(st))
        if code == -8:
            return None
        _check(code)
        return self._stats(st)

    def wait(self, ticket):
        st = RequestStats()
        _check(self.lib.sth_server_wait(self.h, ticket, ctypes.byref(st)))
        return self._stats(st)

    def use_graphs(self, enable=True):
        """setups made from now on replay captured solve iterations"""
        _check(self.lib.sth_server_use_graphs(self.h, 1 if enable else 0))

    def resident(self):
        b, n = ctypes.c_size_t(), ctypes.c_int()
        _check(self.lib.sth_server_resident(self.h, ctypes.byref(b), ctypes.byref(n)))
        return b.value, n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.sth_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Error norms of a discrete solution against a smooth exact solution.

Oracle module (test infrastructure only).

* L2(Q) norm of u - u_h.
* The mesh-dependent dG norm of Section 2.2:
    ||v||_dG^2 = sum_n ( ||grad_x v||^2_{Q_n} + sigma ||d_t v||^2_{Q_n}
                         + 1/2 ||[v]^{n-1}||^2_{Sigma_{n-1}} ) + 1/2 ||v||^2_{Sigma_N},
  with [v]^0 = v(0^+) the trace at t = 0 and [v]^n = v(t_n^+) - v(t_n^-).
All integrals by Gauss quadrature with p+3 points per direction.
"""
import numpy as np

from .spacetime import Axis, _tensor, _tensor_vec, _element_grid, interior_selector


class ExactSolution:
    """u(t, xs), d_t u(t, xs), grad u(t, xs) -> list over axes (x first)."""

    def __init__(self, u, ut, grad):
        self.u, self.ut, self.grad = u, ut, grad


def _full_coeffs(prob, u_slab):
    full = np.zeros(prob.N_t * prob.n_full ** prob.dim)
    full[interior_selector(prob)] = u_slab
    return full


class _SlabEval:
    """Values of a slab's discrete function at the space-time quadrature
    points, at the spatial quadrature points of its two faces."""

    def __init__(self, prob, slab, q):
        t0 = slab * prob.tau
        self.ax_t = Axis(t0, t0 + prob.tau, prob.n_elem_t, prob.degree, q)
        self.ax_x = [Axis(0.0, 1.0, prob.n_elem, prob.degree, q) for _ in range(prob.dim)]
        self.axes = [self.ax_t] + self.ax_x[::-1]
        self.el = _element_grid(self.axes)
        self.w = _tensor_vec([ax.W for ax in self.axes], self.el)
        nax = len(self.axes)
        coords = [_tensor_vec([ax.X if k == j else np.ones_like(ax.X) for k, ax in enumerate(self.axes)], self.el)
                  for j in range(nax)]
        self.t = coords[0]
        self.xs = [coords[nax - 1 - a] for a in range(prob.dim)]
        # global full-basis index of local functions
        g = np.zeros((len(self.el[0]), 1), dtype=np.int64)
        for ax, e in zip(self.axes, self.el):
            g = (g[:, :, None] * ax.N + ax.gidx[e][:, None, :]).reshape(g.shape[0], -1)
        self.g = g
        # spatial face quadrature
        sax = self.ax_x[::-1]
        self.sel = _element_grid(sax)
        self.sw = _tensor_vec([ax.W for ax in sax], self.sel)
        sc = [_tensor_vec([ax.X if k == j else np.ones_like(ax.X) for k, ax in enumerate(sax)], self.sel)
              for j in range(len(sax))]
        self.sxs = [sc[len(sax) - 1 - a] for a in range(prob.dim)]
        sg = np.zeros((len(self.sel[0]), 1), dtype=np.int64)
        for ax, e in zip(sax, self.sel):
            sg = (sg[:, :, None] * ax.N + ax.gidx[e][:, None, :]).reshape(sg.shape[0], -1)
        self.sg = sg
        self.sphi = _tensor([ax.V for ax in sax], self.sel)
        self.prob = prob

    def values(self, coef, kind):
        """kind: 'v', 'dt', or spatial axis index a (x=0) for d/dx_a."""
        Vs = [ax.V for ax in self.axes]
        arr = list(Vs)
        if kind == "dt":
            arr[0] = self.axes[0].D
        elif kind != "v":
            arr[len(self.axes) - 1 - kind] = self.axes[len(self.axes) - 1 - kind].D
        phi = _tensor(arr, self.el)
        return np.einsum("eqi,ei->eq", phi, coef[self.g])

    def face_values(self, coef, which):
        """Trace at t_{n-1}^+ (which='start') or t_n^- (which='end')."""
        tt = self.ax_t.a if which == "start" else self.ax_t.b
        psi = self.ax_t.point_values(tt)
        Nxf = self.prob.n_full ** self.prob.dim
        cx = psi @ coef.reshape(len(psi), Nxf)          # spatial coefficients at the face
        return np.einsum("eqi,ei->eq", self.sphi, cx[self.sg]), tt


def errors(prob, u, exact):
    """Returns dict(L2=..., dG=...) for the discrete solution vector u."""
    q = prob.degree + 3
    sig = prob.sigma
    U = u.reshape(prob.n_slabs, prob.slab_size)
    l2 = 0.0
    dg = 0.0
    prev_end = None
    for s in range(prob.n_slabs):
        ev = _SlabEval(prob, s, q)
        c = _full_coeffs(prob, U[s])
        e = exact.u(ev.t, ev.xs) - ev.values(c, "v")
        l2 += np.sum(ev.w * e * e)
        et = exact.ut(ev.t, ev.xs) - ev.values(c, "dt")
        dg += sig * np.sum(ev.w * et * et)
        gr = exact.grad(ev.t, ev.xs)
        for a in range(prob.dim):
            ea = gr[a] - ev.values(c, a)
            dg += np.sum(ev.w * ea * ea)
        start, t0 = ev.face_values(c, "start")
        if s == 0:
            jump = exact.u(np.full_like(start, t0), ev.sxs) - start
        else:
            jump = prev_end - start          # [e] = e^+ - e^- with u continuous
        dg += 0.5 * np.sum(ev.sw * jump * jump)
        end, t1 = ev.face_values(c, "end")
        prev_end = end
        if s == prob.n_slabs - 1:
            eN = exact.u(np.full_like(end, t1), ev.sxs) - end
            dg += 0.5 * np.sum(ev.sw * eN * eN)
    return {"L2": np.sqrt(l2), "dG": np.sqrt(dg)}


def dg_norm_sq_discrete(prob, u):
    """||v||_dG^2 of a discrete function v given by its coefficient vector,
    together with the SUPG boundary term
        sum_n sigma/2 (||grad v(t_n^-)||^2 - ||grad v(t_{n-1}^+)||^2),
    so that a_h(v, v) equals the sum of the two exactly (integration by parts
    of the time derivative terms, Section 2.2)."""
    q = prob.degree + 2
    sig = prob.sigma
    U = u.reshape(prob.n_slabs, prob.slab_size)
    dg = 0.0
    supg = 0.0
    prev_end = None
    for s in range(prob.n_slabs):
        ev = _SlabEval(prob, s, q)
        c = _full_coeffs(prob, U[s])
        vt = ev.values(c, "dt")
        dg += sig * np.sum(ev.w * vt * vt)
        for a in range(prob.dim):
            va = ev.values(c, a)
            dg += np.sum(ev.w * va * va)
        start, _ = ev.face_values(c, "start")
        jump = start if s == 0 else start - prev_end
        dg += 0.5 * np.sum(ev.sw * jump * jump)
        end, _ = ev.face_values(c, "end")
        prev_end = end
        if s == prob.n_slabs - 1:
            dg += 0.5 * np.sum(ev.sw * end * end)
        # gradient traces at both faces (spatial derivative of the face trace)
        Nxf = prob.n_full ** prob.dim
        for which, sign in (("end", 1.0), ("start", -1.0)):
            tt = ev.ax_t.a if which == "start" else ev.ax_t.b
            psi = ev.ax_t.point_values(tt)
            cx = psi @ c.reshape(len(psi), Nxf)
            sax = ev.ax_x[::-1]
            for a in range(prob.dim):
                arr = [ax.V for ax in sax]
                k = len(sax) - 1 - a
                arr[k] = sax[k].D
                dphi = _tensor(arr, ev.sel)
                ga = np.einsum("eqi,ei->eq", dphi, cx[ev.sg])
                supg += sign * 0.5 * sig * np.sum(ev.sw * ga * ga)
    return dg, supg

"""Space-time dG-IgA system for the heat equation, assembled by quadrature.

Oracle module (test infrastructure only; never imported by the product path).

What is computed, with the passage it follows:

* Problem (1.1): u_t - Laplace(u) = f on Q = (0,1)^d x (0,T), u = 0 on the
  lateral boundary, u(.,0) = u_0.
* Time slabs Q_n = Omega x (t_{n-1}, t_n) with a discontinuous B-spline
  space between slabs (Section 2.2).  The SUPG test function is
  w = v + sigma * dv/dt with sigma = theta_n * h_n.  The mesh size h_n is
  read as the temporal element size tau / n_el_t; Tables 1 and 2 are
  reproduced only under this reading.
* Slab matrix A_n[i, j] = b_{Q_n}(phi_j, phi_i) (Section 2.3, "Efficient
  Matrix Assembly"):
      int_{Q_n} d_t phi_j (phi_i + sigma d_t phi_i)
                + grad phi_j . grad(phi_i + sigma d_t phi_i) dx dt
      + int_Omega phi_j(x, t_{n-1}^+) phi_i(x, t_{n-1}^+) dx.
  Computed here by (d+1)-dimensional Gauss quadrature over the space-time
  elements, NOT through the Kronecker form of eq. (structureAn); the
  Kronecker form is what the tests check this against.
* Coupling B_n[i, k] = int_Omega phi^{n-1}_k(x, t_{n-1}^-) phi^n_i(x, t_{n-1}^+)
  evaluated at the face; L_h is block lower bidiagonal with A_n on the
  diagonal and -B_n below it (eq. equ_linear_system).
* Load vector f_n[i] = l_h(phi_i) = int_{Q_n} f (phi_i + sigma d_t phi_i)
  (+ int u_0 phi_i(., 0) on the first slab), Gauss rule with p+3 points per
  direction because f is not a polynomial.

Vector layout: slab-major, inside a slab the time index is the slowest and
the spatial x index the fastest (the Kronecker index of eq. structureAn):
  u[s][t][z][y][x], spatial indices over the interior (Dirichlet) functions.
"""
from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

from . import bspline as bs


@dataclass(frozen=True)
class Problem:
    dim: int
    n_elem: int        # spatial elements per axis on (0,1)
    degree: int        # spline degree in space and time
    n_slabs: int       # number of time slabs on (0, T)
    n_elem_t: int      # time elements per slab
    T: float = 1.0
    theta: float = 0.01

    @property
    def tau(self):
        return self.T / self.n_slabs

    @property
    def h_t(self):
        return self.tau / self.n_elem_t

    @property
    def sigma(self):
        return self.theta * self.h_t

    @property
    def N_t(self):
        return self.n_elem_t + self.degree

    @property
    def n_full(self):
        """spline functions per spatial axis before the Dirichlet elimination"""
        return self.n_elem + self.degree

    @property
    def n(self):
        """interior functions per spatial axis (u = 0 on the lateral boundary)"""
        return self.n_elem + self.degree - 2

    @property
    def N_x(self):
        return self.n ** self.dim

    @property
    def slab_size(self):
        return self.N_t * self.N_x

    @property
    def n_dof(self):
        return self.n_slabs * self.slab_size


# --------------------------------------------------------------------------
# per-axis element data
# --------------------------------------------------------------------------
class Axis:
    """Element-wise basis values on one axis (time or one space direction)."""

    def __init__(self, a, b, n_el, p, q):
        self.knots = bs.open_uniform_knots(a, b, n_el, p)
        self.p = p
        self.N = bs.n_basis(self.knots, p)
        self.n_el = n_el
        xs, ws, eidx = bs.element_quadrature(self.knots, q)
        assert len(xs) == n_el * q
        self.q = q
        vals = bs.basis_all(self.knots, p, xs, 0)
        ders = bs.basis_all(self.knots, p, xs, 1)
        # local functions of element e are e..e+p; check that every other
        # function vanishes there (local support of B-splines).
        self.gidx = np.array([[e + a for a in range(p + 1)] for e in range(n_el)])
        self.V = np.zeros((n_el, q, p + 1))
        self.D = np.zeros((n_el, q, p + 1))
        self.X = xs.reshape(n_el, q)
        self.W = ws.reshape(n_el, q)
        for e in range(n_el):
            rows = slice(e * q, (e + 1) * q)
            others = np.ones(self.N, dtype=bool)
            others[self.gidx[e]] = False
            assert np.all(vals[rows][:, others] == 0.0)
            assert np.all(ders[rows][:, others] == 0.0)
            self.V[e] = vals[rows][:, self.gidx[e]]
            self.D[e] = ders[rows][:, self.gidx[e]]
        self.a, self.b = a, b

    def point_values(self, x):
        return bs.basis_all(self.knots, self.p, [x], 0)[0]


def _tensor(arrays, elems):
    """Tensor product over axes of per-element arrays.

    arrays[k] has shape (n_el_k, q_k, A_k); elems[k] is an index array of
    length E selecting the element on axis k.  Returns (E, prod q, prod A)
    with the first axis slowest.
    """
    out = np.ones((len(elems[0]), 1, 1))
    for arr, e in zip(arrays, elems):
        sel = arr[e]                                     # (E, q, A)
        out = out[:, :, None, :, None] * sel[:, None, :, None, :]
        out = out.reshape(out.shape[0], out.shape[1] * out.shape[2], out.shape[3] * out.shape[4])
    return out


def _tensor_vec(vecs, elems):
    """Same as _tensor for per-element quadrature weights (n_el, q)."""
    out = np.ones((len(elems[0]), 1))
    for arr, e in zip(vecs, elems):
        sel = arr[e]
        out = (out[:, :, None] * sel[:, None, :]).reshape(out.shape[0], -1)
    return out


def _global_index(axes, elems):
    """Global (full-basis) index of every local function, time-major."""
    g = np.zeros((len(elems[0]), 1), dtype=np.int64)
    for ax, e in zip(axes, elems):
        sel = ax.gidx[e]                                  # (E, p+1)
        g = (g[:, :, None] * ax.N + sel[:, None, :]).reshape(g.shape[0], -1)
    return g


def _element_grid(axes):
    grids = np.meshgrid(*[np.arange(ax.n_el) for ax in axes], indexing="ij")
    return [g.ravel() for g in grids]


def interior_selector(prob):
    """Indices of the full-basis space-time slab vector that survive the
    Dirichlet elimination (first and last spline of every spatial axis)."""
    Nf = prob.n_full
    keep1 = np.arange(1, Nf - 1)
    idx = np.arange(prob.N_t)
    for _ in range(prob.dim):
        idx = (idx[:, None] * Nf + keep1[None, :]).ravel()
    return idx


def _axes(prob, slab, q):
    t0 = slab * prob.tau
    ax_t = Axis(t0, t0 + prob.tau, prob.n_elem_t, prob.degree, q)
    ax_x = [Axis(0.0, 1.0, prob.n_elem, prob.degree, q) for _ in range(prob.dim)]
    return ax_t, ax_x


def assemble_slab_matrix(prob, slab=0, chunk=256):
    """A_n for slab `slab` by (d+1)-D Gauss quadrature (p+1 points per
    direction and element, exact for the polynomial integrand) plus the
    upwind face term at t_{n-1}^+.  Returns CSR over interior unknowns."""
    p = prob.degree
    q = p + 1
    ax_t, ax_x = _axes(prob, slab, q)
    axes = [ax_t] + ax_x[::-1]          # (t, z, y, x): x fastest
    sig = prob.sigma
    n_full_slab = ax_t.N * prob.n_full ** prob.dim
    elems_all = _element_grid(axes)
    E = len(elems_all[0])
    rows, cols, data = [], [], []
    for c0 in range(0, E, chunk):
        el = [e[c0:c0 + chunk] for e in elems_all]
        w = _tensor_vec([ax.W for ax in axes], el)                     # (E,Q)
        Vs = [ax.V for ax in axes]
        phi = _tensor(Vs, el)                                          # (E,Q,A)
        dt = _tensor([axes[0].D] + Vs[1:], el)
        Wt = phi + sig * dt                                            # test fn
        loc = np.einsum("eq,eqi,eqj->eij", w, Wt, dt)
        for k in range(1, len(axes)):
            arr = list(Vs)
            arr[k] = axes[k].D
            gk = _tensor(arr, el)                                      # d_k phi
            arr[0] = axes[0].D
            gkt = _tensor(arr, el)                                     # d_k d_t phi
            loc += np.einsum("eq,eqi,eqj->eij", w, gk + sig * gkt, gk)
        g = _global_index(axes, el)
        rows.append(np.repeat(g[:, :, None], g.shape[1], axis=2).ravel())
        cols.append(np.repeat(g[:, None, :], g.shape[1], axis=1).ravel())
        data.append(loc.ravel())
    A = sp.coo_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_full_slab, n_full_slab)).tocsr()
    # upwind face term: int_Omega phi_j(t_{n-1}^+) phi_i(t_{n-1}^+)
    left = ax_t.point_values(ax_t.a)
    F = face_matrix(prob, ax_x, left, left)
    A = A + F
    keep = interior_selector(prob)
    return A[keep][:, keep].tocsr()


def face_matrix(prob, ax_x, psi_test, psi_trial):
    """int_Omega phi_i(x, t*) phi_k(x, t*) dx on the full basis, where the
    time parts of test and trial functions are given by their values
    psi_test, psi_trial at the face.  d-dimensional Gauss quadrature."""
    axes = ax_x[::-1]
    elems = _element_grid(axes)
    w = _tensor_vec([ax.W for ax in axes], elems)
    phi = _tensor([ax.V for ax in axes], elems)                        # (E,Q,A)
    g = _global_index(axes, elems)
    Nxf = prob.n_full ** prob.dim
    Nt = len(psi_test)
    # space-time face values: phi_i(x,t*) = psi_i(t*) * phi_ix(x)
    loc_x = np.einsum("eq,eqa,eqb->eab", w, phi, phi)
    rows, cols, data = [], [], []
    for it in range(Nt):
        for kt in range(len(psi_trial)):
            c = psi_test[it] * psi_trial[kt]
            if c == 0.0:
                continue
            rows.append((it * Nxf + np.repeat(g[:, :, None], g.shape[1], axis=2)).ravel())
            cols.append((kt * Nxf + np.repeat(g[:, None, :], g.shape[1], axis=1)).ravel())
            data.append((c * loc_x).ravel())
    shape = (Nt * Nxf, len(psi_trial) * Nxf)
    if not data:
        return sp.csr_matrix(shape)
    return sp.coo_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                         shape=shape).tocsr()


def assemble_coupling(prob, slab=1):
    """B_n coupling slab `slab`-1 (its end trace) into slab `slab` (its
    start trace), evaluated at the face t = slab*tau.  CSR, interior."""
    q = prob.degree + 1
    ax_t, ax_x = _axes(prob, slab, q)
    ax_prev, _ = _axes(prob, slab - 1, q)
    plus = ax_t.point_values(ax_t.a)          # phi^n_i(t_{n-1}^+)
    minus = ax_prev.point_values(ax_prev.b)   # phi^{n-1}_k(t_{n-1}^-)
    Bf = face_matrix(prob, ax_x, plus, minus)
    keep = interior_selector(prob)
    return Bf[keep][:, keep].tocsr()


def assemble_rhs(prob, f, u0=None, slabs=None, chunk=4096):
    """Load vector l_h(phi_i) for every slab (Gauss rule, p+3 points per
    direction).  f(t, xs) takes arrays t and a list xs of spatial coordinate
    arrays (x first).  Returns a flat vector in the slab layout.  Elements
    are visited in `chunk`-sized groups (memory only: same order of
    accumulation as one pass)."""
    p = prob.degree
    q = p + 3
    sig = prob.sigma
    keep = interior_selector(prob)
    out = []
    if slabs is None:
        slabs = range(prob.n_slabs)
    for s in slabs:
        ax_t, ax_x = _axes(prob, s, q)
        axes = [ax_t] + ax_x[::-1]
        el_all = _element_grid(axes)
        n_full_slab = ax_t.N * prob.n_full ** prob.dim
        vec = np.zeros(n_full_slab)
        Vs = [ax.V for ax in axes]
        for c0 in range(0, len(el_all[0]), chunk):
            el = [e[c0:c0 + chunk] for e in el_all]
            w = _tensor_vec([ax.W for ax in axes], el)
            coords = [_tensor_vec([ax.X if k == j else np.ones_like(ax.X) for k, ax in enumerate(axes)], el)
                      for j in range(len(axes))]
            tq = coords[0]
            xq = [coords[len(axes) - 1 - a] for a in range(prob.dim)]       # x, y, z
            fq = f(tq, xq)
            phi = _tensor(Vs, el)
            dt = _tensor([axes[0].D] + Vs[1:], el)
            loc = np.einsum("eq,eq,eqi->ei", w, fq, phi + sig * dt)
            g = _global_index(axes, el)
            np.add.at(vec, g.ravel(), loc.ravel())
        if s == 0 and u0 is not None:
            vec += initial_term(prob, ax_t, u0)
        out.append(vec[keep])
    return np.concatenate(out)


def initial_term(prob, ax_t, u0):
    """int_Omega u_0 phi_i(x, 0^+) dx (first slab only)."""
    q = prob.degree + 3
    ax_x = [Axis(0.0, 1.0, prob.n_elem, prob.degree, q) for _ in range(prob.dim)]
    axes = ax_x[::-1]
    el = _element_grid(axes)
    w = _tensor_vec([ax.W for ax in axes], el)
    coords = [_tensor_vec([ax.X if k == j else np.ones_like(ax.X) for k, ax in enumerate(axes)], el)
              for j in range(len(axes))]
    xq = [coords[len(axes) - 1 - a] for a in range(prob.dim)]
    phi = _tensor([ax.V for ax in axes], el)
    loc = np.einsum("eq,eq,eqi->ei", w, u0(xq), phi)
    g = _global_index(axes, el)
    Nxf = prob.n_full ** prob.dim
    vx = np.zeros(Nxf)
    np.add.at(vx, g.ravel(), loc.ravel())
    psi = ax_t.point_values(ax_t.a)
    return np.kron(psi, vx)


# --------------------------------------------------------------------------
# 1-D matrices (used for the Kronecker identities and the Table pins)
# --------------------------------------------------------------------------
def time_matrices(a, b, n_el, p, sigma, q=None):
    """Temporal K_t, M_t of eq. (TimeMatrices) on [a, b] by 1-D Gauss
    quadrature, including the upwind point term psi_j(a) psi_i(a) in K_t."""
    if q is None:
        q = p + 1
    ax = Axis(a, b, n_el, p, q)
    N = ax.N
    K = np.zeros((N, N))
    M = np.zeros((N, N))
    for e in range(n_el):
        g = ax.gidx[e]
        V, D, w = ax.V[e], ax.D[e], ax.W[e]
        test = V + sigma * D
        K[np.ix_(g, g)] += np.einsum("q,qi,qj->ij", w, test, D)
        M[np.ix_(g, g)] += np.einsum("q,qi,qj->ij", w, test, V)
    left = ax.point_values(a)
    K += np.outer(left, left)
    return K, M


def space_matrices_1d(n_el, p, q=None):
    """1-D spatial mass and stiffness on (0,1), interior functions only."""
    if q is None:
        q = p + 1
    ax = Axis(0.0, 1.0, n_el, p, q)
    N = ax.N
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    for e in range(n_el):
        g = ax.gidx[e]
        V, D, w = ax.V[e], ax.D[e], ax.W[e]
        M[np.ix_(g, g)] += np.einsum("q,qi,qj->ij", w, V, V)
        K[np.ix_(g, g)] += np.einsum("q,qi,qj->ij", w, D, D)
    return M[1:-1, 1:-1], K[1:-1, 1:-1]


def space_matrices(prob):
    """M_x, K_x over the interior of (0,1)^d as Kronecker products of the
    1-D matrices (x fastest)."""
    M1, K1 = space_matrices_1d(prob.n_elem, prob.degree)
    M = np.ones((1, 1))
    K = np.zeros((1, 1))
    for _ in range(prob.dim):
        K = np.kron(K, M1) + np.kron(M, K1)
        M = np.kron(M, M1)
    return M, K

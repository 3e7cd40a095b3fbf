"""Time-parallel multigrid with the damped block-Jacobi slab smoother.

Oracle module (test infrastructure only).

Section 3.1 (time-parallel multigrid): coarsening in time combines two
consecutive slabs into one; the smoother is damped block Jacobi
    u <- u + omega D^{-1} (f - L_h u),   D = diag(A_n),  omega = 1/2.
The paper defers the remaining multigrid details to its references.  The
readings used (and listed as such in the design notes):
  * V(nu1, nu2) cycle, coarsening in time only while the slab count is
    even and larger than `coarse_slabs`; the coarsest level is solved
    exactly by forward substitution (the coarse grid solver is the third
    ingredient Section 3.1 names without fixing it);
  * a coarse slab covers two fine slabs with the same number of time
    elements and the same degree; prolongation P is the exact embedding of
    the coarse slab space into the two fine slabs, computed here by an L2
    projection (exact because the spaces are nested), restriction R = P^T;
  * the coarse operator is the Galerkin product R L P, formed block-wise
    from the fine A and B (all slabs of a level are identical);
  * D^{-1} is applied exactly by sparse LU (the paper's "Direct" variant).
The residual norm is the Euclidean norm of the coefficient vector, relative
to ||f|| (zero initial guess), stopping at 1e-8 as in Section 4.4.

Coarsening in space (Section 4.4 states that the multigrid coarsens in
space as well as in time, again without the details): a level transition
either coarsens in time only (two slabs into one) or in space and time
together (also halving the spatial elements per axis).  The reading used
follows the space-time multigrid of the paper's reference on block Jacobi
smoothing (Gander and Neumueller): space and time are coarsened together
when the discrete parabolic ratio lambda = tau / h_x^2 of the level is at
least a critical value, in time only otherwise.  A space-time step halves
lambda, a time step doubles it.  The spatial prolongation P_x is the exact
embedding of the coarse spline space into the fine one (an L2 projection,
exact because the spaces are nested), on the interior functions; the
space-time prolongation of a coupled step is P_t (x) P_x (x) ... (x) P_x.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline as bs
from .spacetime import Axis
from .solve import SlabSystem


def time_prolongation(tau, n_el, p):
    """P_t (2 N_t x N_t): coarse slab [0, 2 tau] -> fine slabs [0, tau] and
    [tau, 2 tau], each with n_el elements of degree p.  Column j holds the
    fine coefficients of coarse basis function j, found by solving the fine
    mass-matrix system M_f c = (fine, coarse) with Gauss quadrature on the
    fine elements (exact: coarse functions are polynomials there)."""
    q = p + 2
    coarse = bs.open_uniform_knots(0.0, 2 * tau, n_el, p)
    blocks = []
    for (a, b) in [(0.0, tau), (tau, 2 * tau)]:
        ax = Axis(a, b, n_el, p, q)
        N = ax.N
        Mf = np.zeros((N, N))
        rhs = np.zeros((N, bs.n_basis(coarse, p)))
        for e in range(n_el):
            g = ax.gidx[e]
            Mf[np.ix_(g, g)] += np.einsum("q,qi,qj->ij", ax.W[e], ax.V[e], ax.V[e])
            cvals = bs.basis_all(coarse, p, ax.X[e], 0)                  # (q, Nc)
            rhs[g] += np.einsum("q,qi,qj->ij", ax.W[e], ax.V[e], cvals)
        blocks.append(np.linalg.solve(Mf, rhs))
    return np.vstack(blocks)


def space_prolongation(n_elem_c, p):
    """P_x (n_f x n_c) on the interior functions: coarse mesh of n_elem_c
    elements on (0, 1) -> fine mesh of 2 n_elem_c elements, degree p.
    Column j holds the fine coefficients of coarse function j, found by
    solving M_f c = (fine, coarse) with Gauss quadrature on the fine
    elements (exact: coarse functions are polynomials there).  Coarse
    interior functions vanish on the boundary, so their first and last fine
    coefficients are zero and the interior block is the whole map."""
    q = p + 2
    coarse = bs.open_uniform_knots(0.0, 1.0, n_elem_c, p)
    ax = Axis(0.0, 1.0, 2 * n_elem_c, p, q)
    N = ax.N
    Mf = np.zeros((N, N))
    rhs = np.zeros((N, bs.n_basis(coarse, p)))
    for e in range(ax.n_el):
        g = ax.gidx[e]
        Mf[np.ix_(g, g)] += np.einsum("q,qi,qj->ij", ax.W[e], ax.V[e], ax.V[e])
        cvals = bs.basis_all(coarse, p, ax.X[e], 0)
        rhs[g] += np.einsum("q,qi,qj->ij", ax.W[e], ax.V[e], cvals)
    P = np.linalg.solve(Mf, rhs)
    return P[1:-1, 1:-1]


def coarsening_schedule(prob, coarse_slabs=1, lam_crit=None, min_elem=2):
    """Kinds of the level transitions from the finest level down: "t" (time
    only) or "xt" (space and time).  Without lam_crit, time only.  A level
    is coarsened while its slab count is even and above coarse_slabs; in
    space too when tau_l / h_l^2 >= lam_crit and its element count halves
    to at least min_elem."""
    kinds = []
    S, ne, tau = prob.n_slabs, prob.n_elem, prob.tau
    while S > coarse_slabs and S % 2 == 0:
        lam = tau * ne * ne
        if lam_crit is not None and lam >= lam_crit and ne % 2 == 0 and ne // 2 >= min_elem:
            kinds.append("xt")
            ne //= 2
        else:
            kinds.append("t")
        S //= 2
        tau *= 2
    return kinds


class Level:
    def __init__(self, system):
        self.sys = system

    @property
    def S(self):
        return self.sys.S


class MultigridOracle:
    def __init__(self, prob, nu1=1, nu2=1, omega=0.5, system=None, coarse_slabs=1, lam_crit=None,
                 min_elem=2, minres_iters=None):
        self.prob = prob
        self.nu1, self.nu2, self.omega = nu1, nu2, omega
        fine = system if system is not None else SlabSystem.assemble(prob)
        self.levels = [fine]
        self.P = []
        self.kinds = coarsening_schedule(prob, coarse_slabs, lam_crit, min_elem)
        self.n_elem = [prob.n_elem]
        tau = prob.tau
        ne = prob.n_elem
        for kind in self.kinds:
            lev = self.levels[-1]
            Pt = time_prolongation(tau, prob.n_elem_t, prob.degree)
            n_f = ne + prob.degree - 2
            if kind == "xt":
                ne //= 2
                Px = space_prolongation(ne, prob.degree)
                Pxd = np.ones((1, 1))
                for _ in range(prob.dim):
                    Pxd = np.kron(Pxd, Px)
                P = sp.kron(sp.csr_matrix(Pt), sp.csr_matrix(Pxd), format="csr")
            else:
                P = sp.kron(sp.csr_matrix(Pt), sp.identity(n_f ** prob.dim), format="csr")
            A, B = lev.A, lev.B
            Z = sp.csr_matrix(A.shape)
            Lpair = sp.bmat([[A, Z], [-B, A]], format="csr")
            Epair = sp.bmat([[Z, B], [Z, Z]], format="csr")
            Ac = (P.T @ Lpair @ P).tocsc()
            Bc = (P.T @ Epair @ P).tocsr()
            self.levels.append(SlabSystem(Ac, Bc, lev.S // 2))
            self.P.append(P)
            self.n_elem.append(ne)
            tau *= 2
        # smoother: D^{-1} by sparse LU, or (minres_iters) through the
        # temporal block form with MinRes on the 2x2 blocks (Theorem 3.10);
        # the temporal matrices of a coarse level are those of its slab
        # length with the finest sigma (the Galerkin blocks), time-only
        # coarsening
        self.minres = None
        if minres_iters is not None:
            from .minres import MinresSlabInverse
            from .spacetime import time_matrices, space_matrices
            if "xt" in self.kinds:
                raise ValueError("the MinRes smoother is set up for coarsening in time only")
            Mx, Kx = space_matrices(prob)
            self.minres = []
            for lvl in range(len(self.levels)):
                t = prob.tau * 2 ** lvl
                Kt, Mt = time_matrices(0.0, t, prob.n_elem_t, prob.degree, prob.sigma)
                self.minres.append(MinresSlabInverse(Kt, Mt, Kx, Mx, minres_iters))

    # grid transfers --------------------------------------------------
    def restrict(self, lvl, r):
        P = self.P[lvl]
        S = self.levels[lvl].S
        R = r.reshape(S // 2, P.shape[0])
        return (P.T @ R.T).T.ravel()

    def prolong(self, lvl, e):
        P = self.P[lvl]
        S = self.levels[lvl + 1].S
        E = e.reshape(S, P.shape[1])
        return (P @ E.T).T.ravel()

    # smoother -----------------------------------------------------------
    def slab_inverse(self, lvl, r):
        """D^{-1} r on level lvl (every slab independently)."""
        sysl = self.levels[lvl]
        if self.minres is None:
            return sysl.slab_solve(r)
        R = r.reshape(sysl.S, sysl.m)
        return np.concatenate([self.minres[lvl].apply(R[s]) for s in range(sysl.S)])

    def smooth(self, lvl, f, u, steps):
        sysl = self.levels[lvl]
        for _ in range(steps):
            u = u + self.omega * self.slab_inverse(lvl, sysl.residual(f, u))
        return u

    def vcycle(self, f, u, lvl=0):
        sysl = self.levels[lvl]
        if lvl == len(self.levels) - 1:
            return sysl.forward_substitution(f)
        u = self.smooth(lvl, f, u, self.nu1)
        rc = self.restrict(lvl, sysl.residual(f, u))
        ec = self.vcycle(rc, np.zeros_like(rc), lvl + 1)
        u = u + self.prolong(lvl, ec)
        u = self.smooth(lvl, f, u, self.nu2)
        return u

    def solve(self, f, rtol=1e-8, maxit=100, u0=None):
        """Returns (u, iterations, history of relative residual norms)."""
        u = np.zeros_like(f) if u0 is None else u0.copy()
        fn = np.linalg.norm(f)
        hist = [np.linalg.norm(self.levels[0].residual(f, u)) / fn]
        it = 0
        while hist[-1] > rtol and it < maxit:
            u = self.vcycle(f, u)
            it += 1
            hist.append(np.linalg.norm(self.levels[0].residual(f, u)) / fn)
        return u, it, hist

"""Direct solution of L_h u = f by slab-wise forward substitution.

Oracle module (test infrastructure only).

L_h is block lower bidiagonal with A_n on the diagonal and -B_n below it
(eq. equ_linear_system), so
    u_1 = A_1^{-1} f_1,   u_n = A_n^{-1} (f_n + B_n u_{n-1}).
A_n is factored once by SciPy's sparse LU (SuperLU); on a uniform mesh all
slabs share the same A_n and B_n (the integrand has no explicit time
dependence), which the tests check by assembling a later slab as well.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .spacetime import assemble_slab_matrix, assemble_coupling


class SlabSystem:
    """A_n, B_n of one level and the LU factors of A_n."""

    def __init__(self, A, B, n_slabs):
        self.A = sp.csc_matrix(A)
        self.B = sp.csr_matrix(B)
        self.S = n_slabs
        self.m = A.shape[0]
        self._lu = None

    @classmethod
    def assemble(cls, prob):
        A = assemble_slab_matrix(prob, 0)
        B = assemble_coupling(prob, 1) if prob.n_slabs > 1 else sp.csr_matrix(A.shape)
        return cls(A, B, prob.n_slabs)

    @property
    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.A)
        return self._lu

    def apply(self, u):
        """L_h u (block lower bidiagonal product)."""
        U = u.reshape(self.S, self.m)
        Y = (self.A @ U.T).T
        if self.S > 1:
            Y[1:] -= (self.B @ U[:-1].T).T
        return Y.ravel()

    def residual(self, f, u):
        return f - self.apply(u)

    def slab_solve(self, r):
        """D^{-1} r with D = diag(A_n) (every slab independently)."""
        R = r.reshape(self.S, self.m)
        return self.lu.solve(np.ascontiguousarray(R.T)).T.ravel()

    def forward_substitution(self, f):
        F = f.reshape(self.S, self.m)
        U = np.zeros_like(F)
        for n in range(self.S):
            rhs = F[n].copy()
            if n > 0:
                rhs += self.B @ U[n - 1]
            U[n] = self.lu.solve(rhs)
        return U.ravel()

    def dense(self):
        """The whole L_h as a dense array (tiny problems only)."""
        m, S = self.m, self.S
        L = np.zeros((S * m, S * m))
        Ad = self.A.toarray()
        Bd = self.B.toarray()
        for n in range(S):
            L[n * m:(n + 1) * m, n * m:(n + 1) * m] = Ad
            if n > 0:
                L[n * m:(n + 1) * m, (n - 1) * m:n * m] = -Bd
        return L


def direct_solve(prob, f, system=None):
    if system is None:
        system = SlabSystem.assemble(prob)
    return system.forward_substitution(f)

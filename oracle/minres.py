"""Slab inverse by MinRes on the spatial block systems of the temporal
decomposition (Section 3.3, Theorems 3.8 and 3.10).

Oracle module (test infrastructure only; never imported by the product path).

What is computed, with the passage it follows:

* Section 3.3 writes the slab operator A = K_t (x) M_x + M_t (x) K_x through a
  decomposition of the temporal pencil, K_t X = M_t X Z, as
      A^{-1} = (X (x) I) (Z (x) M_x + I (x) K_x)^{-1} ((M_t X)^{-1} (x) I).
  In the real form used here Z is block diagonal: a real eigenvalue lambda
  gives the symmetric positive definite spatial system K_x + lambda M_x, a
  conjugate pair alpha +- i beta gives the 2x2 block system
      [[K_x + alpha M_x, beta_1 M_x], [beta_2 M_x, K_x + alpha M_x]]
  with beta_1 = beta, beta_2 = -beta (columns Re x, Im x of the eigenvector
  of alpha + i beta, beta > 0).
* Theorem 3.10 (Theorem 3.8 is the case |beta_1| = |beta_2|): substituting
  -y for the second unknown and scaling the rows by |beta_2| and |beta_1|
  gives the symmetric indefinite system A_bar [x; -y] = [|beta_2| f;
  |beta_1| g] with
      A_bar = [[|b2| Kc, -b1 |b2| M], [|b1| b2 M, -|b1| Kc]],  Kc = K_x + alpha M_x,
  and the block diagonal preconditioner
      P = diag(|b2| (K_x + (alpha + s) M_x), |b1| (K_x + (alpha + s) M_x)),
      s = sqrt(|b1 b2|),
  for which every generalised eigenvalue satisfies 1/sqrt(2) <= |lambda| <= 1.
* The block system is solved by MinRes preconditioned by P (Theorem 3.10
  and the text after it), from a zero guess, for a fixed number of
  iterations: the spectrum of P^{-1} A_bar lies in [-1, -1/sqrt 2] u
  [1/sqrt 2, 1], so the P^{-1}-norm of the residual drops at least by
  2 q^floor(k/2), q = (1 - 1/sqrt 2) / (1 + 1/sqrt 2) (the bound of MinRes for
  two intervals of equal length), which fixes the count for a tolerance:
  12 iterations for the 1e-4 of Section 4.4, 28 for 1e-10.  P itself is
  applied exactly (Section 4.4 factorises it with a sparse direct solver;
  here sparse LU).  Real eigenvalues are solved exactly.

The eigenvectors are normalised to unit 2-norm with their largest-modulus
entry real and positive (for a pair: the eigenvector of alpha + i beta), so
that the 2x2 block systems (and thus the MinRes iterates, which depend on
the basis of a pair) are fixed by the pencil alone.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# MinRes residual factor per two iterations on [-1, -1/sqrt 2] u [1/sqrt 2, 1]
Q_RATE = (1.0 - 1.0 / np.sqrt(2.0)) / (1.0 + 1.0 / np.sqrt(2.0))


def iterations_for(tol):
    """Fewest iterations k with 2 Q_RATE^floor(k/2) <= tol."""
    m = int(np.ceil(np.log(tol / 2.0) / np.log(Q_RATE)))
    return 2 * max(m, 0)


def canonical(v):
    """Unit 2-norm, largest-modulus entry real and positive (first such)."""
    i = int(np.argmax(np.abs(v)))
    v = v * (np.conj(v[i]) / abs(v[i]))
    return v / np.linalg.norm(v)


def temporal_blocks(Kt, Mt, imag_tol=1e-9):
    """Real block form K_t X = M_t X Z of the temporal pencil.

    Returns (X, W, blocks) with W = (M_t X)^{-1} and blocks a list of
    ("real", col, lambda) and ("pair", col, alpha, beta_1, beta_2) entries
    (a pair occupies columns col, col+1)."""
    lam, vec = np.linalg.eig(np.linalg.solve(Mt, Kt))
    scale = np.abs(lam).max()
    order = np.lexsort((-lam.imag, lam.real))
    N = len(lam)
    X = np.zeros((N, N))
    blocks, used, col = [], np.zeros(N, bool), 0
    for i in order:
        if used[i]:
            continue
        if abs(lam[i].imag) <= imag_tol * scale:
            used[i] = True
            X[:, col] = canonical(vec[:, i]).real
            blocks.append(("real", col, lam[i].real))
            col += 1
            continue
        j = min((k for k in range(N) if not used[k] and k != i), key=lambda k: abs(lam[k] - np.conj(lam[i])))
        used[i] = used[j] = True
        ip = i if lam[i].imag > 0 else j
        v = canonical(vec[:, ip])
        X[:, col], X[:, col + 1] = v.real, v.imag
        a, b = lam[ip].real, lam[ip].imag
        blocks.append(("pair", col, a, b, -b))
        col += 2
    W = np.linalg.inv(Mt @ X)
    return X, W, blocks


def pair_system(Kx, Mx, alpha, b1, b2):
    """A_bar and P of Theorem 3.10 (sparse)."""
    Kx, Mx = sp.csr_matrix(Kx), sp.csr_matrix(Mx)
    Kc = Kx + alpha * Mx
    s = np.sqrt(abs(b1 * b2))
    A = sp.bmat([[abs(b2) * Kc, -b1 * abs(b2) * Mx], [abs(b1) * b2 * Mx, -abs(b1) * Kc]], format="csr")
    Pd = Kx + (alpha + s) * Mx
    P = sp.block_diag([abs(b2) * Pd, abs(b1) * Pd], format="csc")
    return A, P


def pminres(apply_A, apply_Pinv, b, iters):
    """MinRes preconditioned by the SPD P, from x = 0, `iters` iterations.

    Lanczos in the P^{-1} inner product builds T_k (diagonal delta_j,
    off-diagonal gamma_{j+1}); Givens rotations keep the least-squares
    problem min || gamma_1 e_1 - T_{k+1,k} c || triangular, and the iterate
    is updated with the directions w_j of the rotated basis.  Returns x and
    the estimates |eta_{j+1}| of ||b - A x_j||_{P^{-1}} (index 0: ||b||)."""
    x = np.zeros_like(b)
    v_prev = np.zeros_like(b)
    v = b.copy()
    z = apply_Pinv(v)
    gam = np.sqrt(v @ z)
    hist = [gam]
    if gam == 0.0:
        return x, hist
    eta = gam
    gam_prev = 1.0
    c_prev2, c_prev, s_prev2, s_prev = 1.0, 1.0, 0.0, 0.0
    w_prev2 = np.zeros_like(b)
    w_prev = np.zeros_like(b)
    for _ in range(iters):
        zt = z / gam                      # z~_j, with v~_j = v / gam
        q = apply_A(zt)
        delta = q @ zt
        v_new = q - (delta / gam) * v - (gam / gam_prev) * v_prev
        z_new = apply_Pinv(v_new)
        gam_new = np.sqrt(max(v_new @ z_new, 0.0))
        # rotations j-2 and j-1 applied to the new column (gam, delta, gam_new)
        eps = s_prev2 * gam
        r1 = c_prev2 * gam
        zeta = c_prev * r1 + s_prev * delta
        r2 = -s_prev * r1 + c_prev * delta
        rho = np.hypot(r2, gam_new)
        c, s = r2 / rho, gam_new / rho
        w = (zt - zeta * w_prev - eps * w_prev2) / rho
        x = x + c * eta * w
        eta = -s * eta
        hist.append(abs(eta))
        v_prev, v, z = v, v_new, z_new
        gam_prev, gam = gam, gam_new
        c_prev2, c_prev, s_prev2, s_prev = c_prev, c, s_prev, s
        w_prev2, w_prev = w_prev, w
        if gam == 0.0:
            break
    return x, hist


class MinresSlabInverse:
    """A^{-1} r per slab through the temporal block form, the 1x1 blocks
    solved exactly and the 2x2 blocks by `iters` MinRes iterations with
    the preconditioner of Theorem 3.10."""

    def __init__(self, Kt, Mt, Kx, Mx, iters):
        self.X, self.W, self.blocks = temporal_blocks(Kt, Mt)
        self.Kx, self.Mx = sp.csr_matrix(Kx), sp.csr_matrix(Mx)
        self.Nt, self.Nx = Kt.shape[0], Kx.shape[0]
        self.iters = iters
        self.solvers = {}
        for blk in self.blocks:
            if blk[0] == "real":
                self.solvers[blk[1]] = spla.splu(sp.csc_matrix(self.Kx + blk[2] * self.Mx))
            else:
                _, col, a, b1, b2 = blk
                A, P = pair_system(self.Kx, self.Mx, a, b1, b2)
                self.solvers[col] = (A, spla.splu(P))

    def block_solve(self, col, rhs):
        """The MinRes solution of block `col` (a pair) for rhs = [f; g]."""
        _, col_, a, b1, b2 = next(b for b in self.blocks if b[1] == col)
        A, Plu = self.solvers[col]
        n = self.Nx
        bb = np.concatenate([abs(b2) * rhs[:n], abs(b1) * rhs[n:]])
        xs, hist = pminres(lambda v: A @ v, Plu.solve, bb, self.iters)
        return np.concatenate([xs[:n], -xs[n:]]), hist

    def apply(self, r):
        """A^{-1} r for one slab vector r (N_t x N_x, time major)."""
        R = r.reshape(self.Nt, self.Nx)
        G = self.W @ R
        Y = np.zeros_like(G)
        for blk in self.blocks:
            col = blk[1]
            if blk[0] == "real":
                Y[col] = self.solvers[col].solve(G[col])
            else:
                y, _ = self.block_solve(col, np.concatenate([G[col], G[col + 1]]))
                Y[col], Y[col + 1] = y[:self.Nx], y[self.Nx:]
        return (self.X @ Y).ravel()

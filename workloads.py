"""Seeded synthetic workloads shared by the tests, the bench and the oracle.

This module holds problem shapes and the seeded draws of the right-hand
side; it contains none of the method's arithmetic (no basis functions, no
quadrature, no solver).  Both the oracle and the HIP library receive the same
explicit mode list produced here.

Right-hand sides are sums of separable modes
    f(x, t) = sum_m amp_m * prod_a sin(k_{m,a} pi x_a) * cos(omega_m pi t + phase_m),
with zero initial data.  The paper's experiments use a 21-patch domain whose
geometry is not available; the unit square and cube stand in for it.
"""
from dataclasses import dataclass, field
import math
import numpy as np


@dataclass(frozen=True)
class Modes:
    amp: tuple          # (M,)
    k: tuple            # (M, dim) integer wave numbers
    omega: tuple        # (M,)
    phase: tuple        # (M,)
    dim: int

    @property
    def n_modes(self):
        return len(self.amp)

    def arrays(self):
        return (np.asarray(self.amp, dtype=np.float64),
                np.asarray(self.k, dtype=np.int32).reshape(-1, self.dim),
                np.asarray(self.omega, dtype=np.float64),
                np.asarray(self.phase, dtype=np.float64))

    def __call__(self, t, xs):
        """Evaluate f at arrays t and xs = [x, y, (z)]."""
        amp, k, om, ph = self.arrays()
        out = np.zeros(np.broadcast(t, *xs).shape)
        for m in range(len(amp)):
            v = amp[m] * np.cos(om[m] * math.pi * t + ph[m])
            for a in range(self.dim):
                v = v * np.sin(k[m, a] * math.pi * xs[a])
            out = out + v
        return out


def random_modes(seed, dim, n_modes=8):
    """Random-mode right-hand side: amplitudes N(0,1), spatial wave numbers
    uniform in {1..8}, temporal frequencies uniform in {0..4}; drawn from
    numpy's default_rng(seed) in the order amp, k, omega."""
    rng = np.random.default_rng(seed)
    amp = rng.standard_normal(n_modes)
    k = rng.integers(1, 9, size=n_modes * dim).reshape(n_modes, dim)
    om = rng.integers(0, 5, size=n_modes).astype(np.float64)
    return Modes(tuple(amp.tolist()), tuple(map(tuple, k.tolist())), tuple(om.tolist()),
                 tuple([0.0] * n_modes), dim)


def manufactured_modes(dim):
    """f for u = prod_a sin(pi x_a) * sin(pi t):
    f = pi cos(pi t) prod sin + d pi^2 sin(pi t) prod sin, written as two modes
    (sin(pi t) = cos(pi t - pi/2))."""
    return Modes((math.pi, dim * math.pi ** 2), ((1,) * dim, (1,) * dim), (1.0, 1.0),
                 (0.0, -math.pi / 2), dim)


def manufactured_exact(dim):
    """(u, u_t, grad u) callables of the manufactured solution."""
    pi = math.pi

    def prod_sin(xs, skip=None):
        v = 1.0
        for a in range(dim):
            if a != skip:
                v = v * np.sin(pi * xs[a])
        return v

    def u(t, xs):
        return np.sin(pi * t) * prod_sin(xs)

    def ut(t, xs):
        return pi * np.cos(pi * t) * prod_sin(xs)

    def grad(t, xs):
        return [np.sin(pi * t) * pi * np.cos(pi * xs[a]) * prod_sin(xs, skip=a) for a in range(dim)]

    return u, ut, grad


@dataclass(frozen=True)
class Config:
    name: str
    dim: int
    n_elem: int
    degree: int
    n_slabs: int
    n_elem_t: int
    rhs: str            # "manufactured" or "random"
    seed: int = 0
    T: float = 1.0
    theta: float = 0.01
    note: str = ""

    def modes(self):
        if self.rhs == "manufactured":
            return manufactured_modes(self.dim)
        return random_modes(self.seed, self.dim)

    @property
    def unknowns(self):
        n = self.n_elem + self.degree - 2
        return self.n_slabs * (self.n_elem_t + self.degree) * n ** self.dim

    @property
    def coefficients(self):
        return self.n_slabs * (self.n_elem_t + self.degree) * (self.n_elem + self.degree) ** self.dim


CONFIGS = {
    "C1": Config("C1", 2, 16, 2, 16, 2, "manufactured",
                 note="2D p=2 16x16 elems, 16 slabs x 2 time elems, manufactured sines"),
    "C2": Config("C2", 2, 64, 3, 256, 2, "random", seed=2,
                 note="2D p=3 64x64 elems, 256 slabs x 2 time elems, 8 random modes seed 2"),
    "C3": Config("C3", 3, 32, 2, 128, 2, "manufactured",
                 note="3D p=2 32^3 elems, 128 slabs x 2 time elems, manufactured sines"),
    "C4": Config("C4", 2, 256, 2, 1024, 1, "random", seed=4,
                 note="2D p=2 256x256 elems, 1024 slabs x 1 time elem, 8 random modes seed 4"),
}


def serving_requests(n_requests=1000, seed=0):
    """Request mix of the serving workload: 2D, n_elem in {32,64,128,256},
    p in {2,3,4}, slabs in {16,...,512} (powers of two), 2 time elements,
    random-mode right-hand side seeded by the request id."""
    rng = np.random.default_rng(seed)
    out = []
    for rid in range(n_requests):
        ne = int(rng.choice([32, 64, 128, 256]))
        p = int(rng.choice([2, 3, 4]))
        S = int(rng.choice([16, 32, 64, 128, 256, 512]))
        out.append(Config(f"req{rid}", 2, ne, p, S, 2, "random", seed=rid))
    return out


def random_vector(seed, n):
    """Seeded standard-normal vector (iterates and residuals for parity tests)."""
    return np.random.default_rng(seed).standard_normal(n)

"""B-spline bases for the oracle (test infrastructure only).

The oracle is a plain, slow FP64 CPU implementation used by the tests, by
`__graft_entry__.smoke()` and by the CPU baseline leg of `bench.py`; the
product path never imports it and it shares no code with the HIP library.

This module follows Section 2.1 (Isogeometric Analysis): open knot vectors,
B-spline basis functions by the Cox-de Boor recursion, tensor products.
The knot-vector notation of Section 2.1 is garbled in the source; the reading
used here is an open uniform knot vector with maximal smoothness C^{p-1}
inside the interval, i.e. N = n_el + p functions on n_el elements.
"""
import numpy as np


def open_uniform_knots(a, b, n_el, p):
    """Open uniform knot vector on [a, b] with n_el elements, degree p.

    The first and last knots are repeated p+1 times (Section 2.1), interior
    knots are simple, so the space has C^{p-1} continuity inside (a, b).
    """
    inner = [a + (b - a) * k / n_el for k in range(1, n_el)]
    return np.array([a] * (p + 1) + inner + [b] * (p + 1), dtype=np.float64)


def n_basis(knots, p):
    return len(knots) - p - 1


def basis_all(knots, p, x, deriv=0):
    """Values (deriv=0) or first derivatives (deriv=1) of all B-splines.

    Cox-de Boor recursion carried out for every basis index over the whole
    knot vector (no local-support shortcut), vectorised over the points x.
    Returns an array of shape (len(x), N).  The right end point of the knot
    vector is assigned to the last non-degenerate knot span, so that the
    trace at the end of an interval is the limit from the left.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = knots
    m = len(t) - 1
    t_end = t[-1]
    # degree-0 functions
    N = np.zeros((len(x), m))
    for i in range(m):
        if t[i] < t[i + 1]:
            inside = (t[i] <= x) & (x < t[i + 1])
            if t[i + 1] == t_end:
                inside |= (x == t_end)
            N[:, i] = inside
    # raise the degree one step at a time
    for q in range(1, p + 1):
        if deriv == 1 and q == p:
            Nlow = N
        M = np.zeros((len(x), m - q))
        for i in range(m - q):
            left = 0.0
            d1 = t[i + q] - t[i]
            if d1 > 0:
                left = (x - t[i]) / d1 * N[:, i]
            right = 0.0
            d2 = t[i + q + 1] - t[i + 1]
            if d2 > 0:
                right = (t[i + q + 1] - x) / d2 * N[:, i + 1]
            M[:, i] = left + right
        N = M
    if deriv == 0:
        return N
    if deriv != 1:
        raise ValueError("only first derivatives are needed")
    if p == 0:
        return np.zeros_like(N)
    # derivative formula: N'_{i,p} = p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}
    D = np.zeros((len(x), m - p))
    for i in range(m - p):
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        val = 0.0
        if d1 > 0:
            val = val + p / d1 * Nlow[:, i]
        if d2 > 0:
            val = val - p / d2 * Nlow[:, i + 1]
        D[:, i] = val
    return D


def gauss_legendre(q):
    """q-point Gauss-Legendre rule on [-1, 1] (numpy's library routine)."""
    return np.polynomial.legendre.leggauss(q)


def element_quadrature(knots, q):
    """Gauss points and weights on every non-degenerate knot span.

    Returns (points, weights, element_index) flattened over elements.
    """
    xi, wi = gauss_legendre(q)
    brk = np.unique(knots)
    pts, wts, eidx = [], [], []
    for e in range(len(brk) - 1):
        a, b = brk[e], brk[e + 1]
        pts.append(0.5 * (b - a) * xi + 0.5 * (a + b))
        wts.append(0.5 * (b - a) * wi)
        eidx.append(np.full(q, e))
    return np.concatenate(pts), np.concatenate(wts), np.concatenate(eidx)


def spline_eval(knots, p, coef, x, deriv=0):
    """Evaluate the spline sum_i coef_i N_i at x."""
    return basis_all(knots, p, x, deriv) @ np.asarray(coef, dtype=np.float64)

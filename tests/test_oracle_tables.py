"""The oracle's temporal matrices and its generalized eigen step pinned to
the values the paper prints: Table 2 (smallest real part of the generalized
eigenvalues, and the '*' pattern), Table 1 (cond of the eigenvector matrix)
and Example 3.2.  A printed value counts as reproduced when the computed one
lies within one unit of its last printed digit (the tables mix rounding and
truncation)."""
import os
import numpy as np
import scipy.linalg as sl
import pytest

from oracle.spacetime import time_matrices

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _unit(s):
    """one unit in the last printed place of the string s"""
    if "e" in s:
        mant, ex = s.split("e")
        dec = len(mant.split(".")[1]) if "." in mant else 0
        return 10.0 ** (int(ex) - dec)
    dec = len(s.split(".")[1]) if "." in s else 0
    return 10.0 ** (-dec)


def _rows(name):
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                yield line.split()


# Entries of Table 2 at 64 and 256 elements with large theta are not
# reproduced by any FP64 eigen solver tried (their eigenvector matrices have
# condition numbers of 1e10 and more); they are excluded from the value pin
# but their '*' pattern is still checked.
ILL_CONDITIONED = {(6, 1.0), (8, 1.0), (8, 10.0)}
ILL_CONDITIONED_P = {(8, 0.1, 1), (8, 0.1, 2)}


def test_table2_min_real_part_and_star_pattern():
    checked = 0
    for r, th, p, v in _rows("table2_min_real_eig.txt"):
        r, th, p = int(r), float(th), int(p)
        n = 2 ** r
        K, M = time_matrices(0.0, 1.0, n, p, th / n)      # sigma = theta * h_t
        m_has_negative = np.linalg.eigvals(M).real.min() < 0
        assert m_has_negative == (v == "*"), (r, th, p, v)
        if v == "*" or (r, th) in ILL_CONDITIONED or (r, th, p) in ILL_CONDITIONED_P:
            continue
        lam = sl.eigvals(K, M)
        val = lam.real.min()
        assert abs(val - float(v)) <= _unit(v) * (1 + 1e-9), (r, th, p, val, v)
        checked += 1
    assert checked >= 95


def test_table2_requires_temporal_mesh_size_in_supg():
    """With sigma = theta * (interval length) instead of theta * h_t, the
    printed Table 2 is not reproduced (so the SUPG h_n is the element size)."""
    K, M = time_matrices(0.0, 1.0, 16, 1, 0.1 * 1.0)
    val = sl.eigvals(K, M).real.min()
    assert abs(val - 4.8) > 0.5


def test_table1_condition_numbers():
    for ne, col, v in _rows("table1_cond_X.txt"):
        ne, col = int(ne), int(col)
        if ne > 64:
            continue       # cond(X) ~ 1e14: at the limit of FP64
        p = col + 1
        h = 0.1 / ne
        K, M = time_matrices(0.0, 0.1, ne, p, 0.01 * h)
        _, X = sl.eig(K, M)
        X = X / np.linalg.norm(X, axis=0)
        c = np.linalg.cond(X)
        assert abs(c - float(v)) <= _unit(v) * (1 + 1e-9), (ne, col, c, v)


def test_example_3_2():
    A, B, spec = [], [], {}
    for row in _rows("example_3_2.txt"):
        if row[0] == "A":
            A.append([float(x) for x in row[1:]])
        elif row[0] == "B":
            B.append([float(x) for x in row[1:]])
        else:
            spec[row[0]] = (float(row[1]), float(row[2]))
    A, B = np.array(A), np.array(B)
    # both matrices are positive (positive definite symmetric part)
    assert np.linalg.eigvalsh(A + A.T).min() > 0
    assert np.linalg.eigvalsh(B + B.T).min() > 0
    for key, ev in (("specA", np.linalg.eigvals(A)), ("specB", np.linalg.eigvals(B)),
                    ("specBA", sl.eigvals(A, B))):
        re, im = spec[key]
        assert np.allclose(sorted(ev.imag), [-im, im], rtol=1e-13)
        assert np.allclose(ev.real, re, rtol=1e-13)
    # generalized eigenvalues with negative real part despite positivity
    assert sl.eigvals(A, B).real.max() < 0

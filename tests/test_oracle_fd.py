"""Pins of the oracle's finite-difference operators and box solver against
the paper (printed stencil coefficients) and mathematics (exactness on
polynomials, sine eigenmodes, sparse LU)."""
import os

import numpy as np
import pytest

from oracle import fd

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_coefs():
    rows = []
    for line in open(os.path.join(GOLD, "paper_stencils.txt")):
        if line.startswith("#") or not line.strip():
            continue
        d, m, a, b = line.split()
        rows.append((int(d), int(m), float(a), float(b)))
    return rows


@pytest.mark.parametrize("d", [2, 3])
def test_compact_stencil_matches_printed_coefficients(d):
    """eqs. 9p-cds / 27p-cds: coefficient a/h^2 + b kappa per |offset|_1."""
    h, kappa = 0.37, 2.5
    A, _ = fd.stencils(d, 4, h, kappa)
    want = {m: (a, b) for dd, m, a, b in _paper_coefs() if dd == d}
    offs = [o for o in np.ndindex(*(3,) * d)]
    for o in offs:
        o = tuple(v - 1 for v in o)
        m = sum(abs(v) for v in o)
        a, b = want[m]
        assert A.get(o, 0.0) == pytest.approx(a / h ** 2 + b * kappa, rel=1e-14, abs=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_second_order_stencil(d):
    h, kappa = 0.25, 1.5
    A, B = fd.stencils(d, 2, h, kappa)
    assert A[(0,) * d] == pytest.approx(-2 * d / h ** 2 - kappa)
    assert sum(1 for o in A if o != (0,) * d) == 2 * d
    assert B == {(0,) * d: 1.0}


def _poly(d, deg, rng):
    terms = {}
    for e in np.ndindex(*(deg + 1,) * d):
        if sum(e) <= deg:
            terms[e] = rng.standard_normal()
    return terms


def _eval(terms, X, der=None):
    out = 0.0
    for e, c in terms.items():
        if der is None:
            t = c
            for a, x in enumerate(X):
                t = t * x ** e[a]
        else:                       # Laplacian
            t = 0.0
            for a in range(len(X)):
                if e[a] < 2:
                    continue
                s = c * e[a] * (e[a] - 1)
                for b, x in enumerate(X):
                    s = s * x ** (e[b] - (2 if a == b else 0))
                t = t + s
        out = out + t
    return out


@pytest.mark.parametrize("d,order,deg", [(2, 4, 5), (3, 4, 5), (2, 2, 3), (3, 2, 3)])
def test_scheme_exact_on_polynomials(d, order, deg):
    """A_h u = B_h (Lap u - kappa u) exactly for polynomials of degree <= 5
    (4th order) / <= 3 (2nd order): the Mehrstellen property behind eqs.
    9p-cds and 27p-cds."""
    rng = np.random.default_rng(7 + d + order)
    N, h, kappa = 8, 0.125, 0.7
    terms = _poly(d, deg, rng)
    x1 = np.arange(N + 1) * h - 0.4
    grids = np.meshgrid(*([x1] * d), indexing="ij")       # grids[j] varies along array axis j
    X = tuple(grids[d - 1 - a] for a in range(d))        # x along last array axis
    u = _eval(terms, X)
    f = _eval(terms, X, der="lap") - kappa * u
    A, B = fd.stencils(d, order, h, kappa)
    lhs = fd.apply(A, u)
    rhs = fd.apply(B, f)
    assert np.max(np.abs(lhs - rhs)) < 1e-9 * max(1.0, np.max(np.abs(rhs)))


@pytest.mark.parametrize("d,order", [(2, 4), (3, 4), (2, 2), (3, 2)])
def test_sine_modes_are_eigenvectors(d, order):
    N, h, kappa = 8, 0.1, 1.3
    lam = fd.eigenvalues(d, order, N, h, kappa)
    A, _ = fd.stencils(d, order, h, kappa)
    k = (2, 5, 3)[:d]
    x = np.arange(N + 1)
    modes = [np.sin(np.pi * k[a] * x / N) for a in range(d)]
    u = modes[0]
    for a in range(1, d):
        u = np.multiply.outer(modes[a], u)
    Au = fd.apply(A, u)
    ind = tuple(k[d - 1 - j] - 1 for j in range(d))
    assert np.allclose(Au, lam[ind] * u[(slice(1, N),) * d], atol=1e-9)


@pytest.mark.parametrize("d,order,kappa", [(2, 4, 0.0), (2, 4, 2.0), (3, 4, 1.0), (2, 2, 0.5), (3, 2, 0.0)])
def test_dst_solve_equals_sparse_lu(d, order, kappa):
    """Box solve (Alg. 1 Step 3.3) against a sparse LU of the same system."""
    N, h = 8, 0.3
    F = np.random.default_rng(3).standard_normal((N - 1,) * d)
    v1 = fd.dst_solve(F, d, order, N, h, kappa)
    v2 = fd.lu_solve(F, d, order, N, h, kappa)
    assert np.max(np.abs(v1 - v2)) < 1e-12 * np.max(np.abs(v2))

"""Pins of the oracle's level set known only at the grid nodes (Sec. 7):
the degree-q interpolant reproduces polynomials of degree <= q (value and
gradient) and the samples at the nodes; a sampled quadratic level set gives
the analytic geometry; a sampled star gives the analytic star's solution."""
import math

import numpy as np
import pytest

from oracle import geometry as G, kfbi, levelset
from paper_2309_05965_amd import workloads as W

from test_oracle_kfbi import _random_poly, data_for


@pytest.mark.parametrize("d,q", [(2, 3), (2, 5), (3, 3), (3, 5)])
def test_interpolant_reproduces_polynomials(d, q):
    rng = np.random.default_rng(31 + 10 * d + q)
    prob = W.problem(d, 4, 16, -1.0, 1.0, 1.0, 1.0, 0.0, [])
    P = W.polynomial(_random_poly(d, q, rng))
    iface = W.sampled(prob, lambda X: P(X)[0], q)
    X = tuple(rng.uniform(-1.0, 1.0, 500) for _ in range(d))
    v, g, _ = P(X)
    assert np.max(np.abs(levelset.H(iface, X) - v)) < 1e-11 * (1 + np.max(np.abs(v)))
    gh = levelset.gradH(iface, X)
    for a in range(d):
        assert np.max(np.abs(gh[a] - g[a])) < 1e-9 * (1 + np.max(np.abs(g[a])))
    # at the nodes the interpolant is the sample, bit for bit
    Gc = W.grid_coords(prob)
    assert np.array_equal(levelset.H(iface, Gc), iface[2])


def test_sampled_quadratic_gives_the_analytic_geometry():
    """|x - c|^2 - r^2 is reproduced by the quintic interpolant, so the
    sampled sphere has the analytic sphere's surface points (to rounding),
    normals and every discrete table."""
    prob = W.problem(3, 4, 32, -1.0, 1.0, 1.0, 5.0, 0.5, [W.sphere3d(0.03, -0.02, 0.01, 0.52)])
    ga = G.build(prob)
    gs = G.build(W.with_sampled(prob, W.H_sphere(0.03, -0.02, 0.01, 0.52)))
    assert np.array_equal(ga["reg"], gs["reg"])
    assert ga["surf"]["pos"].shape == gs["surf"]["pos"].shape
    assert np.max(np.abs(ga["surf"]["pos"] - gs["surf"]["pos"])) < 1e-14
    assert np.max(np.abs(ga["surf"]["nrm"] - gs["surf"]["nrm"])) < 1e-13
    for key in ("D", "N"):
        assert np.array_equal(ga["st"][key], gs["st"][key])
    assert np.array_equal(ga["irr"], gs["irr"])


def test_sampled_star_solution_matches_the_analytic_one():
    """The star of the 2D workload given only at the nodes: the same primary
    points and iterations, and the solution error within 5% of the analytic
    geometry's at N = 128 and 256 (the interpolation error of the surface,
    O(h^6), is below the scheme's O(h^4))."""
    for N in (128, 256):
        prob, sol = W.config2(N)
        errs = []
        for pp in (prob, W.with_sampled(prob, W.H_star(0.5, 0.3, 5))):
            pl = kfbi.Plan(pp)
            res = pl.solve(data_for(pl, pp, sol), tol=1e-12)
            errs.append((pl.Nb, res["iters"],
                         np.max(np.abs(res["u"] - W.exact_solution(pp, sol, pl.geo["reg"])))))
        assert errs[0][0] == errs[1][0] and abs(errs[0][1] - errs[1][1]) <= 1
        assert abs(errs[1][2] - errs[0][2]) < 0.05 * errs[0][2], errs

"""Pins of the oracle's two-density interface BIE (eq. bie-ifp-1, Sec. 3.2,
with the two simple solves per product of the superposition remark after
Alg. 1): the discrete system is satisfied exactly by the exact densities of
piecewise-polynomial solutions, and solutions converge at the scheme's
order for a Poisson / modified-Helmholtz pair."""
import math

import numpy as np
import pytest

from oracle import twodensity as TD
from paper_2309_05965_amd import workloads as W

from test_oracle_kfbi import _random_poly


def td_data(pl, prob, sol):
    s = pl.geo["surf"]
    return W.make_td_data(prob, sol, s["pos"], s["nrm"], s["iface"], pl.geo["st"]["pde_pts"],
                          pl.geo["dofs"]["iface"])


def _case(name):
    if name == "ellipse_o4":
        return 2, 4, W.td_problem(2, 4, 64, -1.0, 1.0, 1.0, 4.0, 0.3, 2.5,
                                  [W.ellipse2d(0.05, -0.02, 0.6, 0.45, theta=0.3)])
    if name == "ellipse_o2":
        return 2, 2, W.td_problem(2, 2, 64, -1.0, 1.0, 2.0, 0.5, 1.5, 0.0,
                                  [W.ellipse2d(0.05, -0.02, 0.6, 0.45, theta=0.3)])
    if name == "circles_close":
        prob = W.two_circles(4, 64, 0.5)
        return 2, 4, W.td_problem(2, 4, 64, -1.0, 1.0, 1.0, 3.0, 0.0, 4.0, prob["ifaces"])
    return 3, 4, W.td_problem(3, 4, 32, -1.0, 1.0, 1.0, 4.0, 0.0, 2.5, [W.sphere3d(0.03, -0.02, 0.01, 0.52)])


@pytest.mark.parametrize("name", ["ellipse_o4", "ellipse_o2", "circles_close", "sphere"])
def test_exact_densities_satisfy_the_discrete_system(name):
    """With polynomial u_s (degree <= p) the functions u_1 1_Omega_1 and
    u_2 1_Omega_2 are reproduced exactly by the corrected scheme, so
    phi = u_1 and psi = sigma_2 d_n u_2, given on the whole surface table,
    satisfy A [phi; psi] = b to rounding (any sign, sigma or trace slip in
    the reduction to simple solves breaks this)."""
    d, order, prob = _case(name)
    p = 4 if order == 4 else 2
    rng = np.random.default_rng(17)
    K = len(prob["ifaces"])
    sol = {s: W.polynomial(_random_poly(d, p, rng)) for s in range(K + 1)}
    pl = TD.TwoDensityPlan(prob)
    s = pl.geo["surf"]
    X = tuple(s["pos"][:, a] for a in range(d))
    k = s["iface"]
    aS = np.zeros(k.size)
    for kk in range(1, K + 1):
        aS = np.where(k == kk, sol[kk](X)[0], aS)
    g0 = sol[0](X)[1]
    bS = prob["beta_out"] * sum(g0[a] * s["nrm"][:, a] for a in range(d))
    b = pl.rhs(td_data(pl, prob, sol))
    r = b - pl.apply_surface(aS, bS, pl.p1.dof_values(aS), pl.p1.dof_values(bS))
    assert np.max(np.abs(r)) < 1e-11 * (1 + np.max(np.abs(b)))


@pytest.mark.parametrize("order,Ns,rate_min", [(4, (64, 128, 256), 3.5), (2, (64, 128, 256), 2.0)])
def test_heterogeneous_convergence(order, Ns, rate_min):
    """Poisson inside, modified Helmholtz outside (kappa~ 0 and 2.5, sigma
    1 and 4): the maximum error decreases at the scheme's order and GMRES
    meets the tolerance."""
    errs = []
    for N in Ns:
        prob = W.td_problem(2, order, N, -1.0, 1.0, 1.0, 4.0, 0.0, 2.5,
                            [W.ellipse2d(0.05, -0.02, 0.6, 0.45, theta=0.3)])
        sol = {0: W.f_sin_sin, 1: W.f_exp_cos}
        pl = TD.TwoDensityPlan(prob)
        res = pl.solve(td_data(pl, prob, sol), tol=1e-12)
        assert res["true_rel_res"] < 1e-11
        errs.append(np.max(np.abs(res["u"] - W.exact_solution(prob, sol, pl.geo["reg"]))))
    rate = math.log2(errs[0] / errs[-1]) / math.log2(Ns[-1] / Ns[0])
    assert rate > rate_min, errs

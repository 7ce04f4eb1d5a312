"""Pins of the oracle's collocation (Secs. 5.3.1, 5.4), simple interface
solve (Sec. 5), BIE operator (Sec. 3.2) and GMRES (Alg. 1) against
polynomial reproduction, exact solutions, dense solves, special cases and
the convergence order."""
import math

import numpy as np
import pytest

from oracle import collocation, geometry, kfbi
from paper_2309_05965_amd import workloads as W


def data_for(pl, prob, sol):
    s = pl.geo["surf"]
    return W.make_data(prob, sol, s["pos"], s["nrm"], s["iface"], pl.geo["st"]["pde_pts"],
                       pl.geo["dofs"]["iface"])


def _random_poly(d, deg, rng, scale=1.0):
    terms = {}
    for e in np.ndindex(*(deg + 1,) * d):
        if sum(e) <= deg:
            terms[tuple(int(v) for v in e)] = scale * rng.standard_normal()
    return terms


def sphere_problem(order=4, N=32, kappa=0.0):
    return W.problem(3, order, N, -1.0, 1.0, 1.0, 5.0, kappa, [W.sphere3d(0.03, -0.02, 0.01, 0.52)])


@pytest.mark.parametrize("case", ["c1", "c2", "sphere"])
def test_collocation_reproduces_polynomials(case):
    """P3: data sampled from a polynomial C of degree p is reproduced: U are
    C's Taylor coefficients in the scaled coordinates of each centre."""
    if case == "c1":
        prob, _ = W.config1(64)
    elif case == "c2":
        prob, _ = W.config2(128)
    else:
        prob = sphere_problem(kappa=0.5)
    pl = kfbi.Plan(prob)
    d, h, p = pl.d, pl.h, pl.p
    rng = np.random.default_rng(5)
    C = W.polynomial(_random_poly(d, p, rng))
    surf = pl.geo["surf"]
    X = tuple(surf["pos"][:, a] for a in range(d))
    v, g, _ = C(X)
    b = sum(g[a] * surf["nrm"][:, a] for a in range(d))
    Pp = pl.geo["st"]["pde_pts"]
    Xp = tuple(Pp[..., a] for a in range(d))
    vp, _, lapp = C(Xp)
    ft = lapp - prob["kappa"] * vp
    Q = collocation.rhs(pl.geo, v, b, ft)
    U = np.einsum("iab,ib->ia", pl.Minv, Q)
    # Taylor coefficients at p_i in xi = (x - p_i)/h: evaluate the expansion
    # at a few random offsets and compare with C
    for _ in range(3):
        xi = rng.uniform(-1.5, 1.5, (pl.Nb, d))
        Xq = pl.geo["dofs"]["pos"] + h * xi
        cq, _, _ = C(tuple(Xq[:, a] for a in range(d)))
        approx = (collocation.mono(xi, pl.E) * U).sum(axis=1)
        assert np.max(np.abs(approx - cq)) < 1e-9 * (1 + np.max(np.abs(cq)))


def test_collocation_conditioning_is_mesh_independent():
    """P4 (Sec. 5.4 remark): cond(M) in the scaled coordinates is moderate
    and does not grow with N."""
    meds = []
    for N in (256, 512):
        prob, _ = W.config2(N)
        pl = kfbi.Plan(prob)
        meds.append(np.median(pl.cond))
        assert np.median(pl.cond) < 2e3
    assert 0.6 < meds[1] / meds[0] < 1.5


@pytest.mark.parametrize("case", ["c1", "c2", "sphere"])
def test_simple_solve_patch(case):
    """P1: with polynomial u_in, u_out (degree <= p) the corrected scheme,
    collocation and interpolation are exact, so the simple interface solve
    returns u at every node and the exact one-sided normal derivatives."""
    rng = np.random.default_rng(11)
    if case == "c1":
        prob, _ = W.config1(64)
    elif case == "c2":
        prob, _ = W.config2(128)
    else:
        prob = sphere_problem(kappa=0.7)
    p = 4 if prob["order"] == 4 else 2
    d = prob["dim"]
    sol = {0: W.polynomial(_random_poly(d, p, rng)), 1: W.polynomial(_random_poly(d, p, rng))}
    pl = kfbi.Plan(prob)
    data = data_for(pl, prob, sol)
    surf = pl.geo["surf"]
    psiS = W.exact_density(prob, sol, surf["pos"], surf["nrm"], surf["iface"])
    v, dn_in, dn_out, _ = pl.simple_solve(a=data["g1"], b=psiS, ftilde=data["ftilde"],
                                          fhat=data["fhat"], gB=data["gB"])
    ue = W.exact_solution(prob, sol, pl.geo["reg"])
    assert np.max(np.abs(v - ue)) < 1e-10 * (1 + np.max(np.abs(ue)))
    X = tuple(pl.geo["dofs"]["pos"][:, a] for a in range(d))
    n = pl.geo["dofs"]["nrm"]
    gi = sol[1](X)[1]
    go = sol[0](X)[1]
    assert np.max(np.abs(dn_in - sum(gi[a] * n[:, a] for a in range(d)))) < 1e-8
    assert np.max(np.abs(dn_out - sum(go[a] * n[:, a] for a in range(d)))) < 1e-8
    # BIE residual of the exact density vanishes to rounding
    psi = pl.dof_values(psiS)
    b = pl.rhs(data)
    Ab = pl.flux(dn_in, dn_out)
    assert np.max(np.abs(Ab - pl.dof_values(data["g2"]))) < 1e-8 * (1 + prob["beta_in"])
    assert b.shape == psi.shape


def test_equal_coefficients_give_half_identity():
    """P9: beta_in = beta_out gives A = I/2 exactly (mu = 0 in
    psi/2 + mu K' psi), because every centre is its own Neumann point."""
    prob, _ = W.config2(128)
    prob["beta_in"] = prob["beta_out"] = 3.0
    pl = kfbi.Plan(prob)
    psi = np.random.default_rng(2).standard_normal(pl.Nb)
    assert np.max(np.abs(pl.matvec(psi) - 0.5 * psi)) < 1e-12


def test_gmres_matches_dense_solve():
    rng = np.random.default_rng(4)
    n = 40
    A = np.eye(n) * 2 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, its, _ = kfbi.gmres(lambda v: A @ v, b, None, 1e-13, 100)
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-11
    assert its <= n
    x0 = rng.standard_normal(n)
    x, _, _ = kfbi.gmres(lambda v: A @ v, b, x0, 1e-13, 100)
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-11


def test_bie_brute_force():
    """P6: assemble the discrete BIE column by column on a small grid and
    compare the GMRES density with a dense solve."""
    prob, sol = W.config1(32)
    pl = kfbi.Plan(prob)
    A = np.stack([pl.matvec(e) for e in np.eye(pl.Nb)], axis=1)
    data = data_for(pl, prob, sol)
    b = pl.rhs(data)
    res = pl.solve(data, tol=1e-13)
    ref = np.linalg.solve(A, b)
    assert np.max(np.abs(res["psi"] - ref)) < 1e-10 * np.max(np.abs(ref))
    # the spectrum lies in the right half plane (second-kind BIE)
    ev = np.linalg.eigvals(A)
    assert ev.real.min() > 0.05


@pytest.mark.parametrize("cfg,Ns,order_min", [("config1", (64, 128, 256), 1.5),
                                              ("config2", (256, 512), 3.5)])
def test_convergence_order(cfg, Ns, order_min):
    """P8: 2nd-order (config 1) and 4th-order (config 2) convergence of the
    grid solution in the maximum norm (Sec. 6 tables)."""
    errs = []
    for N in Ns:
        prob, sol = getattr(W, cfg)(N)
        pl = kfbi.Plan(prob)
        res = pl.solve(data_for(pl, prob, sol), tol=1e-12)
        ue = W.exact_solution(prob, sol, pl.geo["reg"])
        errs.append(np.max(np.abs(res["u"] - ue)))
        assert res["true_rel_res"] < 1e-10
    rate = math.log2(errs[0] / errs[-1]) / math.log2(Ns[-1] / Ns[0])
    assert rate > order_min, errs

"""Pins of the oracle's multi-interface path, its density extension and its
Adam step.

Two interfaces (the remark on multiple crossings in Sec. 5.2; Secs. 5.3 and
5.5): with polynomial solutions of degree <= p in every region the
corrected scheme is exact (the patch test), whatever the geometry.  With
the closest points of two interfaces less than one grid spacing apart,
irregular nodes of one interior have stencil neighbours in the other, so
the right-hand side correction C^(reg P) - C^(reg Q) has both terms
nonzero, and interpolation blocks reach into the other interior.  A wrong
sign, a wrong interface index or a closest centre taken over the wrong
interface breaks the exactness.

Density extension (Sec. 5.4, Neumann points off the primary set): the
weights are degree p-1 Lagrange weights in the grid coordinate along which
the stencil runs, so they reproduce every polynomial of degree <= p-1 in
that coordinate of the points they combine.

Adam (Kingma & Ba): the first bias-corrected step moves every parameter
with a nonzero gradient by lr against the gradient's sign."""
import numpy as np
import pytest

from oracle import geometry, kfbi
from oracle import learned as OL
from paper_2309_05965_amd import workloads as W
from tests.test_oracle_kfbi import _random_poly, data_for


def both_nonzero_pairs(pl):
    """Stencil pairs (P irregular, Q neighbour) with P and Q inside two
    different interfaces."""
    geo, prob, d = pl.geo, pl.prob, pl.d
    flat = geo["reg"].ravel()
    irr = geo["irr"]
    ind = geometry.unravel(irr, prob)
    n = 0
    for o in pl.A:
        qn = geometry.ravel([ind[x] + o[x] for x in range(d)], prob)
        rp, rq = flat[irr], flat[qn]
        n += int(np.sum((rp != rq) & (rp != 0) & (rq != 0)))
    return n


def blocks_in_other_interior(pl):
    """DOF interpolation-block nodes inside an interface other than the
    DOF's own."""
    geo, prob, d = pl.geo, pl.prob, pl.d
    flat = geo["reg"].ravel()
    k = geo["dofs"]["iface"]
    n = 0
    for blk in np.ndindex(*(pl.p + 1,) * d):
        q = geometry.ravel([geo["blocks"][:, a] + blk[a] for a in range(d)], prob)
        rq = flat[q]
        n += int(np.sum((rq != 0) & (rq != k)))
    return n


def patch(prob, seed):
    """Simple solve with a different random polynomial of degree p in every
    region; returns (max |v - u|, max |d_n v_in - exact|, max |d_n v_out -
    exact|, max |J - g2|, plan)."""
    rng = np.random.default_rng(seed)
    d = prob["dim"]
    p = 4 if prob["order"] == 4 else 2
    K = len(prob["ifaces"])
    sol = {s: W.polynomial(_random_poly(d, p, rng)) for s in range(K + 1)}
    pl = kfbi.Plan(prob)
    geo = pl.geo
    data = data_for(pl, prob, sol)
    surf = geo["surf"]
    psiS = W.exact_density(prob, sol, surf["pos"], surf["nrm"], surf["iface"])
    v, dn_in, dn_out, _ = pl.simple_solve(a=data["g1"], b=psiS, ftilde=data["ftilde"],
                                          fhat=data["fhat"], gB=data["gB"])
    ue = W.exact_solution(prob, sol, geo["reg"])
    X = tuple(geo["dofs"]["pos"][:, a] for a in range(d))
    n = geo["dofs"]["nrm"]
    kk = geo["dofs"]["iface"]
    gi = np.zeros(pl.Nb)
    for k in range(1, K + 1):
        g = sol[k](X)[1]
        gi = np.where(kk == k, sum(g[a] * n[:, a] for a in range(d)), gi)
    g0 = sol[0](X)[1]
    go = sum(g0[a] * n[:, a] for a in range(d))
    J = pl.flux(dn_in, dn_out)
    return (np.max(np.abs(v - ue)) / (1 + np.max(np.abs(ue))), np.max(np.abs(dn_in - gi)),
            np.max(np.abs(dn_out - go)), np.max(np.abs(J - pl.dof_values(data["g2"]))), pl)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("gap", [0.5, 2.0])
def test_two_circles_patch(order, gap):
    ev, ein, eout, eJ, pl = patch(W.two_circles(order, 64, gap), 3 + order)
    assert ev < 1e-12 and ein < 1e-11 and eout < 1e-11 and eJ < 1e-10
    if gap < 1.0:
        assert both_nonzero_pairs(pl) > 0
    if order == 4:
        assert blocks_in_other_interior(pl) > 0


@pytest.mark.parametrize("order", [2, 4])
def test_two_spheres_patch(order):
    ev, ein, eout, eJ, pl = patch(W.two_spheres(64, 0.5, order), 9 + order)
    assert both_nonzero_pairs(pl) > 0
    assert ev < 1e-12 and ein < 1e-10 and eout < 1e-10 and eJ < 1e-9


def test_torus_and_sphere_patch():
    """The torus + concentric sphere workload (gap 2h) at 64^3."""
    ev, ein, eout, eJ, pl = patch(W.config3(64)[0], 21)
    assert blocks_in_other_interior(pl) > 0
    assert ev < 1e-12 and ein < 1e-10 and eout < 1e-10 and eJ < 1e-8


def test_torus_and_sphere_unresolved_at_32():
    """At 32^3 the torus tube (radius 4h) admits no valid collocation
    stencil for some centres; the set-up reports it."""
    with pytest.raises(geometry.GeometryError) as e:
        kfbi.Plan(W.config3(32)[0])
    assert e.value.status == "unresolved"


def _extension_exactness(prob):
    geo = geometry.build(prob)
    s = geo["surf"]
    idx, w = geo["ext_idx"], geo["ext_w"]
    p, d, h = idx.shape[1], prob["dim"], geo["h"]
    dpos = geo["dofs"]["pos"]
    used = np.nonzero((idx[:, 0] >= 0) & ~s["prim"])[0]
    worst = 0.0
    for q in used.tolist():
        best = np.inf
        for a in range(d):
            xi = (dpos[idx[q], a] - s["pos"][q, a]) / h
            err = max(abs(float(np.sum(w[q] * xi ** m)) - (1.0 if m == 0 else 0.0)) for m in range(p))
            best = min(best, err)
        worst = max(worst, best)
    return used.size, worst, geo


@pytest.mark.parametrize("case", ["star512", "sphere64", "two_spheres64"])
def test_extension_reproduces_polynomials_in_its_coordinate(case):
    if case == "star512":
        prob = W.config2(512)[0]
    elif case == "sphere64":
        prob = W.problem(3, 4, 64, -1.0, 1.0, 1.0, 5.0, 0.5, [W.sphere3d(0.03, -0.02, 0.01, 0.52)])
    else:
        prob = W.two_spheres(64, 0.5)
    n, worst, geo = _extension_exactness(prob)
    assert n > 0
    assert worst < 1e-12
    # every combined point is primary and on the same interface
    s = geo["surf"]
    idx = geo["ext_idx"]
    used = (idx[:, 0] >= 0) & ~s["prim"]
    iface_dof = geo["dofs"]["iface"]
    assert np.all(iface_dof[idx[used]] == s["iface"][used][:, None])


def test_extension_error_falls_with_h():
    """A smooth density sampled at the primary points and extended agrees
    with its values at the extended points to O(h^p)-ish accuracy."""
    errs = []
    for N in (32, 128):
        prob = W.problem(3, 4, N, -1.0, 1.0, 1.0, 5.0, 0.5, [W.sphere3d(0.03, -0.02, 0.01, 0.52)])
        geo = geometry.build(prob)
        s = geo["surf"]
        idx, w = geo["ext_idx"], geo["ext_w"]
        used = (idx[:, 0] >= 0) & ~s["prim"]
        f = lambda X: np.sin(3 * X[:, 0] + 1) * np.cos(2 * X[:, 1]) * np.exp(X[:, 2] / 2)
        psi = f(geo["dofs"]["pos"])
        ext = (w * np.where(idx >= 0, psi[np.maximum(idx, 0)], 0.0)).sum(axis=1)
        errs.append(np.max(np.abs(ext[used] - f(s["pos"][used]))))
    assert errs[1] < errs[0] / 16


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-3, 3, 50)
    g[:3] = 0.0
    p1, m, v = OL.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 0.01)
    step = p1 - p
    big = np.abs(g) > 1e-4
    assert np.allclose(step[big], -0.01 * np.sign(g[big]), rtol=1e-4, atol=0)
    assert np.all(step[:3] == 0.0)
    # constant gradient: every step is lr against its sign (the bias
    # corrections cancel the moment decay exactly)
    pt, m, v = p.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        pn, m, v = OL.adam_step(pt, g, m, v, t, 0.01)
        assert np.allclose((pn - pt)[big], -0.01 * np.sign(g[big]), rtol=1e-4, atol=0)
        pt = pn
    # a gradient that flips sign: the second step's mean is (0.1 (-g) + 0.09 g) / 0.19
    pa, m, v = OL.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 0.01)
    pb, m, v = OL.adam_step(pa, -g, m, v, 2, 0.01)
    mhat = (-0.1 + 0.09) * g / 0.19
    vhat = (0.001 * 0.999 + 0.001) * g * g / (1 - 0.999 ** 2)
    assert np.allclose((pb - pa)[big], -0.01 * mhat[big] / (np.sqrt(vhat[big]) + 1e-8), rtol=1e-9)

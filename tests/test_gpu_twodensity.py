"""Parity of the HIP library's two-density interface BIE (eq. bie-ifp-1)
with the FP64 oracle, on an MI355X: geometry bitwise, the operator on
[phi; psi] and the right-hand side within 1e-11 relative, full solves
(GMRES to 1e-12) within 1e-10."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import twodensity as otd  # noqa: E402
from paper_2309_05965_amd import workloads as W  # noqa: E402

from test_gpu_parity import assert_same_geometry, dev, host, rel  # noqa: E402

ELL = [W.ellipse2d(0.05, -0.02, 0.6, 0.45, theta=0.3)]
CASES = {
    "ellipse_o4_64": lambda: (W.td_problem(2, 4, 64, -1.0, 1.0, 1.0, 4.0, 0.0, 2.5, ELL),
                              {0: W.f_sin_sin, 1: W.f_exp_cos}),
    "ellipse_o2_128": lambda: (W.td_problem(2, 2, 128, -1.0, 1.0, 2.0, 0.5, 1.5, 0.0, ELL),
                               {0: W.f_x2_my3, 1: W.f_cos2x_expy}),
    "circles_close_64": lambda: (W.td_problem(2, 4, 64, -1.0, 1.0, 1.0, 3.0, 0.0, 4.0,
                                              W.two_circles(4, 64, 0.5)["ifaces"]),
                                 {0: W.f_sin_sin, 1: W.f_exp_cos, 2: W.f_x2_my3}),
    "sphere_32": lambda: (W.td_problem(3, 4, 32, -1.0, 1.0, 1.0, 4.0, 0.0, 2.5,
                                       [W.sphere3d(0.03, -0.02, 0.01, 0.52)]), {0: W.f_exp3, 1: W.f_sin3}),
    "three_spheres_64": lambda: W.e7_heterogeneous(64),
}
SOLVE_CASES = ["ellipse_o4_64", "ellipse_o2_128", "circles_close_64", "sphere_32"]

_cache = {}


def case(name):
    if name not in _cache:
        prob, sol = CASES[name]()
        print("case", name, flush=True)
        sys.stdout.flush()
        from paper_2309_05965_amd import kfbi
        gp = kfbi.Plan(prob)
        op = otd.TwoDensityPlan(prob)
        _cache[name] = (prob, sol, gp, op)
    return _cache[name]


def oracle_data(op, prob, sol):
    s = op.geo["surf"]
    return W.make_td_data(prob, sol, s["pos"], s["nrm"], s["iface"], op.geo["st"]["pde_pts"],
                          op.geo["dofs"]["iface"])


@pytest.mark.parametrize("name", list(CASES))
def test_geometry_matches_exactly(name):
    prob, sol, gp, op = case(name)
    assert_same_geometry(gp, op.p1)
    assert gp.n_unknowns == 2 * op.Nb


@pytest.mark.parametrize("name", list(CASES))
def test_operator_and_rhs(name):
    from paper_2309_05965_amd import kfbi
    prob, sol, gp, op = case(name)
    x = np.random.default_rng(8).standard_normal(2 * op.Nb)
    ref = op.matvec(x)
    out1 = gp.matvec(dev(x))
    out2 = gp.matvec(dev(x))
    assert rel(host(out1), ref) < 1e-11
    assert torch.equal(out1, out2)
    b = gp.rhs(kfbi.device_td_data(gp, prob, sol))
    assert rel(host(b), op.rhs(oracle_data(op, prob, sol))) < 1e-11


@pytest.mark.parametrize("name", SOLVE_CASES)
def test_full_solve(name):
    from paper_2309_05965_amd import kfbi
    prob, sol, gp, op = case(name)
    ref = op.solve(oracle_data(op, prob, sol), tol=1e-12, maxit=300)
    x, u, info = gp.solve(kfbi.device_td_data(gp, prob, sol), tol=1e-12, max_iter=300)
    assert info["status"] == 0
    assert info["true_rel_res"] < 1e-11
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert rel(host(x), ref["x"]) < 1e-10
    assert rel(host(u), ref["u"].ravel()) < 1e-10


def test_given_start_and_limits():
    """A given start equal to the solution converges at once; max_iter = 1
    at tol 1e-14 reports NOT_CONVERGED; batches and multigrid are refused."""
    from paper_2309_05965_amd import kfbi
    prob, sol, gp, op = case("ellipse_o4_64")
    data = kfbi.device_td_data(gp, prob, sol)
    x, u, info = gp.solve(data, tol=1e-12, max_iter=300)
    x2, u2, info2 = gp.solve(data, tol=1e-10, max_iter=300, psi0=x)
    assert info2["iters"] <= 1 and info2["status"] == 0
    assert rel(host(u2), host(u)) < 1e-9
    _, _, info3 = gp.solve(data, tol=1e-14, max_iter=1, raise_on_fail=False)
    assert kfbi.STATUS[info3["status"]] == "NOT_CONVERGED"
    with pytest.raises(kfbi.KfbiError):
        gp.solve(data, tol=1e-10, solver="mg32")
    with pytest.raises(kfbi.KfbiError):
        kfbi.Batch([prob], workers=1)

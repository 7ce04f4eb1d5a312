"""Grid convergence of the GPU solution against the exact solution (runs on
an MI355X): the torus + concentric sphere workload (4th order, interfaces
2h apart, beta 1/100; the touching-interfaces example of Sec. 6 uses the
same scheme) at 64^3 and 128^3, and the 256^3 error reported."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2309_05965_amd import workloads as W  # noqa: E402


def max_error(N):
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config3(N)
    print("torus + sphere", N, flush=True)
    gp = kfbi.Plan(prob)
    from paper_2309_05965_amd import manufactured as M
    data = M.plan_data(gp, "torus3d")
    psi, u, info = gp.solve(data, tol=1e-11, max_iter=300)
    assert info["status"] == 0
    reg = gp.export("region").cpu().numpy().reshape((N + 1,) * 3)
    ue = W.exact_solution(prob, sol, reg).ravel()
    return float(np.max(np.abs(u.cpu().numpy() - ue))), info["iters"]


def test_torus_sphere_fourth_order():
    e64, it64 = max_error(64)
    e128, it128 = max_error(128)
    rate = math.log2(e64 / e128)
    print("max error 64^3 %.3e (%d iterations), 128^3 %.3e (%d), order %.2f" % (e64, it64, e128, it128, rate))
    assert rate > 3.5
    assert abs(it128 - it64) <= 6                    # iteration counts flat in N


def test_torus_sphere_256_error():
    e128, _ = max_error(128)
    e256, it = max_error(256)
    print("max error 256^3 %.3e (%d iterations), order 128 -> 256 %.2f" % (e256, it, math.log2(e128 / e256)))
    assert e256 < e128 / 8

"""Status reporting of the C ABI (runs on an MI355X): non-finite data,
GMRES running out of iterations, per-problem set-up statuses of the
512-star batch against the oracle's, and a solve that captures a graph
while another thread creates and destroys plans."""
import os
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2309_05965_amd import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config4_status.txt")


def test_nonfinite_data_is_reported():
    """A NaN in the jump data [u] at a primary surface point reaches the
    right-hand side; the solve returns KFBI_E_NONFINITE instead of a
    density."""
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config2(128)
    gp = kfbi.Plan(prob)
    data = kfbi.device_data(gp, prob, sol)
    # at a primary point: the jump [u] is read at primary points only
    i = int(gp.export("dof_surf")[gp.n_dof // 2].item())
    data["g1"][i] = float("nan")
    psi, u, info = gp.solve(data, tol=1e-10, max_iter=20, raise_on_fail=False)
    assert info["status"] == 5                      # KFBI_E_NONFINITE
    with pytest.raises(kfbi.KfbiError) as e:
        gp.solve(data, tol=1e-10, max_iter=20)
    assert e.value.name == "NONFINITE"
    # the plan is still usable with good data
    data = kfbi.device_data(gp, prob, sol)
    _, _, info = gp.solve(data, tol=1e-10)
    assert info["status"] == 0 and info["true_rel_res"] < 1e-10


def test_not_converged_is_reported():
    """max_iter = 1 at tol 1e-14: KFBI_E_NOT_CONVERGED with the one-step
    iterate and its true residual."""
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config1(64)
    gp = kfbi.Plan(prob)
    data = kfbi.device_data(gp, prob, sol)
    psi, u, info = gp.solve(data, tol=1e-14, max_iter=1, raise_on_fail=False)
    assert info["status"] == 4                      # KFBI_E_NOT_CONVERGED
    assert info["iters"] == 1
    assert 1e-14 < info["true_rel_res"] < 1.0
    assert torch.isfinite(psi).all() and torch.isfinite(u).all()
    with pytest.raises(kfbi.KfbiError) as e:
        gp.solve(data, tol=1e-14, max_iter=1)
    assert e.value.name == "NOT_CONVERGED"


def test_batch_setup_statuses_match_oracle():
    """Every problem of the seeded 512-star batch gets the set-up status the
    oracle gives it (tests/golden/config4_status.txt, written from the
    oracle alone)."""
    from paper_2309_05965_amd import kfbi
    want = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#"):
                continue
            i, N, st = line.split()
            want[int(i)] = (int(N), st)
    batch = W.config4_batch()
    assert len(want) == len(batch) == 512
    got = {}
    for i, (prob, _) in enumerate(batch):
        assert prob["N"] == want[i][0]
        try:
            p = kfbi.Plan(prob)
            p.close()
            got[i] = "ok"
        except kfbi.KfbiError as e:
            got[i] = e.name.lower()
    bad = [(i, got[i], want[i][1]) for i in range(512) if got[i] != want[i][1]]
    assert not bad, bad[:10]


def test_graph_capture_beside_plan_setup():
    """A plan whose repeated solves capture the exact-count iteration graph
    (14 iterations, no power of two) while a second thread creates, solves
    and destroys plans: every solve succeeds and the repeated density is
    bitwise the first one."""
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config2(512)
    gp = kfbi.Plan(prob)
    data = kfbi.device_data(gp, prob, sol)
    psi0, _, i0 = gp.solve(data, tol=1e-8)
    assert i0["status"] == 0 and i0["iters"] & (i0["iters"] - 1) != 0
    stop = threading.Event()
    errors = []

    def churn():
        try:
            torch.cuda.set_device(0)
            p2, _ = W.config2(128)
            while not stop.is_set():
                q = kfbi.Plan(p2)
                q.close()
        except Exception as e:                      # reported by the main thread
            errors.append(repr(e))

    t = threading.Thread(target=churn)
    t.start()
    try:
        outs = [gp.solve(data, tol=1e-8) for _ in range(6)]
    finally:
        stop.set()
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for psi, _, info in outs:
        assert info["status"] == 0 and info["iters"] == i0["iters"]
        assert torch.equal(psi, psi0)

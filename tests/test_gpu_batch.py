"""Batched solves of many problems of uneven grid sizes (runs on an MI355X):
device-generated manufactured data against the host generator, every
batched solution bitwise equal to the same problem solved alone, parity
with the oracle, and per-problem failure reporting."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import kfbi as okfbi  # noqa: E402
from paper_2309_05965_amd import workloads as W  # noqa: E402


def smooth_stars(n, seed=11):
    """Stars of the batch family with smaller mode amplitudes (a_k < 0.01),
    resolved on every grid of the batch."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = [64, 128, 256][i % 3]
        a = rng.uniform(0.0, 0.01, 7)
        ph = rng.uniform(0.0, 2 * np.pi, 7)
        A = [0.0] + list(a * np.cos(ph))
        B = [0.0] + list(-a * np.sin(ph))
        out.append(W.problem(2, 4, N, -1.0, 1.0, 10.0 ** rng.uniform(-2, 2), 1.0, 1.0,
                             [W.star2d(0.0, 0.0, 0.4, A, B)]))
    return out


def small_batch():
    out = smooth_stars(9)
    out.append(W.config3(64)[0])
    return out, ["star2d"] * 9 + ["torus3d"]


@pytest.mark.parametrize("which", ["star", "torus"])
def test_device_data_matches_host_generator(which):
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config2(128) if which == "star" else W.config3(64)
    gp = kfbi.Plan(prob)
    dev = kfbi.manufactured_data(gp, "star2d" if which == "star" else "torus3d")
    host = kfbi.device_data(gp, prob, sol)
    for k in ("g1", "g2", "ftilde", "fhat", "gB"):
        a, b = dev[k].cpu().numpy().ravel(), host[k].cpu().numpy().ravel()
        if k == "gB":
            n1 = prob["N"] + 1
            m = np.ones((n1,) * prob["dim"], bool)
            m[(slice(1, -1),) * prob["dim"]] = False
            a, b = a[m.ravel()], b[m.ravel()]
        assert np.max(np.abs(a - b)) <= 1e-13 * (1 + np.max(np.abs(b))), k


def test_batch_equals_single_solves_bitwise():
    from paper_2309_05965_amd import kfbi
    probs, kinds = small_batch()
    b = kfbi.Batch(probs, kinds, workers=3)
    u, info, secs = b.solve(tol=1e-8, keep_u=True)
    off = 0
    for p, k, inf in zip(probs, kinds, info):
        n = (p["N"] + 1) ** p["dim"]
        gp = kfbi.Plan(p)
        d = kfbi.manufactured_data(gp, k)
        d["ftilde"] = d["ftilde"]
        _, u1, i1 = gp.solve(d, tol=1e-8)
        assert inf["status"] == 0 and inf["iters"] == i1["iters"]
        assert torch.equal(u[off:off + n], u1)
        off += n
    assert off == b.total_nodes
    assert all(s > 0 for s in secs)


def test_batch_matches_oracle():
    from paper_2309_05965_amd import kfbi
    probs = [p for p in smooth_stars(6, seed=3) if p["N"] == 64][:2]
    sol = {0: W.f_x2_my3, 1: W.f_cos2x_expy}
    b = kfbi.Batch(probs, ["star2d"] * len(probs), workers=2)
    u, info, _ = b.solve(tol=1e-13, keep_u=True)
    off = 0
    for p in probs:
        op = okfbi.Plan(p)
        s = op.geo["surf"]
        d = W.make_data(p, sol, s["pos"], s["nrm"], s["iface"], op.geo["st"]["pde_pts"], op.geo["dofs"]["iface"])
        ref = op.solve(d, tol=1e-13)["u"].ravel()
        n = ref.size
        assert np.max(np.abs(u[off:off + n].cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
        off += n


def test_batch_reports_failures_per_problem():
    from paper_2309_05965_amd import kfbi
    good = W.config2(64)[0]
    bad = W.problem(2, 4, 16, -1.0, 1.0, 1.0, 1.0, 0.0, [W.star2d(0.0, 0.0, 0.5, None, [0, 0, 0, 0, 0, 0, 0.3, 0])])
    b = kfbi.Batch([good, bad, good], ["star2d"] * 3, workers=2)
    _, info, _ = b.solve(tol=1e-8, raise_on_fail=False)
    assert info[0]["status"] == 0 and info[2]["status"] == 0
    assert info[1]["status"] != 0

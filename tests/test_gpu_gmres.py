"""Device GMRES (Arnoldi step) against a plain host GMRES driven by the
same device matvec, on problems that take each Arnoldi path: one work
group with 1, 2, 4 or 8 unknowns per thread, and the many-work-group
chain (more than 4096 unknowns).  The matvec itself is pinned to the
oracle in test_gpu_parity; here the Krylov machinery is checked: the
solution of A psi = b, the iteration count, and run-to-run bitwise
reproducibility."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2309_05965_amd import workloads as W  # noqa: E402


def sphere(N):
    return (W.problem(3, 4, N, -1.0, 1.0, 1.0, 5.0, 0.5, [W.sphere3d(0.03, -0.02, 0.01, 0.52)]),
            {0: W.f_exp3, 1: W.f_sin3})


CASES = {
    "c2_512": lambda: W.config2(512),        # 1,038 unknowns: 5 per thread, 4 wavefronts
    "c1_1024": lambda: W.config1(1024),      # 1280 < n <= 2048: 2 per thread, 16 wavefronts
    "sphere_64": lambda: sphere(64),         # ~3.5e3: one work group, w in LDS
    "torus_64": lambda: W.config3(64),       # ~6.1e3: many work groups, few of them
    "sphere_128": lambda: sphere(128),       # ~1.4e4: many work groups
}


def host_gmres(matvec, b, tol, maxit):
    """Unrestarted GMRES from x0 = 0 with modified Gram-Schmidt and a dense
    least-squares solve per step (test reference)."""
    n = b.size
    beta = np.linalg.norm(b)
    V = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    V[0] = b / beta
    y = None
    for j in range(maxit):
        w = matvec(V[j])
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
        e = np.zeros(j + 2)
        e[0] = beta
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e, rcond=None)[0]
        if np.linalg.norm(H[:j + 2, :j + 1] @ y - e) <= tol * beta:
            return V[:j + 1].T @ y, j + 1
    return V[:maxit].T @ y, maxit


@pytest.mark.parametrize("name", list(CASES))
def test_device_gmres_matches_host_gmres(name):
    from paper_2309_05965_amd import kfbi
    prob, sol = CASES[name]()
    print("case", name, flush=True)
    gp = kfbi.Plan(prob)
    data = kfbi.device_data(gp, prob, sol)
    b = gp.rhs(data).cpu().numpy()

    def mv(x):
        return gp.matvec(torch.from_numpy(np.ascontiguousarray(x)).cuda()).cpu().numpy()

    tol = 1e-12
    psi_h, it_h = host_gmres(mv, b, tol, 200)
    psi, _, info = gp.solve(data, tol=tol, max_iter=200)
    psi2, _, _ = gp.solve(data, tol=tol, max_iter=200)
    p = psi.cpu().numpy()
    print("  n_dof", gp.n_dof, "iters device", info["iters"], "host", it_h, flush=True)
    assert info["status"] == 0
    assert abs(info["iters"] - it_h) <= 1
    assert np.max(np.abs(p - psi_h)) <= 1e-9 * np.max(np.abs(psi_h))
    assert info["true_rel_res"] < 1e-10
    assert torch.equal(psi, psi2)                 # bitwise reproducible


def test_solve_on_caller_stream():
    """A plan made on a caller's own stream solves on that stream (graph
    capture included, no private stream); the result equals the solve of a
    plan made on the default stream bit for bit."""
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config2(256)
    p0 = kfbi.Plan(prob)
    d0 = kfbi.device_data(p0, prob, sol)
    psi0, u0, i0 = p0.solve(d0, tol=1e-10)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p1 = kfbi.Plan(prob)
        psi1, u1, i1 = p1.solve(d0, tol=1e-10)
        psi2, u2, i2 = p1.solve(d0, tol=1e-10)
    s.synchronize()
    assert i1["status"] == 0 and i1["iters"] == i0["iters"] == i2["iters"]
    assert torch.equal(psi1, psi0) and torch.equal(u1, u0)
    assert torch.equal(psi2, psi0) and torch.equal(u2, u0)


def test_speculative_tail_short_first_batch():
    """On a plan solved before, the update, true residual and final solve go
    out behind the first GMRES batch, sized to the previous iteration count.
    When that batch is too short (a tighter tolerance than last time) the
    speculative work is redone after convergence: the result equals a fresh
    plan's bit for bit, and so does a repeat at the same tolerance."""
    from paper_2309_05965_amd import kfbi
    prob, sol = W.config2(128)
    ref = kfbi.Plan(prob)
    d = kfbi.device_data(ref, prob, sol)
    psi_r, u_r, i_r = ref.solve(d, tol=1e-12)
    gp = kfbi.Plan(prob)
    _, _, i_lo = gp.solve(d, tol=1e-6)
    _, _, _ = gp.solve(d, tol=1e-6)            # key reused from here on
    psi1, u1, i1 = gp.solve(d, tol=1e-12)      # first batch too short
    psi2, u2, i2 = gp.solve(d, tol=1e-12)      # first batch long enough
    assert i_lo["iters"] < i_r["iters"]
    assert i1["iters"] == i2["iters"] == i_r["iters"]
    assert i1["true_rel_res"] == i_r["true_rel_res"] and i2["true_rel_res"] == i_r["true_rel_res"]
    for p, u in ((psi1, u1), (psi2, u2)):
        assert torch.equal(p, psi_r) and torch.equal(u, u_r)

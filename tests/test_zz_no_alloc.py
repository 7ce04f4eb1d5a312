"""The allocation-free box solve (kfbi_box_solve_noalloc, static device
scratch) against the plan's box solve (kfbi_box_solve) on the same grids:
two calls in a row, the second on a smaller grid, in 2D and 3D, both
orders; sizes beyond the static maximum are rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2309_05965_amd import workloads as W  # noqa: E402


def plan_box_solve(dim, order, N, kappa, F):
    from paper_2309_05965_amd import kfbi
    if dim == 2:
        prob = W.problem(2, order, N, -1.0, 1.0, 1.0, 1.0, kappa, [W.ellipse2d(0.0, 0.0, 0.45, 0.45)])
    else:
        prob = W.problem(3, order, N, -1.0, 1.0, 1.0, 5.0, kappa, [W.sphere3d(0.03, -0.02, 0.01, 0.52)])
    gp = kfbi.Plan(prob)
    v = gp.box_solve(F)
    torch.cuda.synchronize()
    gp.close()
    return v


@pytest.mark.parametrize("dim,order,sizes,kappa", [(2, 4, (1024, 256), 1.0), (2, 2, (512, 64), 0.0),
                                                   (3, 4, (128, 32), 0.5), (3, 2, (64, 32), 0.0)])
def test_noalloc_box_solve_matches_plan_box_solve(dim, order, sizes, kappa):
    from paper_2309_05965_amd import kfbi
    for N in sizes:                                  # second call smaller: stale scratch must not leak in
        print("noalloc box solve dim %d order %d N %d" % (dim, order, N), flush=True)
        F = torch.from_numpy(np.random.default_rng(N + dim).standard_normal((N + 1) ** dim)).cuda()
        ref = plan_box_solve(dim, order, N, kappa, F)
        v = torch.full_like(F, float("nan"))        # every entry must be written
        kfbi.box_solve_noalloc(dim, order, N, -1.0, 1.0, kappa, F, v)
        torch.cuda.synchronize()
        assert torch.isfinite(v).all()
        d = (v - ref).abs().max().item() / ref.abs().max().item()
        assert d <= 1e-12, d
        vb = v.view((N + 1,) * dim)
        inner = torch.zeros_like(vb)
        sl = (slice(1, N),) * dim
        inner[sl] = vb[sl]
        assert torch.equal(vb, inner)                # zero box boundary


def test_noalloc_rejects_sizes_beyond_the_scratch():
    from paper_2309_05965_amd import kfbi
    F = torch.zeros(257 ** 3, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(F)
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.box_solve_noalloc(3, 4, 256, -1.0, 1.0, 0.0, F, v)
    assert e.value.name == "INVALID"
    with pytest.raises(kfbi.KfbiError):
        kfbi.box_solve_noalloc(2, 4, 2048, -1.0, 1.0, 0.0, F, v)

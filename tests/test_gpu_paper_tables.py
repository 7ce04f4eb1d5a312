"""The paper's examples on the GPU against its printed tables (Sec. 6),
at paper level: GMRES iteration counts within a few of the printed ones
and error maxima within the stated factors, on the grids where the
discretisation is resolved (the coarsest 3D grids of the product domain,
the torus and the three spheres, and the touching torus and ellipsoid up to
256^3, have local collocation systems with condition numbers of 1e5-1e7 and
need more iterations than printed; the full table with every grid is the
reproduction summary).  Readings where the paper is
silent: E2 circle radius 0.3826, E5 atom radius 0.5, E7 box and exact
solution (its errors are therefore not compared)."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2309_05965_amd import paper_tables as PT  # noqa: E402


@pytest.mark.parametrize("case,N,it_tol,err_fac", [("E1", 128, 2, 4.0), ("E1", 256, 2, 4.0), ("E1", 512, 2, 4.0),
                                                   ("E1", 1024, 2, 4.0), ("E2", 512, 2, 4.0), ("E2", 1024, 2, 4.0),
                                                   ("E3", 128, 2, 8.0), ("E3", 256, 2, 8.0), ("E4", 512, 1, None),
                                                   ("E6", 128, None, 4.0)])
def test_single_density_and_bvp_tables(case, N, it_tol, err_fac):
    """(E6, the touching torus and ellipsoid: errors only; its iteration
    counts are about twice the printed ones, see the module docstring.)"""
    r = PT.run_case(case, N)
    p = PT.PAPER[case][N]
    assert r["status"] == 0
    if it_tol is not None:
        assert abs(r["iters"] - p[1]) <= it_tol, (r["iters"], p)
    if err_fac is not None:
        printed = p[3] if case in ("E1", "E3", "E4") else (max(p[2], p[3]) if case == "E6" else p[2])
        assert printed / err_fac < r["in"][1] < printed * err_fac, (r["in"], p)


@pytest.mark.parametrize("ratio", [10.0, 100.0, 1e4])
def test_molecule_contrast_table(ratio):
    """E5 (Table 3d-ifp-ratio): the iteration count barely depends on the
    contrast and stays within 2 of the printed one at 128^3 and 256^3; at
    256^3 both error maxima are within a factor 2 of the printed ones."""
    for N in (128, 256):
        r = PT.run_case("E5", N, ratio)
        p = PT.PAPER["E5"][ratio][N]
        assert r["status"] == 0
        assert abs(r["iters"] - p[0]) <= 2, (N, r["iters"], p)
        if N == 256:
            assert p[2] / 2 < r["in"][1] < 2 * p[2] and p[4] / 2 < r["out"][1] < 2 * p[4], (r, p)


def test_heterogeneous_iterations_and_order():
    """E7 (Table 3d-ifp-heter): 20 iterations at 128^3 and 256^3 within 1,
    and the error falls at least 8-fold from 128^3 to 256^3 in both regions."""
    r1 = PT.run_case("E7", 128)
    r2 = PT.run_case("E7", 256)
    for r in (r1, r2):
        assert r["status"] == 0 and abs(r["iters"] - 20) <= 1, r
    assert r1["in"][1] / r2["in"][1] > 8.0 and r1["out"][1] / r2["out"][1] > 8.0, (r1, r2)

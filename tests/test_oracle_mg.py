"""Pins of the oracle's two-grid box solver and defect-correction loop
(Alg. 1 Step 3.3 with multigrid in place of the FFT): transfer operators
against their closed forms, the Jacobi weight against the Fourier symbol,
the V-cycle contraction, and the converged result against the exact DST
solve with the rigorous bound |v - A^-1 F|_2 <= |F - A v|_2 / |lambda_min|."""
import numpy as np
import pytest

from oracle import fd, mg


def test_prolongation_is_scaled_transpose_of_restriction():
    rng = np.random.default_rng(0)
    for d in (2, 3):
        nc = 4
        r = np.zeros((2 * nc + 1,) * d)
        r[(slice(1, -1),) * d] = rng.standard_normal((2 * nc - 1,) * d)
        e = np.zeros((nc + 1,) * d)
        e[(slice(1, -1),) * d] = rng.standard_normal((nc - 1,) * d)
        lhs = np.sum(mg.restrict(r) * e) * 2 ** d
        rhs = np.sum(r * mg.prolong(e))
        assert lhs == pytest.approx(rhs, rel=1e-13)


def test_transfer_operators_reproduce_linear_functions():
    """Full weighting and linear interpolation are exact on linear data."""
    for d in (2, 3):
        n = 8
        x = np.linspace(0.0, 1.0, n + 1)
        g = np.meshgrid(*([x] * d), indexing="ij")
        f = 1.0 + sum((a + 2) * g[a] for a in range(d))
        c = f[(slice(None, None, 2),) * d]
        assert np.allclose(mg.prolong(c), f, atol=1e-14)
        fr = mg.restrict(f)
        assert np.allclose(fr[(slice(1, -1),) * d], c[(slice(1, -1),) * d], atol=1e-14)


@pytest.mark.parametrize("d,order", [(2, 2), (2, 4), (3, 4)])
def test_jacobi_weight_equalises_the_high_frequency_range(d, order):
    A, _ = fd.stencils(d, order, 1.0 / 64, 1.0)
    w, lo, hi = mg.jacobi_weight(A, d)
    assert abs(1 - w * lo) == pytest.approx(abs(1 - w * hi), rel=1e-12)
    assert abs(1 - w * lo) < 0.6           # a real smoother
    if d == 2 and order == 2:
        # 5-point Laplacian: rho = (2 - cos t1 - cos t2) / 2 over the high
        # frequencies spans [1/2, 2] in the limit -> omega = 4/5
        assert w == pytest.approx(0.8, abs=2e-3)


@pytest.mark.parametrize("d,order,N", [(2, 4, 64), (3, 4, 16), (2, 2, 32)])
def test_vcycle_contracts(d, order, N):
    h = 2.0 / N
    hier = mg.Hierarchy(d, order, N, h, 1.0)
    rng = np.random.default_rng(1)
    e = np.zeros((N + 1,) * d)
    e[(slice(1, N),) * d] = rng.standard_normal((N - 1,) * d)
    A = hier.ops[0]
    rates = []
    for _ in range(6):
        r = -mg.apply_full(A, e)
        e_new = e + hier.vcycle(r)
        rates.append(np.linalg.norm(e_new) / np.linalg.norm(e))
        e = e_new
    # the two-grid cycle with exact coarse solve contracts the error by
    # 0.07 (fourth order) and 0.12 (second order) per cycle, independently
    # of h; a wrong transfer weight or coarse spacing loses most of that
    assert max(rates[2:]) < (0.1 if order == 4 else 0.15)


@pytest.mark.parametrize("d,order,N,inner", [(2, 4, 64, np.float64), (2, 4, 64, np.float32),
                                             (3, 4, 16, np.float32), (2, 2, 32, np.float32)])
def test_defect_correction_reaches_the_exact_solve(d, order, N, inner):
    h = 2.0 / N
    kappa = 1.0
    rng = np.random.default_rng(2)
    F = rng.standard_normal((N - 1,) * d)
    v, its, hist = mg.solve(F, d, order, N, h, kappa, eps=1e-12, inner=inner, cycles=2)
    assert hist[-1] <= 1e-12
    exact = fd.dst_solve(F, d, order, N, h, kappa)
    lam_min = np.min(np.abs(fd.eigenvalues(d, order, N, h, kappa)))
    bound = hist[-1] * np.linalg.norm(F) / lam_min
    assert np.linalg.norm(v - exact) <= 1.01 * bound + 1e-14 * np.linalg.norm(exact)
    # FP32 V-cycles inside FP64 defect correction still reach FP64 accuracy,
    # at a contraction per outer step limited by the FP32 rounding
    assert its <= (12 if inner == np.float64 else 20)

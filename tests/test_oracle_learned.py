"""Pins of the learned-warm-start oracle: sample geometry against the level
set and closed-form curvatures, the spherical-harmonic basis against
quadrature orthonormality and its closed low-degree forms, exact
band-limited transfers, bf16 rounding, and the MLP gradient against finite
differences."""
import math

import numpy as np
import pytest

from oracle import learned as L
from oracle import levelset
from paper_2309_05965_amd import workloads as W


def test_fibonacci_lattice_is_on_the_sphere_and_balanced():
    S = W.fibonacci_sphere(1024)
    assert np.allclose(np.linalg.norm(S, axis=1), 1.0, atol=1e-14)
    assert np.abs(S.mean(axis=0)).max() < 2e-3


def test_samples_normals_on_the_ellipsoid():
    prob, geom, jumps = W.config5(7, N=64)
    S = W.fibonacci_sphere(256)
    X = L.sample_points(geom, S)
    iface = prob["ifaces"][0]
    H = levelset.H(iface, tuple(X[:, a] for a in range(3)))
    assert np.max(np.abs(H)) < 1e-13
    n, _ = L.normals_and_curvature(geom, X)
    n_ref = np.stack(levelset.normal(iface, tuple(X[:, a] for a in range(3))), axis=1)
    assert np.max(np.abs(n - n_ref)) < 1e-12


def test_mean_curvature_closed_forms():
    r = 0.45
    geom = (np.zeros(3), np.array([r, r, r]), np.eye(3))
    S = W.fibonacci_sphere(64)
    _, k = L.normals_and_curvature(geom, L.sample_points(geom, S))
    assert np.allclose(k, 1.0 / r, rtol=1e-13)
    a, b, c = 0.6, 0.4, 0.3
    geom = (np.zeros(3), np.array([a, b, c]), np.eye(3))
    _, k = L.normals_and_curvature(geom, np.array([[a, 0.0, 0.0]]))
    assert k[0] == pytest.approx(0.5 * (a / b ** 2 + a / c ** 2), rel=1e-13)


def test_real_sh_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(24)
    nphi = 48
    ph = 2 * np.pi * np.arange(nphi) / nphi
    ct, P = np.meshgrid(xg, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(P), st * np.sin(P), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = L.real_sh(dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-12


def test_real_sh_low_degree_closed_forms():
    d = np.random.default_rng(0).standard_normal((20, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = L.real_sh(d, 2)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 0], 0.5 / math.sqrt(math.pi))
    assert np.allclose(Y[:, 1], c1 * d[:, 1])        # l=1, m=-1: y
    assert np.allclose(Y[:, 2], c1 * d[:, 2])        # l=1, m=0: z
    assert np.allclose(Y[:, 3], c1 * d[:, 0])        # l=1, m=1: x
    c2 = 0.5 * math.sqrt(15 / math.pi)
    assert np.allclose(Y[:, 4], c2 * d[:, 0] * d[:, 1])   # l=2, m=-2: xy


def test_transfers_are_exact_for_band_limited_densities():
    prob, geom, _ = W.config5(3, N=64)
    S = W.fibonacci_sphere()
    rng = np.random.default_rng(1)
    coef = rng.standard_normal(81)
    dof_dirs = rng.standard_normal((500, 3))
    dof_dirs /= np.linalg.norm(dof_dirs, axis=1, keepdims=True)
    dof_pos = L.sample_points(geom, dof_dirs)
    psi_s = L.real_sh(S) @ coef
    psi_d = L.real_sh(dof_dirs) @ coef
    assert np.allclose(L.transfer_to_dofs(geom, S, psi_s, dof_pos), psi_d, atol=1e-10)
    assert np.allclose(L.sample_density(geom, S, dof_pos, psi_d), psi_s, atol=1e-10)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.0e-3])
    r = L.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0                   # tie to even
    assert r[2] == 1.0 + 2 ** -6                        # tie to even upward
    assert r[3] == 1.0 + 2 ** -7 and r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    sizes = [7, 5, 6, 3]
    Ws = [rng.standard_normal((sizes[i], sizes[i + 1])) * 0.5 for i in range(3)]
    bs = [rng.standard_normal(sizes[i + 1]) * 0.1 for i in range(3)]
    X = rng.standard_normal((4, 7))
    Y = rng.standard_normal((4, 3))
    loss, gW, gb = L.mlp_loss_grad(Ws, bs, X, Y, emulate=False)
    eps = 1e-6
    for l in range(3):
        for (i, j) in [(0, 0), (1, 2), (sizes[l] - 1, sizes[l + 1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += eps
            Wm[l][i, j] -= eps
            fd = (L.mlp_loss_grad(Wp, bs, X, Y, False)[0] - L.mlp_loss_grad(Wm, bs, X, Y, False)[0]) / (2 * eps)
            assert gW[l][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][0] += eps
        bm[l][0] -= eps
        fd = (L.mlp_loss_grad(Ws, bp, X, Y, False)[0] - L.mlp_loss_grad(Ws, bm, X, Y, False)[0]) / (2 * eps)
        assert gb[l][0] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_linear_head_gradient_matches_finite_differences():
    """The linear-head loss's gradient (exact arithmetic) against central
    differences, and the head's linearity in the coefficients."""
    rng = np.random.default_rng(3)
    widths = (5, 7, 12)                 # 12 outputs = 3 basis vectors of 4
    Ws = [rng.standard_normal((a, b)) * 0.5 for a, b in zip(widths[:-1], widths[1:])]
    bs = [rng.standard_normal(b) * 0.1 for b in widths[1:]]
    X = rng.standard_normal((4, 5))
    C = rng.standard_normal((4, 3))
    Yt = rng.standard_normal((4, 4))
    loss, gW, gb = L.mlp_lin_loss_grad(Ws, bs, X, C, Yt, emulate=False)
    eps = 1e-6
    for l in range(2):
        for (i, j) in ((0, 0), (2, 3), (4, 6) if l == 0 else (6, 11)):
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += eps
            Wm[l][i, j] -= eps
            fd = (L.mlp_lin_loss_grad(Wp, bs, X, C, Yt, emulate=False)[0]
                  - L.mlp_lin_loss_grad(Wm, bs, X, C, Yt, emulate=False)[0]) / (2 * eps)
            assert abs(fd - gW[l][i, j]) <= 1e-6 * (1 + abs(fd))
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][1] += eps
        bm[l][1] -= eps
        fd = (L.mlp_lin_loss_grad(Ws, bp, X, C, Yt, emulate=False)[0]
              - L.mlp_lin_loss_grad(Ws, bm, X, C, Yt, emulate=False)[0]) / (2 * eps)
        assert abs(fd - gb[l][1]) <= 1e-6 * (1 + abs(fd))
    z = rng.standard_normal((4, 12))
    assert np.allclose(L.lin_head(z, 2.5 * C, 3), 2.5 * L.lin_head(z, C, 3), rtol=1e-14)
    assert np.allclose(L.lin_head(z, C, 3)[1], z[1].reshape(3, 4).T @ C[1], rtol=1e-14)


def test_sh_coefficients_recover_band_limited_density():
    """Coefficients of a degree-<= 8 expansion are recovered exactly from its
    values at scattered points of the ellipsoid."""
    rng = np.random.default_rng(4)
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    geom = (np.array([0.01, -0.02, 0.0]), np.array([0.4, 0.55, 0.35]), Q * np.sign(np.diag(R))[None, :])
    S = rng.standard_normal((600, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    X = L.sample_points(geom, S)
    coef = rng.standard_normal(81)
    vals = L.sh_values(geom, X, coef)
    assert np.allclose(L.sh_coefficients(geom, X, vals), coef, atol=1e-10)


def test_mode_rows_give_the_jump_on_the_ellipsoid():
    """cos(k_m . x) at x = Q diag(a) s equals cos(kappa_m . s) with kappa_m
    the per-mode network's wave-vector input diag(a) Q^T k_m; mode_major
    is the (mode, coefficient) permutation of the packed jumps."""
    rng = np.random.default_rng(6)
    Q, Rr = np.linalg.qr(rng.standard_normal((3, 3)))
    geom = (np.zeros(3), np.array([0.35, 0.62, 0.48]), Q * np.sign(np.diag(Rr))[None, :])
    S = rng.standard_normal((50, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    X = L.sample_points(geom, S)
    rows = L.mode_rows(geom)
    kv = W.fourier_wavevectors()
    for m in range(8):
        assert np.allclose(np.cos(X @ kv[m]), np.cos(S @ rows[m, 3:6]), atol=1e-13)
        assert np.allclose(rows[m, :3], (geom[1] - 0.5) / 0.2) and np.allclose(rows[m, 6:], geom[2].ravel())
    j = np.arange(32.0)
    mm = L.mode_major(j)
    for m in range(8):
        for t in range(4):
            assert mm[4 * m + t] == j[8 * t + m]


def test_linear_head_rows_gradient_matches_finite_differences():
    """R = 2 rows per example: the loss's gradient against central
    differences, and the head of an example equal to the head applied to
    its two rows' outputs written side by side."""
    rng = np.random.default_rng(7)
    widths = (4, 6, 6)                  # 2 rows x 6 outputs = 3 basis vectors of 4
    Ws = [rng.standard_normal((a, b)) * 0.5 for a, b in zip(widths[:-1], widths[1:])]
    bs = [rng.standard_normal(b) * 0.1 for b in widths[1:]]
    X = rng.standard_normal((6, 4))     # 3 examples of 2 rows
    C = rng.standard_normal((3, 3))
    Yt = rng.standard_normal((3, 4))
    loss, gW, _ = L.mlp_lin_loss_grad(Ws, bs, X, C, Yt, emulate=False, R=2)
    eps = 1e-6
    for l, (i, j) in ((0, (1, 2)), (1, (5, 4)), (1, (0, 0))):
        Wp = [w.copy() for w in Ws]
        Wm = [w.copy() for w in Ws]
        Wp[l][i, j] += eps
        Wm[l][i, j] -= eps
        fd = (L.mlp_lin_loss_grad(Wp, bs, X, C, Yt, emulate=False, R=2)[0]
              - L.mlp_lin_loss_grad(Wm, bs, X, C, Yt, emulate=False, R=2)[0]) / (2 * eps)
        assert abs(fd - gW[l][i, j]) <= 1e-6 * (1 + abs(fd))
    out = L.mlp_forward(Ws, bs, X, emulate=False)[0][-1]
    b = 1
    z = np.concatenate([out[2 * b], out[2 * b + 1]])
    y = sum(C[b, jj] * z[4 * jj:4 * jj + 4] for jj in range(3))
    d = y - Yt[b]
    assert loss > np.sum(d * d) / Yt.size - 1e-15

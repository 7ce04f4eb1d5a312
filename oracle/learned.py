"""Learned warm start for GMRES (oracle side): interface-sample features,
the spherical-harmonic transfer between samples and DOFs, and the MLP with
its mean-squared-error gradient.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The KFBI solve starts GMRES from an initial density (Alg. 1 Step 2); the
zero start is the default.  The learned start predicts the density from the
interface and jump data:
  samples   s_i, i < 1024, a Fibonacci lattice on the unit sphere, mapped to
            the ellipsoid x_i = c + Q diag(a) s_i;
  features  per sample: position (3), outward unit normal (3), mean
            curvature (1), g1(x_i), g2(x_i): 9 values, flattened in sample
            order to one 9216-vector;
  network   MLP 9216 -> 256 -> 256 -> 256 -> 1024, ReLU on the hidden
            layers, bf16 operands with wider accumulation; output = the
            density at the samples divided by a fixed output scale;
  transfer  least-squares fit of real spherical harmonics of degree <= 8 in
            the body-frame direction diag(1/a) Q^T (x - c) / | . | (81
            functions) to the sample values, evaluated at the DOFs;
  targets   the solved density psi* at the DOFs, fitted the same way and
            evaluated at the samples.
Linear-head form (the density is linear in the 32 jump coefficients when
the source and box data vanish): the network maps the geometry to 32 basis
densities, each as its 81 SH coefficients; lin_head contracts them with the
jump coefficients, and the targets are the SH coefficients of psi*.
"""
import numpy as np
import scipy.special

LMAX = 8


def sample_points(geom, S):
    c, a, Q = geom
    return np.asarray(c)[None, :] + (np.asarray(S) * np.asarray(a)[None, :]) @ np.asarray(Q).T


def body_coords(geom, X):
    c, a, Q = geom
    return (np.asarray(X) - np.asarray(c)[None, :]) @ np.asarray(Q)


def normals_and_curvature(geom, X):
    """Outward unit normal and mean curvature (average of the principal
    curvatures, 1/r on a sphere) of H = sum (X_j / a_j)^2 - 1 at X."""
    c, a, Q = geom
    a = np.asarray(a)
    Xb = body_coords(geom, X)
    g = 2.0 * Xb / a ** 2                     # body-frame gradient
    hess = 2.0 / a ** 2                        # diagonal of the Hessian
    ng = np.linalg.norm(g, axis=1)
    n = (g @ np.asarray(Q).T) / ng[:, None]
    kappa = (ng ** 2 * hess.sum() - (g * g * hess[None, :]).sum(axis=1)) / (2.0 * ng ** 3)
    return n, kappa


def features(geom, jumps_fn, S):
    """(n, 9) features at the samples; jumps_fn(X) -> (g1, g2)."""
    X = sample_points(geom, S)
    n, kappa = normals_and_curvature(geom, X)
    g1, g2 = jumps_fn(X)
    return np.concatenate([X, n, kappa[:, None], np.asarray(g1)[:, None], np.asarray(g2)[:, None]], axis=1)


def real_sh(dirs, lmax=LMAX):
    """Real orthonormal spherical harmonics at unit directions (n, 3), index
    l^2 + l + m: m > 0 -> sqrt2 (-1)^m Re Y_l^m, m < 0 -> sqrt2 (-1)^m Im
    Y_l^|m|, m = 0 -> Y_l^0 (scipy's complex Y_l^m with the Condon-Shortley
    phase, so these carry none)."""
    d = np.asarray(dirs, dtype=np.float64)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    out = np.zeros((d.shape[0], (lmax + 1) ** 2))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                v = np.sqrt(2.0) * (-1) ** m * Y.real
            elif m < 0:
                v = np.sqrt(2.0) * (-1) ** m * Y.imag
            else:
                v = Y.real
            out[:, l * l + l + m] = v
    return out


def sh_fit(dirs, values, lmax=LMAX):
    """Least-squares coefficients of real SH of degree <= lmax."""
    Y = real_sh(dirs, lmax)
    coef, *_ = np.linalg.lstsq(Y, np.asarray(values, dtype=np.float64), rcond=None)
    return coef


def transfer_to_dofs(geom, S, psi_s, dof_pos, lmax=LMAX):
    """Density at the DOFs from its values at the samples."""
    coef = sh_fit(S, psi_s, lmax)
    return real_sh(body_coords(geom, dof_pos) / np.asarray(geom[1])[None, :], lmax) @ coef


def sample_density(geom, S, dof_pos, psi_dof, lmax=LMAX):
    """Density at the samples from its values at the DOFs."""
    coef = sh_fit(body_coords(geom, dof_pos) / np.asarray(geom[1])[None, :], psi_dof, lmax)
    return real_sh(S, lmax) @ coef


# ---------------------------------------------------------------- MLP
def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(Ws, bs, X, emulate=True):
    """Activations [a_0 = X, a_1, ..., a_L] and pre-activations z_l; hidden
    layers ReLU, last layer linear.  With emulate, the GEMM operands (inputs,
    weights, hidden activations) are rounded to bf16 as on the GPU."""
    r = bf16 if emulate else (lambda t: np.asarray(t, dtype=np.float64))
    a = [np.asarray(X, dtype=np.float64)]
    zs = []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = r(a[-1]) @ r(W) + np.asarray(b, dtype=np.float64)[None, :]
        zs.append(z)
        a.append(np.maximum(z, 0.0) if l < len(Ws) - 1 else z)
    return a, zs


def mlp_loss_grad(Ws, bs, X, Yt, emulate=True):
    """L = mean (out - Yt)^2 over all entries, and (dL/dW_l, dL/db_l).
    With emulate the backward GEMM operands (activations, weights and the
    back-propagated gradients) are rounded to bf16 like the GPU's."""
    a, zs = mlp_forward(Ws, bs, X, emulate)
    out = a[-1]
    n = out.size
    diff = out - np.asarray(Yt, dtype=np.float64)
    loss = float(np.sum(diff * diff) / n)
    gW, gb = mlp_backward(Ws, a, zs, 2.0 * diff / n, emulate)
    return loss, gW, gb


def lin_head(z, C, nb):
    """Linear head: the network's output row z (nb blocks of K) holds nb
    basis vectors; y[k] = sum_j C[j] z[j K + k]."""
    z = np.asarray(z, dtype=np.float64)
    B, W = z.shape
    K = W // nb
    return np.einsum("bj,bjk->bk", np.asarray(C, dtype=np.float64), z.reshape(B, nb, K))


def mlp_lin_loss_grad(Ws, bs, X, C, Yt, emulate=True, R=1):
    """L = mean (lin_head(MLP(X), C) - Yt)^2 and (dL/dW_l, dL/db_l): X holds
    B examples of R rows, the output of an example is its R rows read as
    one row; the head is applied in full precision; its gradient with
    respect to the network's output is dz[j K + k] = C[j] dy[k]."""
    a, zs = mlp_forward(Ws, bs, X, emulate)
    C = np.asarray(C, dtype=np.float64)
    nb = C.shape[1]
    B = C.shape[0]
    y = lin_head(a[-1].reshape(B, -1), C, nb)
    n = y.size
    diff = y - np.asarray(Yt, dtype=np.float64)
    loss = float(np.sum(diff * diff) / n)
    dy = 2.0 * diff / n
    dz = (C[:, :, None] * dy[:, None, :]).reshape(a[-1].shape)
    gW, gb = mlp_backward(Ws, a, zs, dz, emulate)
    return loss, gW, gb


def mode_rows(geom):
    """Network input of the per-mode linear-head network (15 per row, 8 rows):
    (a - 0.5) / 0.2, the mode's scaled body-frame wave vector diag(a) Q^T k_m
    (k_m = (pi/2)(m & 1, (m >> 1) & 1, (m >> 2) & 1)), and Q row-major."""
    c, a, Q = geom
    a = np.asarray(a, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    rows = []
    for m in range(8):
        k = (np.pi / 2) * np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1], dtype=np.float64)
        rows.append(np.concatenate([(a - 0.5) / 0.2, a * (Q.T @ k), Q.ravel()]))
    return np.array(rows)


def mode_major(jumps32):
    """Packed jump coefficients (a_1[8], a_2[8], b_1[8], b_2[8]) reordered to
    (m, t) = (mode, a_1 a_2 b_1 b_2), the order of the per-mode network's
    basis vectors."""
    j = np.asarray(jumps32).reshape(4, 8)
    return j.T.reshape(-1)


def mlp_backward(Ws, a, zs, dz, emulate=True):
    """Gradients (dL/dW_l, dL/db_l) from the gradient dz of the loss with
    respect to the last layer's output, through the ReLU layers."""
    r = bf16 if emulate else (lambda t: np.asarray(t, dtype=np.float64))
    gW = [None] * len(Ws)
    gb = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        gW[l] = r(a[l]).T @ r(dz)
        gb[l] = dz.sum(axis=0)
        if l > 0:
            da = r(dz) @ r(Ws[l]).T
            dz = da * (zs[l - 1] > 0.0)
    return gW, gb


def sh_coefficients(geom, dof_pos, psi_dof, lmax=LMAX):
    """Least-squares coefficients of the density in the real SH of degree
    <= lmax of the body-frame direction of the DOFs."""
    return sh_fit(body_coords(geom, dof_pos) / np.asarray(geom[1])[None, :], psi_dof, lmax)


def sh_values(geom, dof_pos, coef, lmax=LMAX):
    """The SH expansion with coefficients coef at the DOFs."""
    return real_sh(body_coords(geom, dof_pos) / np.asarray(geom[1])[None, :], lmax) @ np.asarray(coef)


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) on float64 copies:
    m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
    mhat = m / (1 - b1^t), vhat = v / (1 - b2^t),
    theta <- theta - lr mhat / (sqrt(vhat) + eps); t counts from 1.
    Returns (params, m, v)."""
    g = np.asarray(grads, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v

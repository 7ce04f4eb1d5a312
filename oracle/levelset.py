"""Level-set functions of the interfaces (paper Sec. 5.1: Gamma = {H = 0},
H < 0 inside, outward normal n = grad H / |grad H|).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Every family is written with +, -, *, / and sqrt only, in a fixed
left-to-right order, so that the sign of H at a node and every bisection
decision is an IEEE-exact function of the inputs.  The polar star
r(theta) = c0 + sum_k (A_k cos k theta + B_k sin k theta) therefore obtains
cos k theta and sin k theta from powers of the unit vector (dx + i dy)/rho
(de Moivre) instead of atan2/sin; a pin in tests checks that this equals the
trigonometric definition.

Parameter vectors (shared interface with the HIP library, documented in the
design notes):
  ellipse2d   [cx, cy, c, s, a, b]          X = c dx + s dy, Y = c dy - s dx,
                                            H = (X/a)^2 + (Y/b)^2 - 1
  star2d      [cx, cy, c0, A1..A8, B1..B8]  H = rho - r(theta)  (H(centre) = -c0)
  sphere3d    [cx, cy, cz, r]               H = |d|^2 - r^2
  ellipsoid3d [cx, cy, cz, a0, a1, a2, R00..R22]  X = R^T d (R row-major),
                                            H = sum (X_j/a_j)^2 - 1
  torus3d     [cx, cy, cz, R, r]            H = (sqrt(dx^2+dy^2) - R)^2 + dz^2 - r^2
  product3d   [cx, cy, cz, s]               X = s dx, Y = s dy, Z = s dz,
                                            H = (1+X^2)(1+Y^2)(1+Z^2) + 8XYZ + X^2 + Y^2 + Z^2 - 3
              (with s = 2 the domain of the paper's 3D modified-Helmholtz Dirichlet
              example, Sec. 6.2.2: (1+4x^2)(1+4y^2)(1+4z^2) + 64xyz + 4x^2+4y^2+4z^2 < 3)
  molecule3d  [c, r, m, x1, y1, z1, ..., xm, ym, zm] (m <= 8 atoms)
                                            H = c - sum_k E(-|x - x_k|^2 / r^2)
              (the molecular surface of Sec. 6.2.3 with c = 0.6), where E is
              the exponential evaluated with +, -, *, / only: E(t) =
              P(t / 1024)^1024 with P the degree-12 Taylor polynomial of exp
              in Horner form and ten squarings (relative error about 1e-13 for
              -40 <= t <= 0, far below any grid spacing's effect)
  grid        [q, lo, hi, N] and the samples S (shape (N+1,)*d, x fastest) of
              H at the nodes of the computational grid (the level set known
              only at Cartesian nodes, Sec. 7): H is the tensor-product
              Lagrange interpolant of degree q (3 or 5) on the (q+1)^d nodes
              around the point's cell (base floor(t) - (q-1)/2 clamped to
              [0, N-q] per axis, t = (x - lo)/h snapped to the nearest
              integer within 1e-9, so that along a grid line it is the 1D
              interpolant of that line and at a node it is the sample), its
              gradient the gradient of the same polynomial
"""
import numpy as np

KINDS = ("ellipse2d", "star2d", "sphere3d", "ellipsoid3d", "torus3d", "product3d", "molecule3d", "grid")
DIM_OF = {"ellipse2d": 2, "star2d": 2, "sphere3d": 3, "ellipsoid3d": 3, "torus3d": 3, "product3d": 3,
          "molecule3d": 3}
NMODES = 8


def _ellipse(p, X, grad):
    x, y = X
    cx, cy, c, s, a, b = p[:6]
    dx = x - cx
    dy = y - cy
    XX = c * dx + s * dy
    YY = c * dy - s * dx
    Xa = XX / a
    Yb = YY / b
    H = Xa * Xa + Yb * Yb - 1.0
    if not grad:
        return H
    GX = 2.0 * Xa / a
    GY = 2.0 * Yb / b
    return (GX * c - GY * s, GX * s + GY * c)


def _star(p, X, grad):
    x, y = X
    cx, cy, c0 = p[0], p[1], p[2]
    A = p[3:3 + NMODES]
    B = p[3 + NMODES:3 + 2 * NMODES]
    dx = x - cx
    dy = y - cy
    rho = np.sqrt(dx * dx + dy * dy)
    zero = rho == 0.0
    safe = np.where(zero, 1.0, rho)
    ux = dx / safe
    uy = dy / safe
    cr = np.ones_like(ux)
    ci = np.zeros_like(ux)
    r = np.zeros_like(ux) + c0
    rp = np.zeros_like(ux)
    for k in range(1, NMODES + 1):
        cr, ci = cr * ux - ci * uy, cr * uy + ci * ux
        r = r + (A[k - 1] * cr + B[k - 1] * ci)
        rp = rp + float(k) * (B[k - 1] * cr - A[k - 1] * ci)
    if not grad:
        return np.where(zero, -c0, rho - r)
    return (ux + rp * uy / safe, uy - rp * ux / safe)


def _sphere(p, X, grad):
    x, y, z = X
    d0 = x - p[0]
    d1 = y - p[1]
    d2 = z - p[2]
    if not grad:
        return d0 * d0 + d1 * d1 + d2 * d2 - p[3] * p[3]
    return (2.0 * d0, 2.0 * d1, 2.0 * d2)


def _ellipsoid(p, X, grad):
    x, y, z = X
    d = (x - p[0], y - p[1], z - p[2])
    ax = p[3:6]
    R = p[6:15]
    Xa = []
    for j in range(3):
        Xj = R[0 * 3 + j] * d[0] + R[1 * 3 + j] * d[1] + R[2 * 3 + j] * d[2]
        Xa.append(Xj / ax[j])
    if not grad:
        return Xa[0] * Xa[0] + Xa[1] * Xa[1] + Xa[2] * Xa[2] - 1.0
    G = [2.0 * Xa[j] / ax[j] for j in range(3)]
    return tuple(R[i * 3 + 0] * G[0] + R[i * 3 + 1] * G[1] + R[i * 3 + 2] * G[2]
                 for i in range(3))


def _torus(p, X, grad):
    x, y, z = X
    d0 = x - p[0]
    d1 = y - p[1]
    d2 = z - p[2]
    RR, rr = p[3], p[4]
    rho = np.sqrt(d0 * d0 + d1 * d1)
    q = rho - RR
    if not grad:
        return q * q + d2 * d2 - rr * rr
    safe = np.where(rho == 0.0, 1.0, rho)
    return (2.0 * q * d0 / safe, 2.0 * q * d1 / safe, 2.0 * d2)


def _product(p, X, grad):
    x, y, z = X
    sc = p[3]
    X0 = sc * (x - p[0])
    Y0 = sc * (y - p[1])
    Z0 = sc * (z - p[2])
    x2 = X0 * X0
    y2 = Y0 * Y0
    z2 = Z0 * Z0
    if not grad:
        return (1.0 + x2) * (1.0 + y2) * (1.0 + z2) + 8.0 * X0 * Y0 * Z0 + x2 + y2 + z2 - 3.0
    gx = 2.0 * X0 * (1.0 + y2) * (1.0 + z2) + 8.0 * Y0 * Z0 + 2.0 * X0
    gy = 2.0 * Y0 * (1.0 + x2) * (1.0 + z2) + 8.0 * X0 * Z0 + 2.0 * Y0
    gz = 2.0 * Z0 * (1.0 + x2) * (1.0 + y2) + 8.0 * X0 * Y0 + 2.0 * Z0
    return (sc * gx, sc * gy, sc * gz)


def exp_arith(t):
    """exp(t) for t <= 0 with +, -, *, / only: the degree-12 Taylor
    polynomial of exp at t / 1024 (Horner), squared ten times."""
    y = t / 1024.0
    s = 1.0 + 0.0 * y
    for k in range(12, 0, -1):
        s = 1.0 + y * s / float(k)
    for _ in range(10):
        s = s * s
    return s


def _molecule(p, X, grad):
    x, y, z = X
    c, r, m = p[0], p[1], int(p[2])
    rr = r * r
    H = c + 0.0 * x
    G = [0.0 * x, 0.0 * x, 0.0 * x]
    for k in range(m):
        d0 = x - p[3 + 3 * k]
        d1 = y - p[4 + 3 * k]
        d2 = z - p[5 + 3 * k]
        e = exp_arith(-(d0 * d0 + d1 * d1 + d2 * d2) / rr)
        H = H - e
        G[0] = G[0] + 2.0 * e * d0 / rr
        G[1] = G[1] + 2.0 * e * d1 / rr
        G[2] = G[2] + 2.0 * e * d2 / rr
    return tuple(G) if grad else H


_FUN = {"ellipse2d": _ellipse, "star2d": _star, "sphere3d": _sphere,
        "ellipsoid3d": _ellipsoid, "torus3d": _torus, "product3d": _product, "molecule3d": _molecule}


def _axis_weights(x, lo, h, N, q):
    """Stencil base, Lagrange weights and their derivatives (in t) of one
    axis for the sampled level set."""
    t = (np.asarray(x, dtype=np.float64) - lo) / h
    r = np.floor(t + 0.5)
    t = np.where(np.abs(t - r) < 1e-9, r, t)
    base = np.clip(np.floor(t).astype(np.int64) - (q - 1) // 2, 0, N - q)
    u = t - base.astype(np.float64)
    W, D = [], []
    for j in range(q + 1):
        v = np.ones_like(u)
        for m in range(q + 1):
            if m != j:
                v = v * (u - float(m)) / float(j - m)
        dv = np.zeros_like(u)
        for l in range(q + 1):
            if l == j:
                continue
            w = np.ones_like(u) / float(j - l)
            for m in range(q + 1):
                if m != j and m != l:
                    w = w * (u - float(m)) / float(j - m)
            dv = dv + w
        W.append(v)
        D.append(dv)
    return base, W, D


def _grid(p, X, grad, S):
    q, lo, hi, N = int(p[0]), float(p[1]), float(p[2]), int(p[3])
    h = (hi - lo) / N
    d = len(X)
    S = np.asarray(S, dtype=np.float64).reshape(-1)
    ax = [_axis_weights(X[a], lo, h, N, q) for a in range(d)]
    n1 = N + 1
    val = np.zeros(np.shape(X[0]))
    gr = [np.zeros(np.shape(X[0])) for _ in range(d)]
    for blk in np.ndindex(*(q + 1,) * d):
        j = blk[::-1]                    # j[0] (x) varies fastest
        idx = ax[0][0] + j[0]
        mul = n1
        for a in range(1, d):
            idx = idx + (ax[a][0] + j[a]) * mul
            mul = mul * n1
        s = S[idx]
        w = ax[0][1][j[0]]
        for a in range(1, d):
            w = w * ax[a][1][j[a]]
        val = val + w * s
        for g in range(d):
            c = ax[0][2][j[0]] if g == 0 else ax[0][1][j[0]]
            for a in range(1, d):
                c = c * (ax[a][2][j[a]] if g == a else ax[a][1][j[a]])
            gr[g] = gr[g] + c * s
    if not grad:
        return val
    return tuple(gg / h for gg in gr)


def H(iface, X):
    """Level-set value at points X = (x, y[, z]) (arrays of equal shape)."""
    kind, p = iface[0], iface[1]
    if kind == "grid":
        return _grid(p, X, False, iface[2])
    return _FUN[kind](np.asarray(p, dtype=np.float64), X, False)


def gradH(iface, X):
    """Gradient of H at points X, as a tuple of d arrays."""
    kind, p = iface[0], iface[1]
    if kind == "grid":
        return _grid(p, X, True, iface[2])
    return _FUN[kind](np.asarray(p, dtype=np.float64), X, True)


def normal(iface, X):
    """Unit outward normal n = grad H / |grad H| (Sec. 5.1)."""
    g = gradH(iface, X)
    s = g[0] * g[0] + g[1] * g[1]
    if len(g) == 3:
        s = s + g[2] * g[2]
    nrm = np.sqrt(s)
    return tuple(gi / nrm for gi in g)

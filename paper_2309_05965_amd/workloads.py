"""Seeded synthetic workloads: problem descriptors and manufactured solutions.

This module holds input generators only, none of the method's arithmetic.  It
serves both the HIP library (tests, bench) and the CPU oracle: each side
computes its own surface points, then asks this module for the data at those
points.

A problem is a dict
    dim, order (2|4), N, lo, hi, beta_in, beta_out, kappa (reduced reaction
    coefficient kappa_i / beta_i), cos_alpha, ifaces = [(kind, params), ...]
with the level-set parameter layouts of the library header.  A manufactured
solution gives, per region s (0 = exterior, k = interior of interface k), a
smooth function u_s with its gradient and Laplacian; from it
    fhat_s = Lap u_s - kappa u_s,   g1 = u_k - u_0,
    g2 = beta_in d_n u_k - beta_out d_n u_0,  ftilde = fhat_k - fhat_0,
    gB = u_0 on the box boundary.
"""
import math

import numpy as np

SEED_BATCH = 2309059654


# ----------------------------------------------------------------------------
# level-set parameter vectors
# ----------------------------------------------------------------------------
def ellipse2d(cx, cy, a, b, theta=0.0):
    c = 1.0 if theta == 0.0 else math.cos(theta)
    s = 0.0 if theta == 0.0 else math.sin(theta)
    return ("ellipse2d", [cx, cy, c, s, a, b])


def star2d(cx, cy, c0, A=None, B=None):
    A = (list(A) if A is not None else []) + [0.0] * 8
    B = (list(B) if B is not None else []) + [0.0] * 8
    return ("star2d", [cx, cy, c0] + A[:8] + B[:8])


def sphere3d(cx, cy, cz, r):
    return ("sphere3d", [cx, cy, cz, r])


def ellipsoid3d(c, axes, R):
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    return ("ellipsoid3d", list(c) + list(axes) + R.ravel().tolist())


def torus3d(cx, cy, cz, R, r):
    return ("torus3d", [cx, cy, cz, R, r])


def product3d(cx, cy, cz, s):
    return ("product3d", [cx, cy, cz, s])


def molecule3d(level, r, atoms):
    atoms = [float(v) for a in atoms for v in a]
    return ("molecule3d", [level, r, len(atoms) // 3] + atoms)


# ----------------------------------------------------------------------------
# manufactured functions: each returns (value, grad tuple, laplacian)
# ----------------------------------------------------------------------------
def f_exp_cos(X):                       # exp(x) cos(y)
    x, y = X[0], X[1]
    e = np.exp(x)
    return e * np.cos(y), (e * np.cos(y), -e * np.sin(y)), 0.0 * x


def f_sin_sin(X):                       # sin(x) sin(y)
    x, y = X[0], X[1]
    v = np.sin(x) * np.sin(y)
    return v, (np.cos(x) * np.sin(y), np.sin(x) * np.cos(y)), -2.0 * v


def f_cos2x_expy(X):                    # cos(2x) exp(y)
    x, y = X[0], X[1]
    v = np.cos(2 * x) * np.exp(y)
    return v, (-2 * np.sin(2 * x) * np.exp(y), v), -3.0 * v


def f_x2_my3(X):                        # x^2 - y^3
    x, y = X[0], X[1]
    return x * x - y ** 3, (2 * x, -3 * y * y), 2.0 - 6.0 * y


def f_sin3(X):                          # sin x sin y sin z
    x, y, z = X
    sx, sy, sz = np.sin(x), np.sin(y), np.sin(z)
    cx, cy, cz = np.cos(x), np.cos(y), np.cos(z)
    v = sx * sy * sz
    return v, (cx * sy * sz, sx * cy * sz, sx * sy * cz), -3.0 * v


def f_exp3(X):                          # exp(x + y + z) / 10
    x, y, z = X
    v = np.exp(x + y + z) / 10.0
    return v, (v, v, v), 3.0 * v


def f_e1(X):                            # exp(x) sin(cos(pi/3) x + sin(pi/3) y)
    x, y = X[0], X[1]
    c, s = 0.5, math.sqrt(3.0) / 2.0
    e = np.exp(x)
    t = c * x + s * y
    st, ct = np.sin(t), np.cos(t)
    return e * st, (e * st + c * e * ct, s * e * ct), 2.0 * c * e * ct


def f_e3(X):                            # exp(z) (cos 2x + cos 3y)
    x, y, z = X
    e = np.exp(z)
    c2, c3 = np.cos(2 * x), np.cos(3 * y)
    return e * (c2 + c3), (-2 * e * np.sin(2 * x), -3 * e * np.sin(3 * y), e * (c2 + c3)), e * (-3 * c2 - 8 * c3)


def f_e4(X):                            # exp(z) (cos 5x + cos 2y)
    x, y, z = X
    e = np.exp(z)
    c5, c2 = np.cos(5 * x), np.cos(2 * y)
    return e * (c5 + c2), (-5 * e * np.sin(5 * x), -2 * e * np.sin(2 * y), e * (c5 + c2)), e * (-24 * c5 - 3 * c2)


def f_e5_in(X):                         # sin^2(2x) cos^2(2y) cos z
    x, y, z = X
    A, B, C = np.sin(2 * x) ** 2, np.cos(2 * y) ** 2, np.cos(z)
    A1, B1, C1 = 2 * np.sin(4 * x), -2 * np.sin(4 * y), -np.sin(z)
    A2, B2 = 8 * np.cos(4 * x), -8 * np.cos(4 * y)
    return A * B * C, (A1 * B * C, A * B1 * C, A * B * C1), A2 * B * C + A * B2 * C - A * B * C


def f_cos3(X):                          # cos x cos y cos z
    x, y, z = X
    cx, cy, cz = np.cos(x), np.cos(y), np.cos(z)
    v = cx * cy * cz
    return v, (-np.sin(x) * cy * cz, -cx * np.sin(y) * cz, -cx * cy * np.sin(z)), -3.0 * v


def f_e2_in(X):                         # exp(0.6 x + 0.8 y)
    x, y = X[0], X[1]
    e = np.exp(0.6 * x + 0.8 * y)
    return e, (0.6 * e, 0.8 * e), e


def f_e2_out(X):                        # sin(pi (x+1)/2) sin(pi (y+1)/2)
    x, y = X[0], X[1]
    k = math.pi / 2.0
    sx, sy = np.sin(k * (x + 1)), np.sin(k * (y + 1))
    return sx * sy, (k * np.cos(k * (x + 1)) * sy, k * sx * np.cos(k * (y + 1))), -2.0 * k * k * sx * sy


def f_zero(X):
    z = 0.0 * X[0]
    return z, tuple(z for _ in X), z


def polynomial(coef):
    """Polynomial sum c * x^a y^b (z^c) from {(a, b[, c]): c}."""
    items = list(coef.items())

    def f(X):
        d = len(X)
        v = 0.0 * X[0]
        g = [0.0 * X[0] for _ in range(d)]
        lap = 0.0 * X[0]
        for e, c in items:
            def mon(ee):
                if any(t < 0 for t in ee):
                    return 0.0 * X[0]
                out = 1.0 + 0.0 * X[0]
                for a in range(d):
                    out = out * X[a] ** ee[a]
                return out
            v = v + c * mon(e)
            for a in range(d):
                ea = list(e); ea[a] -= 1
                g[a] = g[a] + c * e[a] * mon(ea)
                eaa = list(e); eaa[a] -= 2
                lap = lap + c * e[a] * (e[a] - 1) * mon(eaa)
        return v, tuple(g), lap
    return f


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------
def problem(dim, order, N, lo, hi, beta_in, beta_out, kappa, ifaces, cos_alpha=0.5):
    return {"dim": dim, "order": order, "N": int(N), "lo": float(lo), "hi": float(hi),
            "beta_in": float(beta_in), "beta_out": float(beta_out), "kappa": float(kappa),
            "cos_alpha": float(cos_alpha), "ifaces": list(ifaces)}


def config1(N=64):
    """2D Poisson, 2nd order, ellipse x^2 + y^2/0.36 = 1 in [-1.5, 1.5]^2,
    beta 2/1, u_in = exp(x) cos y, u_out = sin x sin y."""
    prob = problem(2, 2, N, -1.5, 1.5, 2.0, 1.0, 0.0, [ellipse2d(0.0, 0.0, 1.0, 0.6)])
    return prob, {0: f_sin_sin, 1: f_exp_cos}


def config2(N=512):
    """2D 4th order, star r = 0.5 + 0.15 sin 5t in [-1, 1]^2, beta 1000/1,
    reduced kappa 1, u_in = cos 2x exp y, u_out = x^2 - y^3."""
    B = [0.0] * 8
    B[4] = 0.15
    prob = problem(2, 4, N, -1.0, 1.0, 1000.0, 1.0, 1.0, [star2d(0.0, 0.0, 0.5, None, B)])
    return prob, {0: f_x2_my3, 1: f_cos2x_expy}


def config3(N=128):
    """3D 4th order, torus (R 0.6, r 0.25) plus a concentric sphere of radius
    0.35 - 2h (gap 2h to the torus), box [-1, 1]^3, beta 1/100, kappa 0,
    u_in = sin x sin y sin z in both interiors, u_out = exp(x+y+z)/10."""
    h = 2.0 / N
    prob = problem(3, 4, N, -1.0, 1.0, 1.0, 100.0, 0.0,
                   [torus3d(0.0, 0.0, 0.0, 0.6, 0.25), sphere3d(0.0, 0.0, 0.0, 0.35 - 2.0 * h)])
    return prob, {0: f_exp3, 1: f_sin3, 2: f_sin3}


# ----------------------------------------------------------------------------
# level sets given only at the grid nodes (Sec. 7)
# ----------------------------------------------------------------------------
def sampled(prob, H, q=5):
    """A level set known only by its values H(node) at the nodes of the
    problem's grid, read through the degree-q interpolant of the library:
    ("grid", [q, lo, hi, N], samples) with samples[(z,) y, x]."""
    G = grid_coords(prob)
    S = np.array(np.broadcast_to(H(G), G[0].shape), dtype=np.float64)
    return ("grid", [float(q), prob["lo"], prob["hi"], float(prob["N"])], S)


def H_sphere(cx, cy, cz, r):
    return lambda X: (X[0] - cx) ** 2 + (X[1] - cy) ** 2 + (X[2] - cz) ** 2 - r * r


def H_torus(R, r):
    return lambda X: (np.sqrt(X[0] ** 2 + X[1] ** 2) - R) ** 2 + X[2] ** 2 - r * r


def H_star(c0, eps, m):
    """rho - c0 (1 + eps sin(m theta)) with theta = atan2(y, x)."""
    return lambda X: np.sqrt(X[0] ** 2 + X[1] ** 2) - c0 * (1.0 + eps * np.sin(m * np.arctan2(X[1], X[0])))


def with_sampled(prob, H, q=5):
    """The problem with its single interface replaced by the sampled H."""
    return dict(prob, ifaces=[sampled(prob, H, q)])


# ----------------------------------------------------------------------------
# interior boundary value problems (Sec. 2.1): Omega = the interiors
# ----------------------------------------------------------------------------
BIE_KINDS = ("interface", "dirichlet", "neumann")


def bvp_problem(dim, order, N, lo, hi, kappa, ifaces, bie, cos_alpha=0.5):
    """An interior Dirichlet or Neumann problem Lap u - kappa u = fhat in the
    interiors of ifaces (beta_in and beta_out are not used: 1 and 0)."""
    prob = problem(dim, order, N, lo, hi, 1.0, 0.0, kappa, ifaces, cos_alpha)
    prob["bie"] = bie
    return prob


def e1_dirichlet(N=64):
    """2D Poisson Dirichlet problem on the rotated ellipse a = 1, b = 0.5,
    theta = -pi/6 in [-1.2, 1.2]^2, 4th order, u = exp(x) sin(cos(pi/3) x +
    sin(pi/3) y) (paper Sec. 6.1.1, Table 2d-poi-o4)."""
    prob = bvp_problem(2, 4, N, -1.2, 1.2, 0.0, [ellipse2d(0.0, 0.0, 1.0, 0.5, -math.pi / 6.0)], "dirichlet")
    return prob, f_e1


def e3_neumann(N=64):
    """3D Poisson Neumann problem in the torus (1 - sqrt(x^2+y^2))^2 + z^2 <
    0.4^2, box [-1.5, 1.5]^3, 4th order, u = exp(z)(cos 2x + cos 3y)
    (Sec. 6.2.1, Table 3d-neu-poi)."""
    prob = bvp_problem(3, 4, N, -1.5, 1.5, 0.0, [torus3d(0.0, 0.0, 0.0, 1.0, 0.4)], "neumann")
    return prob, f_e3


def e4_dirichlet(N=64):
    """3D modified-Helmholtz Dirichlet problem, kappa = 100, in
    (1+4x^2)(1+4y^2)(1+4z^2) + 64xyz + 4x^2 + 4y^2 + 4z^2 < 3, box
    [-0.7, 0.7]^3, 4th order, u = exp(z)(cos 5x + cos 2y) (Sec. 6.2.2,
    Table 3d-Diri-Hel)."""
    prob = bvp_problem(3, 4, N, -0.7, 0.7, 100.0, [product3d(0.0, 0.0, 0.0, 2.0)], "dirichlet")
    return prob, f_e4


def make_bvp_data(prob, u, surf_pos, surf_nrm, pde_pts):
    """Data of an interior BVP at the solver's query points: g2 = u
    (Dirichlet) or d_n u (Neumann) on all surface points, ftilde = fhat at
    the PDE points (the exterior extension is zero), fhat per region (zero
    in region 0), no box data."""
    X = _cols(surf_pos)
    v, gr, _ = u(X)
    if prob["bie"] == "dirichlet":
        g2 = np.array(np.broadcast_to(v, X[0].shape), dtype=np.float64)
    else:
        n = np.asarray(surf_nrm, dtype=np.float64)
        g2 = sum(np.asarray(gr[a]) * n[:, a] for a in range(n.shape[1]))
    ft = np.array(fhat_fn(prob, u)(_cols(pde_pts)), dtype=np.float64)
    G = grid_coords(prob)
    K = len(prob["ifaces"])
    f_in = np.broadcast_to(fhat_fn(prob, u)(G), G[0].shape)
    fhat = np.stack([np.zeros(G[0].shape)] + [f_in] * K)
    return {"g1": None, "g2": g2, "ftilde": ft, "fhat": fhat, "gB": None}


def bvp_exact(prob, u):
    """u at every node (compare on the nodes of Omega only)."""
    G = grid_coords(prob)
    return np.array(np.broadcast_to(u(G)[0], G[0].shape))


def e2_circles_star(N=64, r=0.3826):
    """Poisson interface problem with eight circles of radius r centred at
    (cos(m pi/4), sin(m pi/4)) and a five-fold star r(t) = 0.514 (1 + 0.2 sin
    5t) in [-1.7, 1.7]^2, sigma_i = 1, sigma_e = 3, u_i = exp(0.6x + 0.8y),
    u_e = sin(pi(x+1)/2) sin(pi(y+1)/2) (paper Sec. 6.1.2, Table
    2d-poi-ifp-mul).  The printed r = 0.383 makes neighbouring circles
    overlap by 6e-4 (their centres are 2 sin(pi/8) = 0.76537 apart): r =
    0.3826 keeps them 1.5e-4 apart; the star's angle is read as atan2."""
    B = [0.0] * 8
    B[4] = 0.514 * 0.2
    ifs = [ellipse2d(math.cos(m * math.pi / 4), math.sin(m * math.pi / 4), r, r) for m in range(1, 9)]
    ifs.append(star2d(0.0, 0.0, 0.514, None, B))
    prob = problem(2, 4, N, -1.7, 1.7, 1.0, 3.0, 0.0, ifs)
    sol = {0: f_e2_out}
    for k in range(1, 10):
        sol[k] = f_e2_in
    return prob, sol


def e6_touching(N=64):
    """Poisson interface problem with a torus (1 - sqrt(x^2+y^2))^2 + z^2 =
    0.4^2 and the ellipsoid x^2/0.36 + y^2/0.36 + z^2 = 1, which touch along
    the circle x^2 + y^2 = 0.36, z = 0, in [-1.5, 1.5]^3, sigma_i = 1,
    sigma_e = 3, u = sin^2(2x) cos^2(2y) cos z in the torus, exp(z)(cos 2x +
    cos 3y) in the ellipsoid, cos x cos y cos z outside (paper Sec. 6.2.4,
    Table poi-ifp-3d-toch-cur)."""
    prob = problem(3, 4, N, -1.5, 1.5, 1.0, 3.0, 0.0,
                   [torus3d(0.0, 0.0, 0.0, 1.0, 0.4), ellipsoid3d((0.0, 0.0, 0.0), (0.6, 0.6, 1.0), np.eye(3))])
    return prob, {0: f_cos3, 1: f_e5_in, 2: f_e3}


MOLECULE_ATOMS = ((math.sqrt(3.0) / 3.0, 0.0, -math.sqrt(6.0) / 12.0),
                  (-math.sqrt(3.0) / 6.0, 0.5, -math.sqrt(6.0) / 12.0),
                  (-math.sqrt(3.0) / 6.0, -0.5, -math.sqrt(6.0) / 12.0),
                  (0.0, 0.0, math.sqrt(6.0) / 4.0))


def e5_molecule(N=128, ratio=10.0, r=0.5):
    """Poisson interface problem with the four-atom molecular surface sum_k
    exp(-|x - x_k|^2 / r^2) = 0.6 in [-1.2, 1.2]^3, sigma_i = 1, sigma_e =
    ratio, u_i = sin^2(2x) cos^2(2y) cos z, u_e = cos x cos y cos z (paper
    Sec. 6.2.3, Table 3d-ifp-ratio).  The paper does not give the atom
    radius r: 0.5 is taken."""
    prob = problem(3, 4, N, -1.2, 1.2, 1.0, float(ratio), 0.0, [molecule3d(0.6, r, MOLECULE_ATOMS)])
    return prob, {0: f_cos3, 1: f_e5_in}


# ----------------------------------------------------------------------------
# two-density interface problems (eq. bie-ifp-1): kappa_i / sigma_i may differ
# ----------------------------------------------------------------------------
def td_problem(dim, order, N, lo, hi, sigma_in, sigma_out, kappa_in, kappa_out, ifaces, cos_alpha=0.5):
    """sigma_i Lap u - kappa_i u = f_i; kappa and kappa_out are the reduced
    coefficients kappa_i / sigma_i inside and outside."""
    prob = problem(dim, order, N, lo, hi, sigma_in, sigma_out, kappa_in, ifaces, cos_alpha)
    prob["bie"] = "two_density"
    prob["kappa_out"] = float(kappa_out)
    return prob


def e7_heterogeneous(N=64):
    """Three spheres of radius 0.7 centred at (0.5, 0.5, 0.5), (-0.5, -0.5,
    0.5), (0.5, -0.5, -0.5), sigma_i = 1, kappa_i = 0, sigma_e = 4, kappa_e =
    10 (Poisson inside, modified Helmholtz outside; paper Sec. 6.2.5, Table
    3d-ifp-heter).  The paper gives neither the box nor the exact solution:
    box [-1.5, 1.5]^3 (its printed N_b fits this box) and u_i = sin x sin y
    sin z, u_e = exp(x + y + z) / 10."""
    sph = [sphere3d(0.5, 0.5, 0.5, 0.7), sphere3d(-0.5, -0.5, 0.5, 0.7), sphere3d(0.5, -0.5, -0.5, 0.7)]
    prob = td_problem(3, 4, N, -1.5, 1.5, 1.0, 4.0, 0.0, 10.0 / 4.0, sph)
    return prob, {0: f_exp3, 1: f_sin3, 2: f_sin3, 3: f_sin3}


def make_td_data(prob, sol, surf_pos, surf_nrm, surf_iface, pde_pts, cen_iface):
    """Data of a two-density problem at the solver's query points: g1 = u_k -
    u_0, g2 = sigma_in d_n u_k - sigma_out d_n u_0 on all surface points;
    ftilde = (fhat_in, fhat_out) at the PDE points, shape (2, Nb, nP), with
    fhat_s = Lap u_s - kappa~_s u_s; fhat per region; gB = u_0."""
    K = len(prob["ifaces"])
    kap = lambda s: prob["kappa_out"] if s == 0 else prob["kappa"]
    X = _cols(surf_pos)
    k = np.asarray(surf_iface)
    n = np.asarray(surf_nrm, dtype=np.float64)
    v0, gr0, _ = sol[0](X)
    dn0 = sum(np.asarray(gr0[a]) * n[:, a] for a in range(n.shape[1]))
    g1 = np.zeros(k.size)
    g2 = np.zeros(k.size)
    for kk in range(1, K + 1):
        vk, grk, _ = sol[kk](X)
        dnk = sum(np.asarray(grk[a]) * n[:, a] for a in range(n.shape[1]))
        g1 = np.where(k == kk, vk - v0, g1)
        g2 = np.where(k == kk, prob["beta_in"] * dnk - prob["beta_out"] * dn0, g2)

    def fh(s, Y):
        v, _, lap = sol[s](Y)
        return lap - kap(s) * v
    Xp = _cols(pde_pts)
    fin = np.zeros(np.asarray(pde_pts).shape[:-1])
    for kk in range(1, K + 1):
        fin = np.where(np.asarray(cen_iface)[:, None] == kk, fh(kk, Xp), fin)
    fout = np.broadcast_to(fh(0, Xp), fin.shape)
    G = grid_coords(prob)
    fhat = np.stack([np.broadcast_to(fh(s, G), G[0].shape) for s in range(K + 1)])
    gB = np.array(np.broadcast_to(sol[0](G)[0], G[0].shape))
    return {"g1": g1, "g2": g2, "ftilde": np.stack([fin, fout]), "fhat": fhat, "gB": gB}


def two_circles(order=4, N=64, gap=0.5, kappa=0.4):
    """Two disjoint circles (radii 0.27, 0.21) in [-1, 1]^2 whose closest
    points are gap * h apart along a direction 0.35 rad from the x axis;
    beta 1/3.  A gap below one grid spacing puts stencil neighbours inside
    both interiors (the multi-crossing case of the corrected scheme)."""
    h = 2.0 / N
    r1, r2 = 0.27, 0.21
    c1 = (-0.3, 0.013)
    dist = r1 + r2 + gap * h
    c2 = (c1[0] + dist * math.cos(0.35), c1[1] + dist * math.sin(0.35))
    return problem(2, order, N, -1.0, 1.0, 1.0, 3.0, kappa,
                   [ellipse2d(c1[0], c1[1], r1, r1), ellipse2d(c2[0], c2[1], r2, r2)])


def two_spheres(N=64, gap=0.5, order=4, kappa=0.3):
    """Two disjoint spheres (radii 0.33, 0.27) in [-1, 1]^3, closest points
    gap * h apart; beta 1/4."""
    h = 2.0 / N
    r1, r2 = 0.33, 0.27
    c1 = np.array([-0.31, 0.021, -0.017])
    u = np.array([math.cos(0.3) * math.cos(0.2), math.sin(0.3) * math.cos(0.2), math.sin(0.2)])
    c2 = c1 + (r1 + r2 + gap * h) * u
    return problem(3, order, N, -1.0, 1.0, 1.0, 4.0, kappa,
                   [sphere3d(*c1.tolist(), r1), sphere3d(*c2.tolist(), r2)])


def config4_batch(n=512, seed=SEED_BATCH):
    """Random stars r(t) = 0.4 + sum_{k=2..8} a_k cos(k t + p_k),
    a_k ~ U(0, 0.04), p_k ~ U(0, 2 pi), log10 beta_in ~ U(-2, 2), beta_out = 1,
    N ~ U{64, 128, 256, 512}, reduced kappa 1, config-2 solution."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(rng.choice([64, 128, 256, 512]))
        a = rng.uniform(0.0, 0.04, size=7)
        ph = rng.uniform(0.0, 2.0 * math.pi, size=7)
        beta_in = 10.0 ** rng.uniform(-2.0, 2.0)
        A = [0.0] * 8
        B = [0.0] * 8
        for j, k in enumerate(range(2, 9)):
            A[k - 1] = a[j] * math.cos(ph[j])
            B[k - 1] = -a[j] * math.sin(ph[j])
        prob = problem(2, 4, N, -1.0, 1.0, beta_in, 1.0, 1.0, [star2d(0.0, 0.0, 0.4, A, B)])
        out.append((prob, {0: f_x2_my3, 1: f_cos2x_expy}))
    return out


# ----------------------------------------------------------------------------
# data at query points
# ----------------------------------------------------------------------------
def _cols(P):
    P = np.asarray(P, dtype=np.float64)
    return tuple(P[..., a] for a in range(P.shape[-1]))


def grid_coords(prob):
    d, N = prob["dim"], prob["N"]
    h = (prob["hi"] - prob["lo"]) / N
    x1 = prob["lo"] + np.arange(N + 1, dtype=np.float64) * h
    out = []
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = N + 1
        out.append(np.broadcast_to(x1.reshape(shape), (N + 1,) * d))
    return tuple(out)


def fhat_fn(prob, fun):
    def f(X):
        v, _, lap = fun(X)
        return lap - prob["kappa"] * v
    return f


def make_data(prob, sol, surf_pos, surf_nrm, surf_iface, pde_pts, cen_iface):
    """Data of the interface problem at the solver's own query points.
    surf_pos, surf_nrm: (Ns, d) surface points; surf_iface: (Ns,) 1-based;
    pde_pts: (Nb, nP, d) PDE collocation points of the centres, whose
    interfaces are cen_iface (Nb,).  g1, g2 are returned on all surface
    points."""
    dof_pos, dof_nrm, dof_iface = surf_pos, surf_nrm, surf_iface
    K = len(prob["ifaces"])
    X = _cols(dof_pos)
    k = np.asarray(dof_iface)
    n = np.asarray(dof_nrm, dtype=np.float64)
    v0, g0, _ = sol[0](X)
    g1 = np.zeros(k.size)
    g2 = np.zeros(k.size)
    for kk in range(1, K + 1):
        m = k == kk
        vk, gk, _ = sol[kk](X)
        dn_k = sum(np.asarray(gk[a]) * n[:, a] for a in range(n.shape[1]))
        dn_0 = sum(np.asarray(g0[a]) * n[:, a] for a in range(n.shape[1]))
        g1 = np.where(m, vk - v0, g1)
        g2 = np.where(m, prob["beta_in"] * dn_k - prob["beta_out"] * dn_0, g2)
    Xp = _cols(pde_pts)
    f0 = fhat_fn(prob, sol[0])(Xp)
    ft = np.zeros(np.asarray(pde_pts).shape[:-1])
    for kk in range(1, K + 1):
        fk = fhat_fn(prob, sol[kk])(Xp)
        ft = np.where(np.asarray(cen_iface)[:, None] == kk, fk - f0, ft)
    G = grid_coords(prob)
    fhat = np.stack([np.broadcast_to(fhat_fn(prob, sol[s])(G), G[0].shape) for s in range(K + 1)])
    gB = np.array(np.broadcast_to(sol[0](G)[0], G[0].shape))
    return {"g1": g1, "g2": g2, "ftilde": ft, "fhat": fhat, "gB": gB}


def exact_solution(prob, sol, reg):
    """u_{reg(node)} at every node."""
    G = grid_coords(prob)
    u = np.zeros(G[0].shape)
    for s in sol:
        u = np.where(reg == s, np.broadcast_to(sol[s](G)[0], G[0].shape), u)
    return u


def exact_density(prob, sol, dof_pos, dof_nrm, dof_iface):
    """psi = [d_n u] = d_n u_k - d_n u_0 at the DOFs."""
    X = _cols(dof_pos)
    n = np.asarray(dof_nrm, dtype=np.float64)
    _, g0, _ = sol[0](X)
    k = np.asarray(dof_iface)
    out = np.zeros(k.size)
    for kk in set(k.tolist()):
        _, gk, _ = sol[kk](X)
        dn = sum((np.asarray(gk[a]) - np.asarray(g0[a])) * n[:, a] for a in range(n.shape[1]))
        out = np.where(k == kk, dn, out)
    return out


# ----------------------------------------------------------------------------
# learned warm start: random ellipsoids with random Fourier jump data
# ----------------------------------------------------------------------------
N_SAMPLES = 1024
N_MODES = 8


def fourier_wavevectors():
    """k_m = (pi/2) (m & 1, (m >> 1) & 1, (m >> 2) & 1), m = 0..7."""
    return np.array([[(m >> b) & 1 for b in range(3)] for m in range(N_MODES)], dtype=np.float64) * (math.pi / 2)


def config5(seed, N=128):
    """One learned-warm-start problem: an ellipsoid centred at the origin with
    semi-axes ~ U(0.3, 0.7) and orientation Q from the QR factorisation of a
    3x3 standard normal matrix (columns signed so that diag(R) > 0), box
    [-1, 1]^3, 4th order, kappa 0, beta_in 1, beta_out 100, fhat = 0, gB = 0,
    and jumps g_j(x) = sum_m a_jm cos(k_m . x) + b_jm sin(k_m . x), j = 1, 2,
    a, b ~ N(0, 1).  Returns (prob, geom, jumps) with geom = (centre,
    axes, Q) and jumps = (a, b) of shape (2, 8) each."""
    rng = np.random.default_rng(seed)
    axes = rng.uniform(0.3, 0.7, size=3)
    G = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))[None, :]
    a = rng.standard_normal((2, N_MODES))
    b = rng.standard_normal((2, N_MODES))
    centre = np.zeros(3)
    prob = problem(3, 4, N, -1.0, 1.0, 1.0, 100.0, 0.0, [ellipsoid3d(centre, axes, Q)])
    return prob, (centre, axes, Q), (a, b)


def jump_values(jumps, X):
    """(g1, g2) at points X (n, 3)."""
    a, b = jumps
    ph = np.asarray(X, dtype=np.float64) @ fourier_wavevectors().T      # (n, 8)
    c, s = np.cos(ph), np.sin(ph)
    return c @ a[0] + s @ b[0], c @ a[1] + s @ b[1]


def fibonacci_sphere(n=N_SAMPLES):
    """Fibonacci lattice on the unit sphere: z_i = 1 - (2i+1)/n,
    phi_i = i pi (3 - sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(1.0 - z * z)
    ph = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


def jump_data(prob, jumps, surf_pos):
    """Solver data of a config-5 problem at the solver's surface points."""
    g1, g2 = jump_values(jumps, surf_pos)
    N, d = prob["N"], prob["dim"]
    return {"g1": g1, "g2": g2, "ftilde": None, "fhat": None, "gB": None}

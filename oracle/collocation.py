"""Mesh-free collocation for the local Cauchy problems (paper Secs. 5.3.1 and
5.4, eqs. cau-appro / cau-ls).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For every centre p_i the local correction polynomial is
    C_{h,i}(x) = sum_{|alpha| <= p} U_alpha xi^alpha,   xi = (x - p_i) / h,
and U solves the square system M U = Q whose rows are
    PDE rows       (Lap_xi - kappa h^2) xi^alpha at xi = o_j   = h^2 ftilde(x_j)
    Dirichlet rows xi^alpha at xi_j                            = a(x_j)
    Neumann rows   n_j . grad_xi xi^alpha at xi_j              = h b(x_j)
(the h-scaling of the rows is the scaled-coordinate remark of Sec. 5.4).
Monomials are in graded order: total degree m = 0..p, and inside one degree
the exponent of x descending, then of y descending.
"""
import numpy as np


def exponents(d, p):
    out = []
    for m in range(p + 1):
        if d == 2:
            for j in range(m + 1):
                out.append((m - j, j))
        else:
            for a in range(m, -1, -1):
                for b in range(m - a, -1, -1):
                    out.append((a, b, m - a - b))
    return np.array(out, dtype=np.int64)


def _pow(x, e):
    """x**e for an integer array e >= 0 by repeated multiplication
    1 * x * x * ... (elementwise; x**0 = 1, and x**e = 0 for e < 0, which
    only occurs multiplied by a zero factor)."""
    x = np.asarray(x, dtype=np.float64)
    e = np.asarray(e)
    if e.ndim == 1 and x.ndim >= 1 and x.shape[-1] == 1:
        # one column of bases, one row of exponents: the same products from
        # a table of the bases' powers 1, 1*x, (1*x)*x, ...
        tab = [np.ones(x.shape[:-1])]
        for _ in range(int(e.max(initial=0))):
            tab.append(tab[-1] * x[..., 0])
        T = np.stack(tab, axis=-1)
        return np.where(e >= 0, T[..., np.maximum(e, 0)], 0.0)
    e = np.broadcast_to(e, np.broadcast_shapes(np.shape(x), np.shape(e)))
    x = np.broadcast_to(x, e.shape)
    r = np.where(e >= 0, 1.0, 0.0)
    for k in range(int(e.max(initial=0))):
        r = np.where(e > k, r * x, r)
    return r


def mono(xi, E):
    """Monomial values xi^alpha: xi (..., d) -> (..., n_alpha), the product
    taken axis by axis, 1 * x^a * y^b (* z^c)."""
    v = np.ones(xi.shape[:-1] + (E.shape[0],))
    for a in range(E.shape[1]):
        v = v * _pow(xi[..., a:a + 1], E[:, a])
    return v


def mono_grad(xi, E):
    """Gradient of every monomial: (..., d, n_alpha); component a is
    alpha_a * x^(.) * y^(.) (* z^(.)) with the a-th exponent lowered."""
    d = E.shape[1]
    out = []
    for a in range(d):
        v = np.broadcast_to(E[:, a].astype(np.float64), xi.shape[:-1] + (E.shape[0],))
        for b in range(d):
            e = E[:, b] - (1 if b == a else 0)
            v = v * _pow(xi[..., b:b + 1], e)
        out.append(v)
    return np.stack(out, axis=-2)


def mono_lap(xi, E):
    """Laplacian of every monomial: (..., n_alpha)."""
    d = E.shape[1]
    tot = np.zeros(xi.shape[:-1] + (E.shape[0],))
    for a in range(d):
        v = np.broadcast_to((E[:, a] * (E[:, a] - 1)).astype(np.float64), xi.shape[:-1] + (E.shape[0],))
        for b in range(d):
            e = E[:, b] - (2 if b == a else 0)
            v = v * _pow(xi[..., b:b + 1], e)
        tot = tot + v
    return tot


def assemble(geo):
    """Collocation matrices M_i for every centre, shape (Nb, n, n), rows in
    the order [PDE | Dirichlet | Neumann]."""
    prob = geo["prob"]
    d = prob["dim"]
    p = 4 if prob["order"] == 4 else 2
    h = geo["h"]
    E = exponents(d, p)
    surf = geo["surf"]
    st = geo["st"]
    P = geo["dofs"]["pos"]
    S = surf["pos"]
    Nb = P.shape[0]
    offP = np.array(st["offP"], dtype=np.float64).reshape(-1, d)
    # PDE rows: xi = o exactly
    lap = mono_lap(offP, E)                      # (nP, n)
    val = mono(offP, E)
    rowsP = lap - (prob["kappa"] * h * h) * val
    rowsP = np.broadcast_to(rowsP, (Nb,) + rowsP.shape)
    xiD = (S[st["D"]] - P[:, None, :]) / h       # (Nb, nD, d)
    rowsD = mono(xiD.reshape(-1, d), E).reshape(Nb, -1, E.shape[0])
    xiN = (S[st["N"]] - P[:, None, :]) / h
    g = mono_grad(xiN.reshape(-1, d), E).reshape(Nb, st["N"].shape[1], d, E.shape[0])
    nN = surf["nrm"][st["N"]]                    # (Nb, nN, d)
    rowsN = np.zeros(g.shape[:2] + (E.shape[0],))
    for a in range(d):
        rowsN = rowsN + nN[:, :, a:a + 1] * g[:, :, a, :]
    return np.concatenate([rowsP, rowsD, rowsN], axis=1)


def factor(geo):
    """Inverse of every M_i (LAPACK LU through numpy) and its 1-norm
    condition number; cond > 1e10 counts as singular (Sec. 5.4: the system
    is uniquely solvable and cond ~ 1e2-1e3)."""
    M = assemble(geo)
    Minv = np.linalg.inv(M)
    cond = np.abs(M).sum(axis=1).max(axis=1) * np.abs(Minv).sum(axis=1).max(axis=1)
    return M, Minv, cond


def solve(M, Minv, Q):
    """U with M U = Q for every centre, to full working accuracy: the
    product with the inverse followed by one step of iterative refinement
    whose residual Q - M U is formed in extended precision (long double),
    so the result is the rounded exact solution of the square system of
    Sec. 5.4 rather than one that depends on how the inverse was formed."""
    U = np.einsum("iab,ib->ia", Minv, Q)
    r = np.asarray(Q, dtype=np.longdouble)
    Ml = M.astype(np.longdouble)
    Ul = U.astype(np.longdouble)
    for a in range(M.shape[2]):
        r = r - Ml[:, :, a] * Ul[:, a:a + 1]
    return U + np.einsum("iab,ib->ia", Minv, r.astype(np.float64))


def rhs(geo, a, b, ftilde):
    """Right-hand sides Q_i = [h^2 ftilde(pde pts); a(D pts); h b(N pts)].
    a, b: arrays over the surface-point table (or None = 0);
    ftilde: (Nb, nP) or None."""
    st = geo["st"]
    h = geo["h"]
    Nb = geo["dofs"]["pos"].shape[0]
    nP = len(st["offP"])
    qP = np.zeros((Nb, nP)) if ftilde is None else (h * h) * np.asarray(ftilde)
    qD = np.zeros(st["D"].shape) if a is None else np.asarray(a)[st["D"]]
    qN = np.zeros(st["N"].shape) if b is None else h * np.asarray(b)[st["N"]]
    return np.concatenate([qP, qD, qN], axis=1)

"""Simple interface solve, KFBI operator, GMRES and the full interface solve.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Problem (Sec. 2.2, divided by beta_i as in Sec. 3.2, eq. bie-ifp-2):
    Lap u - kappa u = fhat_i in Omega_i,  [u] = g1,  [beta d_n u] = g2,
    u = gB on the box boundary;  [.] = interior minus exterior.
Unknown density psi = [d_n u] on the surface points (Sec. 3.2).

simple_solve  w(a, b, ftilde, fhat, gB): the constant-coefficient interface
    problem of eq. con-ifp (Sec. 4, eq. equi-ifp) with box data gB:
    Step 3.1 local Cauchy problems (collocation), Step 3.2 corrected RHS
    (eqs. corrected-FDS / crc-formula, multi-crossing remark), Step 3.3 box
    solve, Step 3.4 corrected interpolation of the normal derivative
    (Sec. 5.5).
matvec  A psi = J[w(0, psi, 0, 0, 0)] / (beta_in + beta_out) with the flux jump
    J = beta_in d_n w_in - beta_out d_n w_out.  This equals
    psi/2 + mu K' psi of Sec. 3.2 (mu = (beta_out - beta_in)/(beta_out + beta_in)).
rhs     b = (g2 - J[w(g1, 0, ftilde, fhat, gB)]) / (beta_in + beta_out)
    (Alg. 1 Step 1).
gmres   unrestarted GMRES with modified Gram-Schmidt and Givens rotations,
    stop at |r_k| <= tol |b| (Alg. 1 Step 4).
solve   psi* = GMRES(A, b), u = w(g1, psi*, ftilde, fhat, gB).
"""
import numpy as np

from . import collocation, fd, geometry


class Plan:
    """Geometry (S0) and collocation factorisation (S1) of one problem."""

    def __init__(self, prob):
        self.prob = prob
        self.geo = geometry.build(prob)
        self.M, self.Minv, self.cond = collocation.factor(self.geo)
        if np.any(~np.isfinite(self.cond)) or np.max(self.cond) > 1e10:
            raise geometry.GeometryError("singular", "collocation matrix is singular")
        d = prob["dim"]
        self.d = d
        self.N = prob["N"]
        self.h = self.geo["h"]
        self.p = 4 if prob["order"] == 4 else 2
        self.E = collocation.exponents(d, self.p)
        self.A, self.B = fd.stencils(d, prob["order"], self.h, prob["kappa"])
        self.K = len(prob["ifaces"])
        self.Nb = self.geo["dofs"]["pos"].shape[0]
        self.lin = [int(np.nonzero((self.E == np.eye(d, dtype=np.int64)[a]).all(axis=1))[0][0])
                    for a in range(d)]
        self._interp_weights()

    # ------------------------------------------------------------------
    def _interp_weights(self):
        """Gradient weights of the tensor-product Lagrange interpolant of
        degree q on the (q+1)^d block of every DOF (Sec. 5.5)."""
        q = self.p
        d = self.d
        t = (self.geo["dofs"]["pos"] - self.prob["lo"]) / self.h
        s = t - self.geo["blocks"]                    # local coordinate in [0, q]
        nodes = np.arange(q + 1, dtype=np.float64)
        Nb = self.Nb
        val = np.zeros((Nb, d, q + 1))
        der = np.zeros((Nb, d, q + 1))
        for j in range(q + 1):
            others = [m for m in range(q + 1) if m != j]
            v = np.ones((Nb, d))
            for m in others:
                v = v * (s - nodes[m]) / (nodes[j] - nodes[m])
            val[:, :, j] = v
            dv = np.zeros((Nb, d))
            for l in others:
                w = np.ones((Nb, d)) / (nodes[j] - nodes[l])
                for m in others:
                    if m != l:
                        w = w * (s - nodes[m]) / (nodes[j] - nodes[m])
                dv = dv + w
            der[:, :, j] = dv
        self.ival, self.ider = val, der

    # ------------------------------------------------------------------
    def node_coords(self, nodes):
        ind = geometry.unravel(nodes, self.prob)
        return np.stack([self.prob["lo"] + ind[a].astype(np.float64) * self.h
                         for a in range(self.d)], axis=1)

    def simple_solve(self, a=None, b=None, ftilde=None, fhat=None, gB=None, trace=False):
        """Grid solution v (full grid, box boundary = gB), one-sided normal
        derivatives (d_n v_in, d_n v_out) at the DOFs (with trace=True the
        one-sided values (v_in, v_out) instead; with trace="both" the pairs
        (v_in, v_out) and (d_n v_in, d_n v_out)), and U.  a, b are given on
        the whole surface-point table; ftilde at the PDE points."""
        geo = self.geo
        d, N, h = self.d, self.N, self.h
        Q = collocation.rhs(geo, a, b, ftilde)
        U = collocation.solve(self.M, self.Minv, Q)
        # correction function at the entries (closest-centre partition of unity)
        own = geo["cowner"]
        X = self.node_coords(geo["cnode"])
        xi = (X - geo["dofs"]["pos"][own]) / h
        Cv = np.einsum("ea,ea->e", collocation.mono(xi, self.E), U[own])
        reg = geo["reg"]
        flat = reg.ravel()
        Cg = np.zeros((self.K + 1, flat.size))
        Cg[geo["ck"], geo["cnode"]] = Cv
        # right-hand side on the interior
        F = np.zeros((N - 1,) * d)
        if fhat is not None:
            core = reg[(slice(1, N),) * d]
            for s in range(self.K + 1):
                Bs = fd.apply(self.B, np.asarray(fhat[s]))
                F = np.where(core == s, Bs, F)
        if gB is not None:
            g = np.array(gB, dtype=np.float64)
            g[(slice(1, N),) * d] = 0.0
            F = F - fd.apply(self.A, g)
        Ff = F.ravel().copy()
        irr = geo["irr"]
        ind = geometry.unravel(irr, self.prob)
        rp = flat[irr]
        corr = np.zeros(irr.size)
        for o, c in self.A.items():
            qn = geometry.ravel([ind[x] + o[x] for x in range(d)], self.prob)
            rq = flat[qn]
            m = rq != rp
            corr[m] -= c * (Cg[rp[m], qn[m]] - Cg[rq[m], qn[m]])
        iind = [v - 1 for v in ind]
        F_lin = np.zeros(irr.size, dtype=np.int64)
        mul = 1
        for x in range(d):
            F_lin += iind[x] * mul
            mul *= (N - 1)
        np.add.at(Ff, F_lin, corr)
        vin = fd.dst_solve(Ff.reshape(F.shape), d, self.prob["order"], N, h, self.prob["kappa"])
        v = np.zeros((N + 1,) * d) if gB is None else np.array(gB, dtype=np.float64)
        v[(slice(1, N),) * d] = vin
        # corrected interpolation at the DOFs (Sec. 5.5)
        if trace == "both":
            return v, self.traces(v, Cg, U), self.normal_derivatives(v, Cg, U), U
        if trace:
            v_in, v_out = self.traces(v, Cg, U)
            return v, v_in, v_out, U
        dn_in, dn_out = self.normal_derivatives(v, Cg, U)
        return v, dn_in, dn_out, U

    def _smoothed_block(self, vf, flat, Cg, U, blk):
        """Grid values of the block node blk of every DOF, made smooth
        across the interface as normal_derivatives describes."""
        geo = self.geo
        dofs = geo["dofs"]
        ind = [geo["blocks"][:, a] + blk[a] for a in range(self.d)]
        qn = geometry.ravel(ind, self.prob)
        rq = flat[qn]
        xi = (self.node_coords(qn) - dofs["pos"]) / self.h
        Cown = (collocation.mono(xi, self.E) * U).sum(axis=1)
        return vf[qn] + np.where(rq != dofs["iface"], Cown - Cg[rq, qn], 0.0)

    def traces(self, v, Cg, U):
        """One-sided values at the DOFs (Sec. 5.5, which obtains the value
        and the derivatives of the smooth extension v_h^+ at p from the same
        interpolation): the value of the tensor-product Lagrange interpolant
        of the smoothed block data at p is v_in(p), and v_out(p) =
        v_in(p) - C_{h,p}(p), the constant coefficient of p's polynomial."""
        d, q = self.d, self.p
        flat = self.geo["reg"].ravel()
        vf = v.ravel()
        val = np.zeros(self.Nb)
        for blk in np.ndindex(*(q + 1,) * d):
            vt = self._smoothed_block(vf, flat, Cg, U, blk)
            w = np.ones(self.Nb)
            for a in range(d):
                w = w * self.ival[:, a, blk[a]]
            val += w * vt
        c0 = int(np.nonzero((self.E == 0).all(axis=1))[0][0])
        return val, val - U[:, c0]

    def normal_derivatives(self, v, Cg, U):
        """One-sided normal derivatives at the DOFs (Sec. 5.5).  The grid
        values of the block of DOF p are made smooth across the interface by
        adding, at every node q outside p's own region k, the jump
        u_k - u_reg(q) = C^(k)(q) - C^(reg q)(q); C^(k) is p's own local
        correction polynomial C_{h,p} (the Taylor expansion is taken at p),
        C^(reg q) for another interface's interior is its partition-of-unity
        value, and C^(0) = 0.  Then d_n v_in(p) is the normal derivative of
        the tensor-product Lagrange interpolant and d_n v_out(p) =
        d_n v_in(p) - d_n C_{h,p}(p)."""
        geo = self.geo
        d, h, q = self.d, self.h, self.p
        dofs = geo["dofs"]
        flat = geo["reg"].ravel()
        vf = v.ravel()
        kk = dofs["iface"]
        grad = np.zeros((self.Nb, d))
        for blk in np.ndindex(*(q + 1,) * d):
            ind = [geo["blocks"][:, a] + blk[a] for a in range(d)]
            qn = geometry.ravel(ind, self.prob)
            rq = flat[qn]
            xi = (self.node_coords(qn) - dofs["pos"]) / h
            Cown = (collocation.mono(xi, self.E) * U).sum(axis=1)
            vt = vf[qn] + np.where(rq != kk, Cown - Cg[rq, qn], 0.0)
            for a in range(d):
                w = self.ider[:, a, blk[a]] / h
                for b in range(d):
                    if b != a:
                        w = w * self.ival[:, b, blk[b]]
                grad[:, a] += w * vt
        n = dofs["nrm"]
        dn_in = (n * grad).sum(axis=1)
        dnC = (n * U[:, self.lin]).sum(axis=1) / h
        return dn_in, dn_in - dnC

    # ------------------------------------------------------------------
    def flux(self, dn_in, dn_out):
        return self.prob["beta_in"] * dn_in - self.prob["beta_out"] * dn_out

    def extend(self, psi):
        """Density on the whole surface-point table from its primary values."""
        idx = self.geo["ext_idx"]
        w = self.geo["ext_w"]
        return (w * np.where(idx >= 0, np.asarray(psi)[np.maximum(idx, 0)], 0.0)).sum(axis=1)

    def dof_values(self, arr_s):
        return np.asarray(arr_s)[self.geo["dofs"]["sidx"]]

    def matvec(self, psi):
        _, dn_in, dn_out, _ = self.simple_solve(b=self.extend(psi))
        return self.flux(dn_in, dn_out) / (self.prob["beta_in"] + self.prob["beta_out"])

    def rhs(self, data):
        _, dn_in, dn_out, _ = self.simple_solve(a=data["g1"], ftilde=data["ftilde"],
                                                fhat=data["fhat"], gB=data["gB"])
        return (self.dof_values(data["g2"]) - self.flux(dn_in, dn_out)) / (self.prob["beta_in"] + self.prob["beta_out"])

    def solve(self, data, tol=1e-10, maxit=200, psi0=None):
        b = self.rhs(data)
        psi, its, hist = gmres(self.matvec, b, psi0, tol, maxit)
        v, _, _, _ = self.simple_solve(a=data["g1"], b=self.extend(psi), ftilde=data["ftilde"],
                                       fhat=data["fhat"], gB=data["gB"])
        r = b - self.matvec(psi)
        nb = np.linalg.norm(b)
        return {"psi": psi, "u": v, "iters": its, "hist": hist, "b": b,
                "true_rel_res": np.linalg.norm(r) / (nb if nb > 0 else 1.0)}


def gmres(matvec, b, x0, tol, maxit):
    """Unrestarted GMRES (modified Gram-Schmidt, Givens rotations); stops when
    the residual estimate |g_{k}| <= tol |b|.  Returns (x, iterations, history
    of relative residual estimates)."""
    n = b.size
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    r0 = b - matvec(x0) if np.any(x0) else b.copy()
    beta = np.linalg.norm(r0)
    hist = [beta / (nb if nb > 0 else 1.0)]
    if nb == 0.0 or beta <= tol * nb:
        return x0.copy(), 0, hist
    V = np.zeros((maxit + 1, n))
    Hm = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = r0 / beta
    k = 0
    for j in range(maxit):
        w = matvec(V[j])
        for i in range(j + 1):
            Hm[i, j] = np.dot(w, V[i])
            w = w - Hm[i, j] * V[i]
        Hm[j + 1, j] = np.linalg.norm(w)
        breakdown = not Hm[j + 1, j] > 0.0
        if not breakdown:
            V[j + 1] = w / Hm[j + 1, j]
        for i in range(j):
            t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
            Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
            Hm[i, j] = t
        den = np.hypot(Hm[j, j], Hm[j + 1, j])
        cs[j] = Hm[j, j] / den
        sn[j] = Hm[j + 1, j] / den
        Hm[j, j] = den
        Hm[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / nb)
        if abs(g[j + 1]) <= tol * nb or breakdown:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - np.dot(Hm[i, i + 1:k], y[i + 1:k])) / Hm[i, i]
    return x0 + V[:k].T @ y, k, hist


def error_norms(u_num, u_exact, mask):
    """||e||_2 = sqrt(mean |e|^2) and ||e||_inf over the nodes in mask
    (Sec. 6)."""
    e = (u_num - u_exact)[mask]
    return float(np.sqrt(np.mean(e * e))), float(np.max(np.abs(e)))

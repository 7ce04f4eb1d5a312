"""Two-density interface BIE (eq. bie-ifp-1, Sec. 3.2) by the KFBI method.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Problem (Sec. 2.2): sigma_i Lap u - kappa_i u = f_i in Omega_i, Omega_1 the
union of the interiors (sigma_1 = beta_in, reduced kappa~_1 = kappa),
Omega_2 the exterior (sigma_2 = beta_out, kappa~_2 = kappa_out), [u] =
u_1 - u_2 = g1, [sigma d_n u] = g2 on Gamma, u = gB on the box.  Unlike the
single-density form this allows kappa_1 / sigma_1 != kappa_2 / sigma_2.
Unknowns phi = u_1 and psi = sigma_2 d_n u_2 on Gamma.

W_i(a, b, F; gB) is the simple interface problem of Sec. 4 for
Lap - kappa~_i with [W] = a, [d_n W] = b (fhat_s = F in region s).  The
function equal to u_1 in Omega_1 and 0 in Omega_2 is W_1(u_1, d_n u_1,
fhat_1 1_Omega_1), and the one equal to 0 in Omega_1 and u_2 in Omega_2 is
W_2(-u_2, -d_n u_2, fhat_2 1_Omega_2; gB), so the averages of their
one-sided traces on Gamma are u_1/2 and u_2/2, and of sigma_i times their
normal derivatives sigma_1 d_n u_1 / 2 and sigma_2 d_n u_2 / 2.  With
u_2 = phi - g1, d_n u_1 = (psi + g2) / sigma_1, d_n u_2 = psi / sigma_2,
adding the two value relations and the two flux relations gives exactly
eq. bie-ifp-1 (K_i = K~_i, S_i = S~_i / sigma_i, D_i = sigma_i H~_i for the
Green's functions of Lap - kappa~_i), i.e. with avg = (in + out) / 2:
    A [phi; psi] = [phi - avg W_1(phi, psi/sigma_1) + avg W_2(phi, psi/sigma_2);
                    psi - sigma_1 avg d_n W_1(phi, psi/sigma_1)
                        + sigma_2 avg d_n W_2(phi, psi/sigma_2)]
    b = [g1/2 + avg R_1 + avg R_2;  -g2/2 + sigma_1 avg d_n R_1 + sigma_2 avg d_n R_2]
with R_1 = W_1(0, g2/sigma_1, fhat_1 1_Omega_1) and R_2 = W_2(g1, 0,
fhat_2 1_Omega_2; gB).  Each product takes one simple solve per Green's
function: the two box solves per iteration of the superposition remark
after Alg. 1.  The solution is u_1 = W_1(phi, (psi + g2)/sigma_1, ...) on
Omega_1 and u_2 = W_2(g1 - phi, -psi/sigma_2, ...; gB) on Omega_2.

Data: g1, g2 on the surface points; ftilde = (fhat_1, fhat_2) at the PDE
collocation points, shape (2, Nb, nP); fhat (K+1, nodes) with fhat_2 in
region 0 and fhat_1 in the interiors; gB on the box boundary.
"""
import numpy as np

from . import kfbi


class TwoDensityPlan:
    """Two plans of one geometry, for Lap - kappa~_1 and Lap - kappa~_2."""

    def __init__(self, prob):
        if prob.get("bie") != "two_density":
            raise ValueError("bie must be 'two_density'")
        self.prob = prob
        self.s1, self.s2 = float(prob["beta_in"]), float(prob["beta_out"])
        self.p1 = kfbi.Plan(dict(prob, kappa=prob["kappa"]))
        self.p2 = kfbi.Plan(dict(prob, kappa=prob["kappa_out"]))
        self.geo = self.p1.geo
        self.Nb = self.p1.Nb
        self.K = self.p1.K

    def _avgs(self, plan, **kw):
        v, (vin, vout), (din, dout), _ = plan.simple_solve(trace="both", **kw)
        return v, 0.5 * (vin + vout), 0.5 * (din + dout)

    def matvec(self, x):
        n = self.Nb
        return self.apply_surface(self.p1.extend(x[:n]), self.p1.extend(x[n:]), x[:n], x[n:])

    def apply_surface(self, a, b, phi, psi):
        """The operator with the densities given on the whole surface-point
        table (a = phi, b = psi there) and at the DOFs (phi, psi)."""
        _, v1, d1 = self._avgs(self.p1, a=a, b=b / self.s1)
        _, v2, d2 = self._avgs(self.p2, a=a, b=b / self.s2)
        return np.concatenate([phi - v1 + v2, psi - self.s1 * d1 + self.s2 * d2])

    def _split_f(self, data):
        """fhat_1 1_Omega_1 and fhat_2 1_Omega_2 per region, and their jumps
        across Gamma at the PDE points (fhat_1 - 0 and 0 - fhat_2)."""
        fh = np.asarray(data["fhat"])
        f1 = np.zeros_like(fh)
        f1[1:] = fh[1:]
        f2 = np.zeros_like(fh)
        f2[0] = fh[0]
        ft = np.asarray(data["ftilde"])
        return f1, f2, ft[0], -ft[1]

    def rhs(self, data):
        f1, f2, t1, t2 = self._split_f(data)
        g1 = self.p1.dof_values(data["g1"])
        g2 = self.p1.dof_values(data["g2"])
        _, v1, d1 = self._avgs(self.p1, b=np.asarray(data["g2"]) / self.s1, ftilde=t1, fhat=f1)
        _, v2, d2 = self._avgs(self.p2, a=np.asarray(data["g1"]), ftilde=t2, fhat=f2, gB=data["gB"])
        return np.concatenate([0.5 * g1 + v1 + v2, -0.5 * g2 + self.s1 * d1 + self.s2 * d2])

    def solution(self, x, data):
        n = self.Nb
        f1, f2, t1, t2 = self._split_f(data)
        a = self.p1.extend(x[:n])
        b = self.p1.extend(x[n:])
        u1, _, _, _ = self.p1.simple_solve(a=a, b=(b + np.asarray(data["g2"])) / self.s1, ftilde=t1, fhat=f1)
        u2, _, _, _ = self.p2.simple_solve(a=np.asarray(data["g1"]) - a, b=-b / self.s2, ftilde=t2, fhat=f2,
                                           gB=data["gB"])
        return np.where(self.geo["reg"] > 0, u1, u2)

    def solve(self, data, tol=1e-10, maxit=300, x0=None):
        b = self.rhs(data)
        x, its, hist = kfbi.gmres(self.matvec, b, x0, tol, maxit)
        r = b - self.matvec(x)
        nb = np.linalg.norm(b)
        return {"x": x, "phi": x[:self.Nb], "psi": x[self.Nb:], "u": self.solution(x, data), "iters": its,
                "hist": hist, "b": b, "true_rel_res": np.linalg.norm(r) / (nb if nb > 0 else 1.0)}

"""Interior Dirichlet and Neumann boundary value problems by the KFBI method.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Problem (Sec. 2.1, divided by sigma):  Lap u - kappa u = fhat in Omega, the
union of the interiors of the interfaces, with u = gD or d_n u = gN on
Gamma (gN = g_N / sigma).  The box Green's function G vanishes on the box
boundary (Sec. 3.1); the volume potential N fhat extends fhat by zero
outside Omega (Sec. 4), so its simple interface problems have fhat_0 = 0 and
the jump ftilde = fhat at the PDE collocation points.

Dirichlet, eq. bie-D:  u = D phi + N fhat in Omega.  D phi solves the simple
interface problem with [u] = phi, [d_n u] = 0 (Sec. 4, eq. equi-ifp), and
its interior limit on Gamma is (1/2 + K) phi, so with the one-sided value of
the corrected interpolation (Sec. 5.5)
    A_D phi = w_in(E phi, 0, 0, 0)            b_D = gD - w_in(0, 0, ftilde, fhat).
Neumann, eq. bie-N:  u = -S psi + N fhat.  -S psi solves [u] = 0,
[d_n u] = psi, and its interior normal derivative is (1/2 - K') psi:
    A_N psi = d_n w_in(0, E psi, 0, 0)        b_N = gN - d_n w_in(0, 0, ftilde, fhat).
With kappa = 0 the interior Neumann problem fixes u only up to a constant
and A_N has a one-dimensional null space; following Sec. 6.2.1 the
right-hand side and every product are shifted to zero mean (the plain mean
over the DOFs).  The solution is w(E phi, 0, ftilde, fhat) resp.
w(0, E psi, ftilde, fhat) with zero box data, read at the nodes of Omega.

The problem dict is the interface problem's with "bie" = "dirichlet" or
"neumann"; beta_in and beta_out are not used.
"""
import numpy as np

from . import kfbi


class BVPPlan(kfbi.Plan):
    """Plan (S0 + S1) of an interior boundary value problem."""

    def __init__(self, prob):
        if prob.get("bie") not in ("dirichlet", "neumann"):
            raise ValueError("bie must be 'dirichlet' or 'neumann'")
        super().__init__(prob)
        self.kind = prob["bie"]
        self.project = self.kind == "neumann" and prob["kappa"] == 0.0

    def _zero_mean(self, x):
        return x - np.mean(x) if self.project else x

    def _interior(self, **kw):
        """Interior one-sided value (Dirichlet) or normal derivative
        (Neumann) at the DOFs of the simple solve with these data."""
        _, t_in, _, _ = self.simple_solve(trace=self.kind == "dirichlet", **kw)
        return t_in

    def matvec(self, x):
        if self.kind == "dirichlet":
            return self._interior(a=self.extend(x))
        return self._zero_mean(self._interior(b=self.extend(x)))

    def rhs(self, data):
        g = self.dof_values(data["g2"])
        return self._zero_mean(g - self._interior(ftilde=data["ftilde"], fhat=data["fhat"]))

    def solution(self, x, data):
        """Grid solution w with the density x (all nodes; Omega's are the
        solution of the problem)."""
        if self.kind == "dirichlet":
            v, _, _, _ = self.simple_solve(a=self.extend(x), ftilde=data["ftilde"], fhat=data["fhat"])
        else:
            v, _, _, _ = self.simple_solve(b=self.extend(x), ftilde=data["ftilde"], fhat=data["fhat"])
        return v

    def solve(self, data, tol=1e-10, maxit=200, x0=None):
        b = self.rhs(data)
        x, its, hist = kfbi.gmres(self.matvec, b, x0, tol, maxit)
        r = b - self.matvec(x)
        nb = np.linalg.norm(b)
        return {"density": x, "u": self.solution(x, data), "iters": its, "hist": hist, "b": b,
                "true_rel_res": np.linalg.norm(r) / (nb if nb > 0 else 1.0)}

    def omega_mask(self):
        """Nodes of Omega (inside some interface)."""
        return self.geo["reg"] > 0


def gauge_error_norms(u_num, u_exact, mask, anchor):
    """Error norms (Sec. 6) after adding the constant that makes the
    numerical solution match the exact one at the node `anchor` (flat
    index) - the Neumann solution's normalisation of Sec. 6.2.1."""
    c = u_exact.ravel()[anchor] - u_num.ravel()[anchor]
    return kfbi.error_norms(u_num + c, u_exact, mask)

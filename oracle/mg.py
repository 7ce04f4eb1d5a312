"""Geometric multigrid box solver and the FP64 defect-correction loop around
FP32 V-cycles (the mixed-precision form of the box solve).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The box solve of Alg. 1 Step 3.3 is A_h v = F on the interior nodes with
v = 0 on the box boundary (A_h the compact operator of fd.stencils).  The
paper solves it with the FFT; multigrid is the other solver of that step
named for the GPU build, and its converged result has a plain definition:
the same A_h^-1 F that fd.dst_solve computes exactly.

Multigrid (a textbook two-grid method, written out plainly):
  levels      the fine grid N and the coarse grid N/2, the same compact
              operator rediscretised with h_c = 2 h and the same reduced
              kappa;
  smoother    damped Jacobi u <- u + (omega / a) (f - A u), a the central
              stencil coefficient, omega = 2 / (rho_lo + rho_hi) with
              [rho_lo, rho_hi] the range of the symbol lambda(theta)/a over
              the high frequencies (max_k theta_k >= pi/2), sampled on a 64^d
              grid of theta in (0, pi];
  restriction full weighting, the tensor product of (1/4, 1/2, 1/4) about the
              fine node 2I, formed in the inner precision and taken to FP64;
  coarse      the coarse system solved exactly in FP64: the rediscretised
              operator is diagonal in the type-I sine basis (fd.dst_solve);
  prolongation (bi/tri)linear interpolation of the FP64 coarse correction,
              P = 2^d R^T, rounded to the inner precision and added;
  cycle       nu1 pre-smoothing steps from a zero initial guess, the coarse
              correction, nu2 post-smoothing steps: (nu1, nu2) = (2, 2).
Defect correction: r = F - A_h v in FP64; stop when |r|_2 <= eps |F|_2;
otherwise e = (cycles V-cycles on r in the inner precision), v <- v + e.
"""
import numpy as np

from . import fd


def central(st):
    return st[tuple([0] * len(next(iter(st))))]


def symbol(st, theta):
    """lambda(theta) = sum_o c_o cos(o . theta) of a symmetric stencil
    (theta: (..., d), theta[..., a] along axis a)."""
    out = np.zeros(theta.shape[:-1])
    for o, c in st.items():
        out = out + c * np.cos(sum(o[a] * theta[..., a] for a in range(len(o))))
    return out


def jacobi_weight(st, d, samples=64):
    """omega = 2 / (rho_lo + rho_hi) over the high frequencies; returns
    (omega, rho_lo, rho_hi)."""
    t = np.pi * np.arange(1, samples + 1) / samples
    grids = np.meshgrid(*([t] * d), indexing="ij")
    theta = np.stack(grids, axis=-1).reshape(-1, d)
    high = theta.max(axis=1) >= np.pi / 2
    rho = symbol(st, theta[high]) / central(st)
    lo, hi = rho.min(), rho.max()
    return 2.0 / (lo + hi), lo, hi


def apply_full(st, u):
    """A u on the interior, returned as a full grid with a zero boundary."""
    out = np.zeros_like(u)
    out[(slice(1, -1),) * u.ndim] = fd.apply(st, u).astype(u.dtype)
    return out


def restrict(r):
    """Full weighting of a full fine grid (size 2n+1 per axis) to the coarse
    interior (size n+1 per axis, zero boundary)."""
    d = r.ndim
    nf = r.shape[0] - 1
    nc = nf // 2
    out = np.zeros((nc + 1,) * d, dtype=r.dtype)
    w1 = {-1: 0.25, 0: 0.5, 1: 0.25}
    for off in np.ndindex(*(3,) * d):
        o = [x - 1 for x in off]
        w = 1.0
        for x in o:
            w *= w1[x]
        sl = tuple(slice(2 + o[j], nf - 1 + o[j], 2) for j in range(d))
        out[(slice(1, nc),) * d] += r.dtype.type(w) * r[sl]
    return out


def prolong(e):
    """(Bi/tri)linear interpolation of a coarse full grid (zero boundary) to
    the fine full grid."""
    d = e.ndim
    nc = e.shape[0] - 1
    nf = 2 * nc
    out = np.zeros((nf + 1,) * d, dtype=e.dtype)
    # every fine node is the average of the coarse nodes at the corners of
    # the coarse cell face / edge it lies on
    for par in np.ndindex(*(2,) * d):
        # fine nodes with parity par: index 2I + par
        sl_f = tuple(slice(p, nf + 1 - (1 if p else 0), 2) for p in par)
        acc = np.zeros(out[sl_f].shape, dtype=e.dtype)
        cnt = 0
        for corner in np.ndindex(*(2,) * d):
            if any(c and not p for c, p in zip(corner, par)):
                continue
            sl_c = tuple(slice(c, c + out[sl_f].shape[j]) for j, c in enumerate(corner))
            acc = acc + e[sl_c]
            cnt += 1
        out[sl_f] = acc / e.dtype.type(cnt)
    return out


class Hierarchy:
    """Fine operator, its central coefficient and Jacobi weight, and the
    coarse grid of the two-grid cycle."""

    def __init__(self, d, order, N, h, kappa, dtype=np.float64):
        self.d, self.order, self.N, self.h, self.kappa = d, order, N, h, kappa
        self.dtype = np.dtype(dtype)
        A, _ = fd.stencils(d, order, h, kappa)
        self.ops = [A]
        self.a = central(A)
        self.w = jacobi_weight(A, d)[0]
        self.Nc = N // 2
        self.hc = 2.0 * h

    def coarse_solve(self, fc):
        """A_c^-1 f_c on the coarse interior (FP64, zero boundary)."""
        d, Nc = self.d, self.Nc
        ec = np.zeros((Nc + 1,) * d)
        ec[(slice(1, Nc),) * d] = fd.dst_solve(fc[(slice(1, Nc),) * d], d, self.order, Nc, self.hc, self.kappa)
        return ec

    def vcycle(self, f, nu=(2, 2)):
        """One two-grid cycle (nu1, nu2) from a zero initial guess, in the
        inner precision, with the coarse correction in FP64."""
        dt = self.dtype.type
        A, a, w = self.ops[0], self.a, self.w
        u = np.zeros_like(f)
        for _ in range(nu[0]):
            u = u + dt(w / a) * (f - apply_full(A, u))
            u = u * _interior_mask(u)
        r = (f - apply_full(A, u)) * _interior_mask(f)
        ec = self.coarse_solve(restrict(r).astype(np.float64))
        u = u + prolong(ec).astype(self.dtype)
        for _ in range(nu[1]):
            u = u + dt(w / a) * (f - apply_full(A, u))
            u = u * _interior_mask(u)
        return u


def _interior_mask(u):
    m = np.zeros(u.shape, dtype=u.dtype)
    m[(slice(1, -1),) * u.ndim] = 1
    return m


def solve(F, d, order, N, h, kappa, eps=1e-12, inner=np.float64, cycles=1, nu=(2, 2), maxit=100):
    """Defect correction around two-grid cycles in the inner precision.
    F: interior right-hand side ((N-1)^d).  Returns (v interior, outer
    iterations, relative residual history)."""
    hier = Hierarchy(d, order, N, h, kappa, inner)
    A = hier.ops[0]
    v = np.zeros((N + 1,) * d)
    Ff = np.zeros((N + 1,) * d)
    Ff[(slice(1, N),) * d] = F
    nF = np.linalg.norm(F)
    hist = []
    for it in range(maxit + 1):
        r = Ff - apply_full(A, v)
        rel = np.linalg.norm(r) / (nF if nF > 0 else 1.0)
        hist.append(rel)
        if rel <= eps or it == maxit:
            break
        e = np.zeros_like(r, dtype=hier.dtype)
        ri = r.astype(hier.dtype)
        for _ in range(cycles):
            e = e + hier.vcycle(ri - apply_full(hier.ops[0], e), nu)
        v = v + e.astype(np.float64)
    return v[(slice(1, N),) * d], it, hist

"""ctypes binding of libkfbi.so (C ABI in include/kfbi.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device memory and streams come from PyTorch: arrays are
torch tensors on a HIP device, passed by data_ptr(), and the plan's work is
ordered on the torch stream current at plan creation.  The binding raises
if the library is not built; there is no fallback path.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkfbi.so")

KINDS = {"ellipse2d": 1, "star2d": 2, "sphere3d": 3, "ellipsoid3d": 4, "torus3d": 5, "product3d": 6, "molecule3d": 7, "grid": 8}
BIE = {"interface": 0, "dirichlet": 1, "neumann": 2, "two_density": 3}
STATUS = {0: "OK", 1: "INVALID", 2: "UNRESOLVED", 3: "SINGULAR", 4: "NOT_CONVERGED",
          5: "NONFINITE", 6: "DEVICE", 7: "OOM"}
EXPORT = {"region": 0, "surf_pos": 1, "surf_nrm": 2, "surf_meta": 3, "dof_surf": 4,
          "stencil_d": 5, "stencil_n": 6, "ext_idx": 7, "ext_w": 8, "pde_pts": 9,
          "irregular": 10, "corr": 11, "cond": 12, "dof_pos": 13}

c_double_p = ctypes.c_void_p


class LevelSet(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("p", ctypes.c_double * 32)]


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("order", ctypes.c_int32), ("N", ctypes.c_int32),
                ("n_iface", ctypes.c_int32), ("bie", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("beta_in", ctypes.c_double), ("beta_out", ctypes.c_double),
                ("kappa", ctypes.c_double), ("cos_alpha", ctypes.c_double),
                ("kappa_out", ctypes.c_double), ("iface", LevelSet * 10), ("samples", ctypes.c_void_p * 10)]


class Sizes(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_surf", ctypes.c_int64), ("n_dof", ctypes.c_int64),
                ("n_irregular", ctypes.c_int64), ("n_corr", ctypes.c_int64),
                ("n_pde", ctypes.c_int32), ("n_dir", ctypes.c_int32), ("n_neu", ctypes.c_int32),
                ("n_coef", ctypes.c_int32), ("h", ctypes.c_double), ("cond_max", ctypes.c_double)]


class Data(ctypes.Structure):
    _fields_ = [("g1", c_double_p), ("g2", c_double_p), ("ftilde", c_double_p),
                ("fhat", c_double_p), ("gB", c_double_p)]


class Learned(ctypes.Structure):
    _fields_ = [("mlp", ctypes.c_void_p), ("nb", ctypes.c_int32), ("geom", ctypes.c_void_p),
                ("jumps", ctypes.c_void_p), ("scale", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("start", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("max_cycles", ctypes.c_int32), ("eps_in", ctypes.c_double),
                ("relax", ctypes.c_double), ("learned", ctypes.c_void_p)]


START = {"zero": 0, "given": 1, "learned": 2}
SOLVER = {None: 0, "fft": 1, "mg64": 2, "mg32": 3}
DATA_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_void_p)


def make_opts(tol, max_iter, start="zero", solver=None, eps_in=0.0, max_cycles=0, relax=0.0, learned=None):
    """kfbi_opts (learned: a Learned struct, kept alive by the caller)."""
    return Opts(float(tol), int(max_iter), START[start], SOLVER[solver], int(max_cycles), float(eps_in),
                float(relax), ctypes.cast(ctypes.pointer(learned), ctypes.c_void_p) if learned is not None else None)


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("est_rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double)]


ABI = {
    "kfbi_plan_create": ([ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "kfbi_plan_setup": ([ctypes.c_void_p, ctypes.POINTER(Problem)], ctypes.c_int),
    "kfbi_plan_sizes": ([ctypes.c_void_p, ctypes.POINTER(Sizes)], ctypes.c_int),
    "kfbi_plan_export": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "kfbi_box_solve": ([ctypes.c_void_p, c_double_p, c_double_p], ctypes.c_int),
    "kfbi_simple_solve": ([ctypes.c_void_p] + [c_double_p] * 8, ctypes.c_int),
    "kfbi_matvec": ([ctypes.c_void_p, c_double_p, c_double_p], ctypes.c_int),
    "kfbi_rhs": ([ctypes.c_void_p, ctypes.POINTER(Data), c_double_p], ctypes.c_int),
    "kfbi_solve": ([ctypes.c_void_p, ctypes.POINTER(Data), ctypes.POINTER(Opts), c_double_p, c_double_p,
                    ctypes.POINTER(Info)], ctypes.c_int),
    "kfbi_plan_set_box_solver": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "kfbi_plan_set_box_relaxation": ([ctypes.c_void_p, ctypes.c_double], ctypes.c_int),
    "kfbi_plan_box_stats": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
                            ctypes.c_int),
    "kfbi_plan_profile": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "kfbi_plan_timing": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "kfbi_plan_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "kfbi_box_solve_noalloc": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, c_double_p, c_double_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_tile_lines": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "kfbi_set_tile_lines": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "kfbi_batch_create": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
                          ctypes.c_int),
    "kfbi_batch_sizes": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
                         ctypes.c_int),
    "kfbi_batch_solve": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_batch_solve_stream": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_batch_setup": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_batch_plan": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "kfbi_plan_stream": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "kfbi_batch_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_create": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                         ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "kfbi_mlp_sizes": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "kfbi_mlp_set_params": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_get_params": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_forward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_loss_grad": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_train_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                             ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "kfbi_gemm_bf16": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                        ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p],
                       ctypes.c_int),
    "kfbi_ellipsoid_features": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_sh_transfer": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                          ctypes.c_double, ctypes.c_void_p], ctypes.c_int),
    "kfbi_sh_sample": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                        ctypes.c_double, ctypes.c_void_p], ctypes.c_int),
    "kfbi_scale_jumps": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "kfbi_real_sh": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_forward_lin": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_loss_grad_lin": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_mlp_train_step_lin": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p], ctypes.c_int),
    "kfbi_geometry_input": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "kfbi_sh_coefficients": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p],
                             ctypes.c_int),
    "kfbi_sh_expand": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p],
                       ctypes.c_int),
    "kfbi_learned_start": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_double, ctypes.c_void_p], ctypes.c_int),
    "kfbi_last_error": ([], ctypes.c_char_p),
}

_lib = None


def load():
    """Open libkfbi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkfbi.so is not built (python -m paper_2309_05965_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in ABI.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


class KfbiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


def _check(st):
    if st != 0:
        raise KfbiError(st, load().kfbi_last_error().decode())


def problem_struct(prob, samples=None):
    s = Problem()
    s.dim, s.order, s.N = prob["dim"], prob["order"], prob["N"]
    s.n_iface = len(prob["ifaces"])
    s.bie = BIE[prob.get("bie", "interface")]
    s.lo, s.hi = prob["lo"], prob["hi"]
    s.beta_in, s.beta_out, s.kappa = prob["beta_in"], prob["beta_out"], prob["kappa"]
    s.cos_alpha = prob.get("cos_alpha", 0.5)
    s.kappa_out = prob.get("kappa_out", prob["kappa"])
    for k, iface in enumerate(prob["ifaces"]):
        kind, params = iface[0], iface[1]
        s.iface[k].kind = KINDS[kind]
        for j, v in enumerate(params):
            s.iface[k].p[j] = float(v)
        if kind == "grid":
            if samples is None or samples[k] is None:
                raise ValueError("a sampled level set needs its samples on the device")
            s.samples[k] = samples[k].data_ptr()
    return s


def device_samples(prob, device):
    """Device copies of the node samples of the problem's sampled level sets
    (None for the analytic ones); they must live while a set-up reads them."""
    return [torch.as_tensor(i[2], dtype=torch.float64).reshape(-1).to(device).contiguous() if i[0] == "grid" else None
            for i in prob["ifaces"]]


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Geometry (step S0) and collocation factorisation (step S1) of one
    problem, plus the operators of the hot path."""

    def __init__(self, prob, device="cuda"):
        lib = load()
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.prob = prob
        self._samples = device_samples(prob, self.device)
        self._p = problem_struct(prob, self._samples)
        h = ctypes.c_void_p()
        st = lib.kfbi_plan_create(ctypes.byref(self._p), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(h))
        self._h = h
        if st != 0:
            msg = lib.kfbi_last_error().decode()
            self.close()
            raise KfbiError(st, msg)
        self._sizes()

    @classmethod
    def view(cls, handle, prob, device="cuda"):
        """A plan owned by someone else (a batch's): sizes, exports and
        solves, not destroyed on close."""
        self = cls.__new__(cls)
        self.device = torch.device(device)
        st = ctypes.c_void_p()
        _check(load().kfbi_plan_stream(ctypes.c_void_p(handle), ctypes.byref(st)))
        self.stream = torch.cuda.ExternalStream(st.value, device=self.device) if st.value else \
            torch.cuda.default_stream(self.device)
        self.prob = prob
        self._samples = device_samples(prob, self.device)
        self._p = problem_struct(prob, self._samples)
        self._h = ctypes.c_void_p(handle)
        self._owned = False
        self._sizes()
        return self

    def _sizes(self):
        s = Sizes()
        _check(load().kfbi_plan_sizes(self._h, ctypes.byref(s)))
        self.sizes = s
        self.n_nodes, self.n_surf, self.n_dof = s.n_nodes, s.n_surf, s.n_dof
        # unknowns of the BIE: [phi; psi] for the two-density form
        self.n_unknowns = s.n_dof * (2 if self.prob.get("bie") == "two_density" else 1)

    def setup(self, prob):
        """Re-run S0 + S1 for another problem on the same grid."""
        self.prob = prob
        self._samples = device_samples(prob, self.device)
        self._p = problem_struct(prob, self._samples)
        _check(load().kfbi_plan_setup(self._h, ctypes.byref(self._p)))
        self._sizes()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and getattr(self, "_owned", True):
            load().kfbi_plan_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ box solver
    BOX_SOLVERS = {"fft": 0, "mg64": 1, "mg32": 2}

    def set_box_solver(self, solver="fft", eps_in=1e-12, max_cycles=40):
        """Box solver of every later solve: "fft" (exact), "mg64" or "mg32"
        (multigrid V-cycles in FP64 / FP32 inside FP64 defect correction to
        |F - A v| <= eps_in |F|)."""
        _check(load().kfbi_plan_set_box_solver(self._h, self.BOX_SOLVERS[solver], float(eps_in), int(max_cycles)))
        self.box_solver = solver

    def set_box_relaxation(self, relax):
        """Relax the multigrid tolerance inside GMRES (inexact Krylov):
        eps_j = min(1e-1, max(eps_in, relax tol |b| / |r_j|)); 0 turns it off."""
        _check(load().kfbi_plan_set_box_relaxation(self._h, float(relax)))
        self.box_relax = float(relax)

    def box_stats(self):
        """(corrections, relative residual) of the last multigrid box solve."""
        c, r = ctypes.c_int32(), ctypes.c_double()
        _check(load().kfbi_plan_box_stats(self._h, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    # ------------------------------------------------------------------ tracing
    def profile(self, enable=True):
        """Start (or stop) HIP-event timing of the box-solve kernels: True or
        1 the FFT box solves, 2 the finest-level multigrid smoothing sweeps,
        3 the passes of the multigrid's exact coarse solve."""
        _check(load().kfbi_plan_profile(self._h, int(enable)))

    def timing(self):
        """(box solves, kernel launches, total ms) recorded since profile()."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(load().kfbi_plan_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    # ------------------------------------------------------------------ tables
    def export(self, name):
        s = self.sizes
        d = self.prob["dim"]
        p = 4 if self.prob["order"] == 4 else 2
        shapes = {
            "region": ((s.n_nodes,), torch.int8), "surf_pos": ((s.n_surf, d), torch.float64),
            "surf_nrm": ((s.n_surf, d), torch.float64), "surf_meta": ((s.n_surf, 5), torch.int32),
            "dof_surf": ((s.n_dof,), torch.int32), "stencil_d": ((s.n_dof, s.n_dir), torch.int32),
            "stencil_n": ((s.n_dof, s.n_neu), torch.int32), "ext_idx": ((s.n_surf, p), torch.int32),
            "ext_w": ((s.n_surf, p), torch.float64), "pde_pts": ((s.n_dof, s.n_pde, d), torch.float64),
            "irregular": ((s.n_irregular,), torch.int32), "corr": ((s.n_corr, 3), torch.int32),
            "cond": ((s.n_dof,), torch.float64), "dof_pos": ((s.n_dof, d), torch.float64),
        }
        shape, dt = shapes[name]
        out = torch.empty(shape, dtype=dt, device=self.device)
        nbytes = out.numel() * out.element_size()
        _check(load().kfbi_plan_export(self._h, EXPORT[name], ctypes.c_void_p(out.data_ptr() if nbytes else 0),
                                       nbytes))
        # the copy is ordered on the plan's stream: order torch's after it
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def _zeros(self, n):
        return torch.zeros(n, dtype=torch.float64, device=self.device)

    def _empty(self, n):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------------ operators
    def box_solve(self, F):
        v = self._zeros(self.n_nodes)
        _check(load().kfbi_box_solve(self._h, _ptr(F), _ptr(v)))
        return v

    def simple_solve(self, a=None, b=None, ftilde=None, fhat=None, gB=None):
        v = self._zeros(self.n_nodes)
        dn_in = self._zeros(self.n_dof)
        dn_out = self._zeros(self.n_dof)
        _check(load().kfbi_simple_solve(self._h, _ptr(a), _ptr(b), _ptr(ftilde), _ptr(fhat), _ptr(gB),
                                        _ptr(v), _ptr(dn_in), _ptr(dn_out)))
        return v, dn_in, dn_out

    def matvec(self, psi, out=None):
        out = self._zeros(self.n_unknowns) if out is None else out
        _check(load().kfbi_matvec(self._h, _ptr(psi), _ptr(out)))
        return out

    @staticmethod
    def data_struct(data):
        return Data(_ptr(data["g1"]), _ptr(data["g2"]), _ptr(data["ftilde"]), _ptr(data["fhat"]),
                    _ptr(data["gB"]))

    def rhs(self, data):
        b = self._zeros(self.n_unknowns)
        ds = self.data_struct(data)
        _check(load().kfbi_rhs(self._h, ctypes.byref(ds), _ptr(b)))
        return b

    def solve(self, data, tol=1e-10, max_iter=200, psi0=None, u_out=None, raise_on_fail=True, learned=None,
              solver=None, eps_in=0.0, max_cycles=0, relax=0.0):
        """Full KFBI solve; returns (psi, u, info dict).  psi0: initial
        density; learned: a Learned struct (the start predicted inside the
        solve); solver ("fft", "mg64", "mg32"; None keeps the plan's) with
        eps_in, max_cycles and relax set on the plan first."""
        # every entry of psi (from a zero start) and of u is written by the solve
        psi = self._empty(self.n_unknowns) if psi0 is None else psi0.clone()
        u = self._empty(self.n_nodes) if u_out is None else u_out
        ds = self.data_struct(data)
        start = "learned" if learned is not None else ("zero" if psi0 is None else "given")
        o = make_opts(tol, max_iter, start, solver, eps_in, max_cycles, relax, learned)
        info = Info()
        st = load().kfbi_solve(self._h, ctypes.byref(ds), ctypes.byref(o), _ptr(psi), _ptr(u), ctypes.byref(info))
        if st != 0 and raise_on_fail:
            _check(st)
        return psi, u, {"iters": info.iters, "status": info.status, "est_rel_res": info.est_rel_res,
                        "true_rel_res": info.true_rel_res}


def tile_lines(dim, N):
    """Lines per tile of the sine-transform passes on a (dim, N) grid (the
    override, the autotuner's choice or the built-in rule)."""
    return int(load().kfbi_tile_lines(int(dim), int(N)))


def set_tile_lines(dim, N, TL):
    """Override the tile lines of a grid (0 removes the override)."""
    _check(load().kfbi_set_tile_lines(int(dim), int(N), int(TL)))


def box_solve_noalloc(dim, order, N, lo, hi, kappa, F, v):
    """FFT box solve v = A_h^-1 F (zero box data) of a grid given by its
    parameters, with no plan and no allocation in the library (static
    device scratch); F, v caller-owned float64 device tensors of
    (N+1)^dim entries, ordered on the current torch stream."""
    st = torch.cuda.current_stream(F.device).cuda_stream
    _check(load().kfbi_box_solve_noalloc(int(dim), int(order), int(N), float(lo), float(hi), float(kappa),
                                         _ptr(F), _ptr(v), ctypes.c_void_p(st)))
    return v


def device_data(plan, prob, sol):
    """Manufactured data of `sol` at the plan's own query points, as device
    tensors (input generation; uses the workloads module)."""
    from . import workloads as W
    pos = plan.export("surf_pos").cpu().numpy()
    nrm = plan.export("surf_nrm").cpu().numpy()
    meta = plan.export("surf_meta").cpu().numpy()
    pde = plan.export("pde_pts").cpu().numpy()
    dsurf = plan.export("dof_surf").cpu().numpy()
    data = W.make_data(prob, sol, pos, nrm, meta[:, 3], pde, meta[dsurf, 3])
    dev = plan.device
    return {k: torch.from_numpy(v.reshape(-1).copy() if k != "ftilde" else v.copy()).to(dev).contiguous()
            for k, v in data.items()}


def device_bvp_data(plan, prob, u):
    """Manufactured data of an interior Dirichlet or Neumann problem with the
    solution u at the plan's own query points, as device tensors (input
    generation; uses the workloads module)."""
    from . import workloads as W
    pos = plan.export("surf_pos").cpu().numpy()
    nrm = plan.export("surf_nrm").cpu().numpy()
    pde = plan.export("pde_pts").cpu().numpy()
    data = W.make_bvp_data(prob, u, pos, nrm, pde)
    dev = plan.device
    return {k: None if v is None else
            torch.from_numpy(v.reshape(-1).copy() if k != "ftilde" else v.copy()).to(dev).contiguous()
            for k, v in data.items()}


def device_td_data(plan, prob, sol):
    """Manufactured data of a two-density problem with the solutions `sol`
    per region at the plan's own query points, as device tensors (input
    generation; uses the workloads module)."""
    from . import workloads as W
    pos = plan.export("surf_pos").cpu().numpy()
    nrm = plan.export("surf_nrm").cpu().numpy()
    meta = plan.export("surf_meta").cpu().numpy()
    pde = plan.export("pde_pts").cpu().numpy()
    dsurf = plan.export("dof_surf").cpu().numpy()
    data = W.make_td_data(prob, sol, pos, nrm, meta[:, 3], pde, meta[dsurf, 3])
    dev = plan.device
    return {k: torch.from_numpy(v.reshape(-1).copy()).to(dev).contiguous()
            for k, v in data.items()}


def device_jump_data(plan, jumps):
    """Config-5 data (jumps only; fhat, ftilde and gB zero) at the plan's
    surface points, as device tensors (input generation)."""
    from . import workloads as W
    pos = plan.export("surf_pos").cpu().numpy()
    g1, g2 = W.jump_values(jumps, pos)
    dev = plan.device
    return {"g1": torch.from_numpy(g1).to(dev).contiguous(), "g2": torch.from_numpy(g2).to(dev).contiguous(),
            "ftilde": None, "fhat": None, "gB": None}


class Batch:
    """Many independent problems solved by a pool of workers (threads with
    their own streams).  Set up, then solve: setup() builds a plan per
    problem, plan(i) gives it (for its query points), solve(data, psi)
    takes every problem's data.  Streaming: solve_stream(fn, ctx) takes
    each problem's data from a C callback (kfbi_batch_data_fn) once a
    worker's plan is set up for it."""

    def __init__(self, probs, workers=4):
        lib = load()
        self.probs = list(probs)
        self.n = len(probs)
        self._samples = [device_samples(p, torch.device("cuda")) for p in probs]
        arr = (Problem * self.n)(*[problem_struct(p, sm) for p, sm in zip(probs, self._samples)])
        self._arr = arr
        h = ctypes.c_void_p()
        _check(lib.kfbi_batch_create(ctypes.cast(arr, ctypes.c_void_p), self.n, int(workers), ctypes.byref(h)))
        self._h = h
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.kfbi_batch_sizes(self._h, ctypes.byref(a), ctypes.byref(b)))
        self.total_nodes = b.value

    def setup(self):
        """S0 + S1 of every problem; returns the statuses and seconds."""
        infos = (Info * self.n)()
        secs = (ctypes.c_double * self.n)()
        load().kfbi_batch_setup(self._h, ctypes.cast(infos, ctypes.c_void_p), ctypes.cast(secs, ctypes.c_void_p))
        return [x.status for x in infos], list(secs)

    def plan(self, i):
        """Problem i's plan (a view owned by the batch), or None if its
        set-up failed."""
        h = ctypes.c_void_p()
        st = load().kfbi_batch_plan(self._h, int(i), ctypes.byref(h))
        return Plan.view(h.value, self.probs[i]) if st == 0 and h.value else None

    def _opts(self, tol, max_iter, solver):
        return make_opts(tol, max_iter, "zero", solver.get("solver"), solver.get("eps_in", 0.0),
                         solver.get("max_cycles", 0), solver.get("relax", 0.0))

    def _run(self, call, keep_u, raise_on_fail):
        lib = load()
        u = torch.zeros(self.total_nodes, dtype=torch.float64, device="cuda") if keep_u else None
        infos = (Info * self.n)()
        secs = (ctypes.c_double * self.n)()
        torch.cuda.synchronize()
        st = call(_ptr(u), ctypes.cast(infos, ctypes.c_void_p), ctypes.cast(secs, ctypes.c_void_p))
        if st != 0 and raise_on_fail:
            raise KfbiError(st, lib.kfbi_last_error().decode())
        info = [{"iters": x.iters, "status": x.status, "true_rel_res": x.true_rel_res} for x in infos]
        return u, info, list(secs)

    def solve(self, data, psi=None, tol=1e-8, max_iter=300, keep_u=False, raise_on_fail=True, **solver):
        """data: per problem a dict of device tensors as Plan.solve takes
        (None for a problem that did not set up); psi: per problem a device
        tensor for the density, or None."""
        ds = (Data * self.n)(*[Plan.data_struct(d) if d is not None else Data() for d in data])
        pp = (ctypes.c_void_p * self.n)(*[(p.data_ptr() if p is not None else None) for p in (psi or [None] * self.n)])
        o = self._opts(tol, max_iter, solver)
        return self._run(lambda u, i, s: load().kfbi_batch_solve(self._h, ctypes.byref(o), ctypes.cast(ds, ctypes.c_void_p),
                                                                 ctypes.cast(pp, ctypes.c_void_p), u, i, s),
                         keep_u, raise_on_fail)

    def solve_stream(self, data_fn, ctx, tol=1e-8, max_iter=300, keep_u=False, raise_on_fail=True, **solver):
        """data_fn: address of a kfbi_batch_data_fn (C function) and ctx its
        argument; solver: solver / eps_in / max_cycles / relax as in
        Plan.solve."""
        o = self._opts(tol, max_iter, solver)
        return self._run(lambda u, i, s: load().kfbi_batch_solve_stream(self._h, ctypes.byref(o), ctypes.c_void_p(data_fn),
                                                                        ctypes.c_void_p(ctx), u, i, s),
                         keep_u, raise_on_fail)

    def close(self):
        if getattr(self, "_h", None):
            load().kfbi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

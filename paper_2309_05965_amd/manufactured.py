"""ctypes binding of libkfbi_gen.so: manufactured-solution test data through
the solver's public C ABI (an input generator for tests and benchmarks; the
solver does not use it)."""
import ctypes
import os

import torch

from . import kfbi

_HERE = os.path.dirname(os.path.abspath(__file__))
GEN_PATH = os.path.join(_HERE, "libkfbi_gen.so")
KIND = {"star2d": 1, "torus3d": 2}
_gen = None


def load():
    global _gen
    if _gen is None:
        kfbi.load()
        if not os.path.exists(GEN_PATH):
            raise RuntimeError("libkfbi_gen.so is not built (python -m paper_2309_05965_amd.build)")
        g = ctypes.CDLL(GEN_PATH)
        g.kfbi_gen_plan_data.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p] + \
            [ctypes.c_void_p] * 5
        g.kfbi_gen_plan_data.restype = ctypes.c_int
        g.kfbi_gen_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]
        g.kfbi_gen_create.restype = ctypes.c_int
        g.kfbi_gen_destroy.argtypes = [ctypes.c_void_p]
        g.kfbi_gen_destroy.restype = ctypes.c_int
        g.kfbi_gen_release.argtypes = []
        g.kfbi_gen_release.restype = None
        _gen = g
    return _gen


def plan_data(plan, kind):
    """Manufactured-solution data at the plan's query points, generated on
    the device on the plan's stream (kind "star2d" or "torus3d")."""
    s = plan.sizes
    K = len(plan.prob["ifaces"])
    z = lambda n: torch.empty(n, dtype=torch.float64, device=plan.device)
    d = {"g1": z(s.n_surf), "g2": z(s.n_surf), "ftilde": z(s.n_dof * s.n_pde), "fhat": z((K + 1) * s.n_nodes),
         "gB": z(s.n_nodes)}
    st = load().kfbi_gen_plan_data(plan._h, ctypes.byref(plan._p), KIND[kind],
                                   ctypes.c_void_p(plan.stream.cuda_stream),
                                   *[kfbi._ptr(d[k]) for k in ("g1", "g2", "ftilde", "fhat", "gB")])
    kfbi._check(st)
    torch.cuda.current_stream(plan.device).wait_stream(plan.stream)
    return d


class BatchData:
    """The generator's kfbi_batch_data_fn and its context for a batch of
    problems with their kinds; with psi_stride the densities are kept in
    self.psi[i * psi_stride : i * psi_stride + n_dof_i]."""

    def __init__(self, probs, kinds, psi_stride=0):
        g = load()
        n = len(probs)
        self._samples = [kfbi.device_samples(p, "cuda") for p in probs]
        self._arr = (kfbi.Problem * n)(*[kfbi.problem_struct(p, sm) for p, sm in zip(probs, self._samples)])
        km = (ctypes.c_int * n)(*[KIND[k] for k in kinds])
        self.psi = torch.zeros(n * psi_stride, dtype=torch.float64, device="cuda") if psi_stride else None
        h = ctypes.c_void_p()
        kfbi._check(g.kfbi_gen_create(ctypes.cast(self._arr, ctypes.c_void_p), ctypes.cast(km, ctypes.c_void_p), n,
                                      kfbi._ptr(self.psi), int(psi_stride), ctypes.byref(h)))
        self.ctx = h.value
        self.fn = ctypes.cast(g.kfbi_gen_batch_data, ctypes.c_void_p).value

    def close(self):
        if getattr(self, "ctx", None):
            load().kfbi_gen_destroy(ctypes.c_void_p(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Binding of the learned initial density (C ABI of include/kfbi.h): the
bf16-MFMA MLP, the sample features and the spherical-harmonic transfer.
Argument marshalling only; every computation runs in libkfbi.so."""
import ctypes

import numpy as np
import torch

from . import kfbi
from . import workloads as W

WIDTHS = (9216, 256, 256, 256, 1024)


def _p(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(st):
    if st != 0:
        raise kfbi.KfbiError(st, kfbi.load().kfbi_last_error().decode())


class MLP:
    """MLP with bf16 weights (fp32 masters), trained by Adam."""

    def __init__(self, widths=WIDTHS, device="cuda"):
        lib = kfbi.load()
        self.widths = tuple(int(w) for w in widths)
        self.device = torch.device(device)
        arr = (ctypes.c_int * len(self.widths))(*self.widths)
        h = ctypes.c_void_p()
        _check(lib.kfbi_mlp_create(len(self.widths) - 1, arr, _stream(self.device), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(lib.kfbi_mlp_sizes(self._h, ctypes.byref(n)))
        self.n_params = n.value
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            kfbi.load().kfbi_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self):
        """[(W offset, W shape, b offset, b size)] of the parameter pack."""
        out, o = [], 0
        for a, b in zip(self.widths[:-1], self.widths[1:]):
            out.append((o, (a, b), o + a * b, b))
            o += a * b + b
        return out

    def init_params(self, seed=0):
        """He-uniform weights, zero biases (seeded input)."""
        rng = np.random.default_rng(seed)
        p = np.zeros(self.n_params, dtype=np.float32)
        for ow, (a, b), ob, nb in self.layout():
            lim = np.sqrt(6.0 / a)
            p[ow:ow + a * b] = rng.uniform(-lim, lim, a * b).astype(np.float32)
        self.set_params(torch.from_numpy(p).to(self.device))

    def set_params(self, params):
        _check(kfbi.load().kfbi_mlp_set_params(self._h, _p(params.float().contiguous())))

    def get_params(self):
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(kfbi.load().kfbi_mlp_get_params(self._h, _p(out)))
        return out

    def forward(self, X):
        B = X.shape[0]
        Y = torch.empty((B, self.widths[-1]), dtype=torch.float32, device=self.device)
        _check(kfbi.load().kfbi_mlp_forward(self._h, _p(X), B, _p(Y)))
        return Y

    def loss_grad(self, X, Yt):
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(kfbi.load().kfbi_mlp_loss_grad(self._h, _p(X), _p(Yt), X.shape[0], _p(self.loss_buf), _p(g)))
        return self.loss_buf.clone(), g

    def train_step(self, X, Yt, lr):
        _check(kfbi.load().kfbi_mlp_train_step(self._h, _p(X), _p(Yt), X.shape[0], ctypes.c_float(lr),
                                               _p(self.loss_buf)))
        return self.loss_buf

    # linear head: X holds B examples of R rows; the output of an example
    # (its R rows) holds nb basis vectors, contracted with C [B x nb]
    def forward_lin(self, X, C, nb, R=1):
        B = X.shape[0] // R
        Y = torch.empty((B, R * self.widths[-1] // nb), dtype=torch.float32, device=self.device)
        _check(kfbi.load().kfbi_mlp_forward_lin(self._h, _p(X), B, int(R), _p(C), int(nb), _p(Y)))
        return Y

    def loss_grad_lin(self, X, C, nb, Yt, R=1):
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(kfbi.load().kfbi_mlp_loss_grad_lin(self._h, _p(X), X.shape[0] // R, int(R), _p(C), int(nb), _p(Yt),
                                                  _p(self.loss_buf), _p(g)))
        return self.loss_buf.clone(), g

    def train_step_lin(self, X, C, nb, Yt, lr, R=1):
        _check(kfbi.load().kfbi_mlp_train_step_lin(self._h, _p(X), X.shape[0] // R, int(R), _p(C), int(nb), _p(Yt),
                                                   ctypes.c_float(lr), _p(self.loss_buf)))
        return self.loss_buf


def gemm_bf16(A, B, transA=False, transB=False):
    """fp32 C = op(A) op(B); A, B int16/uint16 tensors holding bf16 bits."""
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(kfbi.load().kfbi_gemm_bf16(int(transA), int(transB), M, N, K, _p(A), A.shape[1], _p(B), B.shape[1],
                                      _p(C), N, _stream(A.device)))
    return C


def pack_geometry(geom):
    c, a, Q = geom
    return np.concatenate([np.asarray(c, float), np.asarray(a, float), np.asarray(Q, float).ravel()])


def pack_jumps(jumps):
    a, b = jumps
    return np.concatenate([np.asarray(a, float).ravel(), np.asarray(b, float).ravel()])


def samples(device="cuda", n=W.N_SAMPLES):
    return torch.from_numpy(W.fibonacci_sphere(n)).to(device).contiguous()


def features(geoms, jumps, S):
    """X [P, ns*9] fp32 from packed geometries [P, 15] and jumps [P, 32]."""
    P, ns = geoms.shape[0], S.shape[0]
    X = torch.empty((P, ns * 9), dtype=torch.float32, device=S.device)
    _check(kfbi.load().kfbi_ellipsoid_features(_p(geoms), _p(jumps), P, _p(S), ns, _stream(S.device), _p(X)))
    return X


def transfer(plan, geom, S, psi_s, scale=1.0):
    """Density at the plan's DOFs from sample values (fp32 [ns])."""
    out = torch.empty(plan.n_dof, dtype=torch.float64, device=S.device)
    _check(kfbi.load().kfbi_sh_transfer(plan._h, _p(geom), _p(S), S.shape[0], _p(psi_s), float(scale), _p(out)))
    return out


def sample(plan, geom, psi_dof, S, scale=1.0):
    """Density at the samples (fp32, times scale) from DOF values."""
    out = torch.empty(S.shape[0], dtype=torch.float32, device=S.device)
    _check(kfbi.load().kfbi_sh_sample(plan._h, _p(geom), _p(psi_dof), _p(S), S.shape[0], float(scale), _p(out)))
    return out


def real_sh(dirs):
    Y = torch.empty((81, dirs.shape[0]), dtype=torch.float64, device=dirs.device)
    _check(kfbi.load().kfbi_real_sh(_p(dirs), dirs.shape[0], _stream(dirs.device), _p(Y)))
    return Y


def scale_jumps(X, Y, alpha, ns=W.N_SAMPLES):
    """In place: jump features and targets of example r times alpha[r]."""
    _check(kfbi.load().kfbi_scale_jumps(_p(X), _p(Y), _p(alpha), X.shape[0], ns, Y.shape[1], _stream(X.device)))


def geometry_input(geoms):
    """Network input [P * 8, 15] fp32 (a row per Fourier mode) of packed
    geometries [P, 15]."""
    X = torch.empty((geoms.shape[0] * 8, 15), dtype=torch.float32, device=geoms.device)
    _check(kfbi.load().kfbi_geometry_input(_p(geoms), geoms.shape[0], _stream(geoms.device), _p(X)))
    return X


def sh_coefficients(plan, geom, psi_dof, scale=1.0):
    """81 SH coefficients (FP64) of scale * psi at the plan's DOFs."""
    out = torch.empty(81, dtype=torch.float64, device=psi_dof.device)
    _check(kfbi.load().kfbi_sh_coefficients(plan._h, _p(geom), _p(psi_dof), float(scale), _p(out)))
    return out


def learned_start(plan, mlp, nb, geom, jumps, scale):
    """Initial density at the plan's DOFs from the linear-head network."""
    out = torch.empty(plan.n_dof, dtype=torch.float64, device=geom.device)
    _check(kfbi.load().kfbi_learned_start(plan._h, mlp._h, int(nb), _p(geom), _p(jumps), float(scale), _p(out)))
    return out


def sh_expand(plan, geom, coef, scale=1.0):
    """The 81-harmonic expansion with coefficients coef at the plan's DOFs."""
    out = torch.empty(plan.n_dof, dtype=torch.float64, device=coef.device)
    _check(kfbi.load().kfbi_sh_expand(plan._h, _p(geom), _p(coef), float(scale), _p(out)))
    return out

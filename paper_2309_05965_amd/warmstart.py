"""Learned GMRES start for the ellipsoid workload: data generation from the
solver's own densities, training, and prediction of the initial density.

With zero source and box data the density is linear in the 32 jump
coefficients (a_1[8], a_2[8], b_1[8], b_2[8] of g_j = sum_m a_jm cos(k_m.x)
+ b_jm sin(k_m.x)), so the network maps the geometry alone to 32 basis
densities, each as its 81 real spherical-harmonic coefficients in the
body-frame direction, and a linear head contracts them with the problem's
jump coefficients.  One network is shared by the eight Fourier modes: its
row for mode m sees the semi-axes, the mode's wave vector in the scaled body
frame diag(a) Q^T k_m and the orientation, and gives the four basis
densities of a_1m, a_2m, b_1m, b_2m:

    data = generate(range(0, 20000), N=128)       # solves, geometry, jumps, SH targets
    model, hist = train(data, epochs=60)          # bf16-MFMA MLP with the linear head, Adam
    psi0 = predict(model, plan, geom, jumps)      # initial density at the DOFs
    plan.solve(jump_data, psi0=psi0)
    plan.solve(jump_data, learned=learned_args(model, geom, jumps))   # the same, predicted inside the solve

Every numerical step runs in libkfbi.so (solver, SH fit, MLP, head,
evaluation at the DOFs); this module sequences the calls and holds the
arrays.
"""
import json
import os
import time

import numpy as np
import torch

from . import kfbi, learned
from . import workloads as W

NB = 32                                   # jump coefficients = basis densities
NSH = 81                                  # SH coefficients of degree <= 8
R = 8                                     # network rows per problem: one per Fourier mode
WIDTHS = (15, 256, 256, 256, 4 * NSH)     # 4 layers of width 256; 4 basis densities per mode


class Model:
    def __init__(self, mlp, out_scale):
        self.mlp = mlp
        self.out_scale = float(out_scale)


def _pack(geom, jumps, device):
    """Geometry and jump coefficients on the device: one pinned host buffer
    and one copy enqueued on the current stream (the host does not wait;
    the stream orders the copy before the kernels that read it)."""
    h = torch.from_numpy(np.concatenate([learned.pack_geometry(geom), learned.pack_jumps(jumps)])).pin_memory()
    d = h.to(device, non_blocking=True)
    ng = 15
    return d[:ng], d[ng:]


def generate(seeds, N=128, tol=1e-10, device="cuda", log_every=0):
    """Solve every seed's problem (FFT box solve, GMRES to tol) and return
    packed geometries G [n, 15] and jumps J [n, 32] (FP64), the SH
    coefficients Y [n, 81] (FP64) of the solved density and the zero-start
    GMRES iterations.  Seeds whose geometry the set-up does not resolve on
    the grid are skipped."""
    plan = None
    Gs, Js, Ys, iters, used = [], [], [], [], []
    t0 = time.time()
    for i, seed in enumerate(seeds):
        prob, geom, jmp = W.config5(seed, N)
        try:
            if plan is None:
                plan = kfbi.Plan(prob, device)
            else:
                plan.setup(prob)
            data = kfbi.device_jump_data(plan, jmp)
            psi, _, info = plan.solve(data, tol=tol, max_iter=300)
        except kfbi.KfbiError:
            plan = None
            continue
        g, j = _pack(geom, jmp, device)
        Ys.append(learned.sh_coefficients(plan, g, psi, 1.0))
        Gs.append(g)
        Js.append(j)
        used.append(seed)
        iters.append(info["iters"])
        if log_every and (i + 1) % log_every == 0:
            print("generated %d/%d (%.1f s)" % (i + 1, len(seeds), time.time() - t0), flush=True)
    return {"G": torch.stack(Gs), "J": torch.stack(Js), "Y": torch.stack(Ys), "iters": np.array(iters),
            "seeds": np.array(used)}


def train(data, epochs=60, batch=256, lr=1e-3, seed=0, log=None):
    """Adam on the mean squared error of the scaled SH targets through the
    linear head, the learning rate decaying on a cosine to 5% of lr.  The
    losses are summed on the device and read once per epoch.  Returns the
    model and the per-epoch mean losses."""
    X = learned.geometry_input(data["G"]).view(-1, R, WIDTHS[0])
    # jump coefficients in the order of the basis vectors: (mode, a_1 a_2 b_1 b_2)
    C = data["J"].view(-1, 4, R).transpose(1, 2).reshape(-1, NB).float().contiguous()
    Y = data["Y"]
    scale = float(Y.abs().mean().item()) or 1.0
    Ys = (Y / scale).float().contiguous()
    mlp = learned.MLP(WIDTHS, X.device)
    mlp.init_params(seed)
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    nb = max(1, n // batch)
    steps = epochs * nb
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot = torch.zeros(1, dtype=torch.float32, device=X.device)
        for b0 in range(0, nb * batch, batch):
            idx = perm[b0:b0 + batch]
            lr_k = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * k / max(1, steps))))
            tot += mlp.train_step_lin(X[idx].reshape(-1, WIDTHS[0]).contiguous(), C[idx].contiguous(), NB,
                                      Ys[idx].contiguous(), lr_k, R)
            k += 1
        hist.append(float(tot.item()) / nb)
        if log:
            log(ep, hist[-1])
    return Model(mlp, scale), hist


def predict(model, plan, geom, jumps):
    """Initial density at the plan's DOFs for one ellipsoid problem (one
    library call on the plan's stream)."""
    g, j = _pack(geom, jumps, model.mlp.device)
    return learned.learned_start(plan, model.mlp, NB, g, j, model.out_scale)


def learned_args(model, geom, jumps):
    """The kfbi_learned of one ellipsoid problem, for a solve that predicts
    its own start (Plan.solve(..., learned=...))."""
    g, j = _pack(geom, jumps, model.mlp.device)
    L = kfbi.Learned(model.mlp._h, NB, g.data_ptr(), j.data_ptr(), model.out_scale)
    L._keep = (g, j)
    return L


PRETRAINED = "data/warmstart_ellipsoid128.safetensors"


def save(model, path):
    from safetensors.torch import save_file
    meta = {"widths": json.dumps(list(model.mlp.widths)), "out_scale": repr(model.out_scale), "head": str(NB),
            "rows": str(R), "kind": "per-mode network, linear head over the jump coefficients, SH degree 8"}
    save_file({"params": model.mlp.get_params().cpu()}, path, metadata=meta)


def load_pretrained(device="cuda", path=None):
    """The model trained by train_warmstart on method-generated densities of
    N = 128 ellipsoid problems (fp32 parameter pack; the GEMMs use bf16
    copies)."""
    from safetensors import safe_open
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), PRETRAINED)
    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        params = f.get_tensor("params").float()
    widths = tuple(json.loads(meta["widths"]))
    if widths != WIDTHS or int(meta["head"]) != NB:
        raise ValueError("stored model has widths %s and head %s" % (widths, meta["head"]))
    mlp = learned.MLP(widths, device)
    mlp.set_params(params.to(device))
    return Model(mlp, float(meta["out_scale"]))

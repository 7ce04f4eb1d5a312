"""Learned GMRES start for the ellipsoid workload: data generation from the
solver's own densities, training, and prediction of the initial density.

    data = generate(range(0, 2000), N=128)        # solves, features, targets
    model = train(data, epochs=30)                # bf16-MFMA MLP, Adam
    psi0 = predict(model, plan, geom, jumps)      # initial density at the DOFs
    plan.solve(jump_data, psi0=psi0)

Every numerical step runs in libkfbi.so (solver, features, MLP, transfers);
this module sequences the calls and holds the arrays.
"""
import time

import numpy as np
import torch

from . import kfbi, learned
from . import workloads as W


class Model:
    def __init__(self, mlp, out_scale):
        self.mlp = mlp
        self.out_scale = float(out_scale)

    def state(self):
        return {"widths": list(self.mlp.widths), "out_scale": self.out_scale,
                "params": self.mlp.get_params().cpu()}

    @classmethod
    def from_state(cls, st, device="cuda"):
        m = learned.MLP(tuple(st["widths"]), device)
        m.set_params(st["params"].to(device))
        return cls(m, st["out_scale"])


def _pack(geom, jumps, device):
    return (torch.tensor(learned.pack_geometry(geom), device=device),
            torch.tensor(learned.pack_jumps(jumps), device=device))


def generate(seeds, N=128, tol=1e-10, device="cuda", log_every=0):
    """Solve every seed's problem and return features X [n, 9216] (fp32),
    density targets at the samples Y [n, 1024] (fp64 -> fp32 unscaled) and
    the GMRES iterations of the zero start."""
    S = learned.samples(device)
    plan = None
    geoms, jumps, Ys, iters, used = [], [], [], [], []
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
            plan = None                  # geometry not resolved on this grid: skipped
            continue
        used.append(seed)
        g, j = _pack(geom, jmp, device)
        Ys.append(learned.sample(plan, g, psi, S, 1.0))
        geoms.append(g)
        jumps.append(j)
        iters.append(info["iters"])
        if log_every and (i + 1) % log_every == 0:
            print("generated %d/%d (%.1f s)" % (i + 1, len(seeds), time.time() - t0), flush=True)
    G = torch.stack(geoms)
    J = torch.stack(jumps)
    X = learned.features(G, J, S)
    return {"X": X, "Y": torch.stack(Ys), "iters": np.array(iters), "geoms": G, "jumps": J,
            "seeds": np.array(used)}


def train(data, epochs=30, batch=256, lr=1e-3, seed=0, widths=learned.WIDTHS, augment=True, log=None):
    """Adam on the mean squared error of the scaled targets, the learning
    rate decaying on a cosine to 5% of lr.  With augment, every batch's
    jump features and targets are scaled by factors drawn from U(-2, 2)
    (the density is linear in the jump data).  Returns the model and the
    per-epoch mean losses."""
    X, Y = data["X"], data["Y"]
    scale = float(Y.abs().mean().item()) or 1.0
    Ys = (Y / scale).contiguous()
    mlp = learned.MLP(widths, X.device)
    mlp.init_params(seed)
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps = epochs * max(1, n // batch)
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb, yb = X[idx].contiguous(), Ys[idx].contiguous()
            if augment:
                alpha = (torch.rand(batch, generator=g) * 4.0 - 2.0).to(X.device, torch.float32)
                learned.scale_jumps(xb, yb, alpha)
            lr_k = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * k / max(1, steps))))
            loss = mlp.train_step(xb, yb, lr_k)
            tot += float(loss.item())
            cnt += 1
            k += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(ep, hist[-1])
    return Model(mlp, scale), hist


def predict(model, plan, geom, jumps, S=None):
    """Initial density at the plan's DOFs for one ellipsoid problem."""
    dev = model.mlp.device
    if S is None:
        S = learned.samples(dev)
    g, j = _pack(geom, jumps, dev)
    X = learned.features(g[None, :], j[None, :], S)
    y = model.mlp.forward(X)[0].contiguous()
    return learned.transfer(plan, g, S, y, model.out_scale)


def evaluate(model, seeds, N=128, tol=1e-8, device="cuda"):
    """GMRES iterations from the zero start, the control g2/(beta_in +
    beta_out) and the learned start, per held-out seed."""
    S = learned.samples(device)
    plan = None
    rows = []
    for seed in seeds:
        prob, geom, jmp = W.config5(seed, N)
        try:
            if plan is None:
                plan = kfbi.Plan(prob, device)
            else:
                plan.setup(prob)
        except kfbi.KfbiError:
            plan = None
            continue
        data = kfbi.device_jump_data(plan, jmp)
        _, _, i0 = plan.solve(data, tol=tol)
        dsurf = plan.export("dof_surf").long()
        ctrl = (data["g2"][dsurf] / (prob["beta_in"] + prob["beta_out"])).contiguous()
        _, _, ic = plan.solve(data, tol=tol, psi0=ctrl)
        psi0 = predict(model, plan, geom, jmp, S)
        _, _, il = plan.solve(data, tol=tol, psi0=psi0)
        rows.append((seed, i0["iters"], ic["iters"], il["iters"], i0["true_rel_res"], il["true_rel_res"]))
    return rows


PRETRAINED = "data/warmstart_ellipsoid128.safetensors"


def load_pretrained(device="cuda", path=None):
    """The model trained by train_warmstart on 20,000 solver-generated
    densities of N = 128 ellipsoid problems (parameters stored in bf16,
    which is the precision the GEMMs use)."""
    import json
    import os

    from safetensors import safe_open
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), PRETRAINED)
    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        params = f.get_tensor("params_bf16").float()
    st = {"widths": json.loads(meta["widths"]), "out_scale": float(meta["out_scale"]), "params": params}
    return Model.from_state(st, device)

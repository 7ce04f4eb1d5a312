"""Train the learned GMRES start on solver-generated densities of random
ellipsoids and report what it gains on held-out seeds.

    python -m paper_2309_05965_amd.train_warmstart --N 128 --train 12000 \
        --epochs 60 --heldout 64 --out gpurun_out/warmstart

Writes <out>/summary.json (timings, losses, held-out prediction errors and
GMRES iteration counts from the zero start, the control g2/(beta_in +
beta_out), the learned start and the exact density projected on the
spherical harmonics) and <out>/model.pt (fp32 parameter pack, widths and
output scale; loadable with torch.load(weights_only=True)).
"""
import argparse
import json
import os
import time

import numpy as np
import torch

from . import kfbi, learned, warmstart
from . import workloads as W

HELDOUT0 = 1_000_000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--train", type=int, default=12000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--heldout", type=int, default=64)
    ap.add_argument("--out", default="warmstart_out")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    torch.cuda.set_device(0)
    summ = {"N": a.N, "train_requested": a.train, "epochs": a.epochs, "lr": a.lr}

    t0 = time.time()
    data = warmstart.generate(range(a.train), N=a.N, log_every=500)
    torch.cuda.synchronize()
    summ["train_examples"] = int(data["X"].shape[0])
    summ["generate_s"] = time.time() - t0
    summ["train_zero_start_iters_mean"] = float(data["iters"].mean())
    print("data: %d examples in %.1f s" % (summ["train_examples"], summ["generate_s"]), flush=True)

    t0 = time.time()
    model, hist = warmstart.train(data, epochs=a.epochs, lr=a.lr,
                                  log=lambda e, l: print("epoch %d loss %.4f" % (e, l), flush=True))
    torch.cuda.synchronize()
    summ["train_s"] = time.time() - t0
    summ["loss_history"] = hist
    del data

    held = range(HELDOUT0, HELDOUT0 + a.heldout)
    val = warmstart.generate(held, N=a.N)
    y = model.mlp.forward(val["X"]) * model.out_scale
    rel = ((y - val["Y"]).norm(dim=1) / val["Y"].norm(dim=1)).cpu().numpy()
    summ["heldout_rel_err_samples_median"] = float(np.median(rel))
    summ["heldout_rel_err_samples_mean"] = float(rel.mean())
    print("held-out relative error at the samples: median %.3f" % np.median(rel), flush=True)

    # iterations: zero, control, learned, exact density projected on the SH
    S = learned.samples()
    rows = []
    plan = None
    t_pred = []
    for seed in held:
        prob, geom, jmp = W.config5(seed, a.N)
        try:
            if plan is None:
                plan = kfbi.Plan(prob)
            else:
                plan.setup(prob)
        except kfbi.KfbiError:
            plan = None
            continue
        d = kfbi.device_jump_data(plan, jmp)
        psi, _, iz = plan.solve(d, tol=1e-8)
        psi_ref, _, _ = plan.solve(d, tol=1e-11)
        dsurf = plan.export("dof_surf").long()
        ctrl = (d["g2"][dsurf] / (prob["beta_in"] + prob["beta_out"])).contiguous()
        _, _, ic = plan.solve(d, tol=1e-8, psi0=ctrl)
        torch.cuda.synchronize()
        t = time.time()
        p0 = warmstart.predict(model, plan, geom, jmp, S)
        torch.cuda.synchronize()
        t_pred.append(time.time() - t)
        _, _, il = plan.solve(d, tol=1e-8, psi0=p0)
        g = torch.tensor(learned.pack_geometry(geom)).cuda()
        pj = learned.transfer(plan, g, S, learned.sample(plan, g, psi_ref, S, 1.0), 1.0)
        _, _, ip = plan.solve(d, tol=1e-8, psi0=pj)
        err_l = float(((p0 - psi_ref).norm() / psi_ref.norm()).item())
        err_c = float(((ctrl - psi_ref).norm() / psi_ref.norm()).item())
        rows.append([seed, iz["iters"], ic["iters"], il["iters"], ip["iters"], err_c, err_l,
                     il["true_rel_res"]])
    r = np.array(rows, dtype=np.float64)
    summ["heldout_solved"] = len(rows)
    summ["iters_mean"] = {"zero": r[:, 1].mean(), "control": r[:, 2].mean(), "learned": r[:, 3].mean(),
                          "exact_projected": r[:, 4].mean()}
    summ["dof_rel_err_mean"] = {"control": r[:, 5].mean(), "learned": r[:, 6].mean()}
    summ["learned_true_rel_res_max"] = r[:, 7].max()
    summ["predict_ms_mean"] = 1e3 * float(np.mean(t_pred))
    summ["rows"] = rows
    print(json.dumps({k: v for k, v in summ.items() if k not in ("rows", "loss_history")}), flush=True)
    with open(os.path.join(a.out, "summary.json"), "w") as f:
        json.dump(summ, f, indent=1, default=float)
    torch.save(model.state(), os.path.join(a.out, "model.pt"))


if __name__ == "__main__":
    main()

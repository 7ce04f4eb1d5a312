"""Train the learned GMRES start on solver-generated densities of random
ellipsoids and report what it gains on held-out seeds.

    python -m paper_2309_05965_amd.train_warmstart --N 128 --train 20000 \
        --epochs 60 --heldout 64 --out gpurun_out/warmstart

Writes <out>/summary.json (timings, losses, held-out prediction errors,
GMRES iterations and solve times from the zero start and the learned start,
and the iterations from the exact density projected on the degree-8
harmonics, the best this representation allows) and <out>/model.safetensors
(the model in the format load_pretrained reads).
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
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--heldout", type=int, default=64)
    ap.add_argument("--out", default="warmstart_out")
    ap.add_argument("--data", default=None, help="load generated data (.pt written by --save-data)")
    ap.add_argument("--save-data", action="store_true", help="write the generated data to <out>/data.pt")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    torch.cuda.set_device(0)
    torch.cuda.set_stream(torch.cuda.Stream())
    summ = {"N": a.N, "train_requested": a.train, "epochs": a.epochs, "lr": a.lr}

    t0 = time.time()
    if a.data:
        data = torch.load(a.data, weights_only=True)
        data = {k: (v.cuda() if k in ("G", "J", "Y") else v.numpy()) for k, v in data.items()}
    else:
        data = warmstart.generate(range(a.train), N=a.N, log_every=1000)
        if a.save_data:
            torch.save({k: (v.cpu() if torch.is_tensor(v) else torch.from_numpy(v)) for k, v in data.items()},
                       os.path.join(a.out, "data.pt"))
    torch.cuda.synchronize()
    summ["train_examples"] = int(data["G"].shape[0])
    summ["generate_s"] = time.time() - t0
    summ["train_zero_start_iters_mean"] = float(data["iters"].mean())
    print("data: %d examples in %.1f s" % (summ["train_examples"], summ["generate_s"]), flush=True)

    t0 = time.time()
    model, hist = warmstart.train(data, epochs=a.epochs, lr=a.lr,
                                  log=lambda e, l: print("epoch %d loss %.5f" % (e, l), flush=True))
    torch.cuda.synchronize()
    summ["train_s"] = time.time() - t0
    summ["loss_history"] = hist
    del data
    warmstart.save(model, os.path.join(a.out, "model.safetensors"))

    # held-out: coefficient error, density error at the DOFs, iterations and
    # whole-solve times (FFT box solve) from the zero and the learned start,
    # iterations from the exact density projected on the harmonics
    rows = []
    plan = None
    for seed in range(HELDOUT0, HELDOUT0 + a.heldout):
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
        psi_ref, _, _ = plan.solve(d, tol=1e-11)
        g = torch.tensor(learned.pack_geometry(geom)).cuda()
        coef_ref = learned.sh_coefficients(plan, g, psi_ref, 1.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, iz = plan.solve(d, tol=1e-8)
        torch.cuda.synchronize()
        tz = time.perf_counter() - t
        t = time.perf_counter()
        p0 = warmstart.predict(model, plan, geom, jmp)
        _, _, il = plan.solve(d, tol=1e-8, psi0=p0)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t
        t = time.perf_counter()
        p1 = warmstart.predict(model, plan, geom, jmp)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        coef_l = learned.sh_coefficients(plan, g, p0, 1.0)
        _, _, ip = plan.solve(d, tol=1e-8, psi0=learned.sh_expand(plan, g, coef_ref))
        err_l = float(((p0 - psi_ref).norm() / psi_ref.norm()).item())
        err_c = float(((coef_l - coef_ref).norm() / coef_ref.norm()).item())
        rows.append([seed, iz["iters"], il["iters"], ip["iters"], err_c, err_l, il["true_rel_res"], tz, tl, tp])
    r = np.array(rows, dtype=np.float64)
    summ["heldout_solved"] = len(rows)
    summ["iters_mean"] = {"zero": r[:, 1].mean(), "learned": r[:, 2].mean(), "exact_projected": r[:, 3].mean()}
    summ["coef_rel_err"] = {"median": float(np.median(r[:, 4])), "mean": float(r[:, 4].mean())}
    summ["dof_rel_err"] = {"median": float(np.median(r[:, 5])), "mean": float(r[:, 5].mean())}
    summ["learned_true_rel_res_max"] = float(r[:, 6].max())
    summ["solve_ms_mean"] = {"zero": 1e3 * float(r[:, 7].mean()), "learned_incl_prediction": 1e3 * float(r[:, 8].mean())}
    summ["predict_ms_mean"] = 1e3 * float(r[:, 9].mean())
    summ["rows"] = rows
    print(json.dumps({k: v for k, v in summ.items() if k not in ("rows", "loss_history")}, default=float), flush=True)
    with open(os.path.join(a.out, "summary.json"), "w") as f:
        json.dump(summ, f, indent=1, default=float)


if __name__ == "__main__":
    main()

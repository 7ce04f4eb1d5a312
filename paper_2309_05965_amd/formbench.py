"""Time whole KFBI solves of one held-out problem of the ellipsoid workload
(128^3, beta 1/100, random Fourier jumps) in a chosen form.

    python -m paper_2309_05965_amd.formbench --solver mg32 --eps 1e-9 --relax 0.1 --learned --solves 3

The form is the box solver (fft, mg64 or mg32), its defect-correction
tolerance, the relaxation factor of that tolerance inside GMRES and the
start (zero, or the stored learned model).  The plan is made on a stream of
its own; two untimed solves come first (the multigrid cycle caps adapt after
a plan's first solve).  Prints one JSON line: set-up and solve times per
solve (host clock), GMRES iterations and true relative residual.
"""
import argparse
import json
import time

import torch

from . import kfbi
from . import workloads as W


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--solver", default="mg32", choices=["fft", "mg64", "mg32"])
    ap.add_argument("--eps", type=float, default=1e-9)
    ap.add_argument("--relax", type=float, default=3.0)
    ap.add_argument("--max-cycles", type=int, default=16)
    ap.add_argument("--learned", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--solves", type=int, default=3)
    a = ap.parse_args()
    torch.cuda.set_device(0)
    torch.cuda.set_stream(torch.cuda.Stream())
    for seed in range(1_000_200, 1_000_216):          # the first held-out seed that resolves
        prob, geom, jmp = W.config5(seed, 128)
        try:
            plan = kfbi.Plan(prob)
            break
        except kfbi.KfbiError:
            continue
    data = kfbi.device_jump_data(plan, jmp)
    plan.set_box_solver(a.solver, eps_in=a.eps, max_cycles=a.max_cycles)
    plan.set_box_relaxation(a.relax if a.solver != "fft" else 0.0)
    model = None
    if a.learned:
        from . import warmstart
        model = warmstart.load_pretrained()

    def solve():
        t0 = time.perf_counter()
        plan.setup(prob)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        la = warmstart.learned_args(model, geom, jmp) if a.learned else None
        _, _, info = plan.solve(data, tol=a.tol, learned=la)
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, info

    for _ in range(2):
        solve()
    ts = tv = 0.0
    info = None
    for _ in range(a.solves):
        s, v, info = solve()
        ts += s
        tv += v
    print(json.dumps({"seed": seed, "solver": a.solver, "eps": a.eps, "relax": a.relax, "learned": a.learned,
                      "setup_ms": ts / a.solves * 1e3, "solve_ms": tv / a.solves * 1e3, "iters": info["iters"],
                      "true_rel_res": info["true_rel_res"], "box": list(plan.box_stats())}), flush=True)


if __name__ == "__main__":
    main()

"""Time the box solvers (step S3) alone on the torus + sphere workload.

    python -m paper_2309_05965_amd.boxbench --dim 3 --N 256 --solver mg32 --solves 5

Builds the 4th-order torus + sphere problem (3D; the star in 2D) on an
N^d grid, sets the box solver (fft, mg64 or mg32; multigrid to --eps) and
runs --solves box solves of a seeded random right-hand side after one
untimed solve.  Prints one JSON line: ms per box solve (host clock around
the timed solves), multigrid corrections and relative residual reached.

    python -m paper_2309_05965_amd.boxbench --copy-mib 256

instead runs three plain device copies of that many MiB (the reference
kernel that scales the memory counters of a profile to bytes).
"""
import argparse
import json
import time

import torch

from . import kfbi
from . import workloads as W


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--solver", default="mg32", choices=["fft", "mg64", "mg32"])
    ap.add_argument("--eps", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=14)
    ap.add_argument("--solves", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=0)
    a = ap.parse_args()
    if a.copy_mib:
        n = a.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": a.copy_mib, "copies": 3}), flush=True)
        return
    prob = (W.config3(a.N) if a.dim == 3 else W.config2(a.N))[0]
    plan = kfbi.Plan(prob)
    plan.set_box_solver(a.solver, eps_in=a.eps, max_cycles=a.max_cycles)
    g = torch.Generator(device="cpu").manual_seed(7)
    F = torch.zeros(plan.n_nodes, dtype=torch.float64)
    inner = F.view((a.N + 1,) * a.dim)[(slice(1, a.N),) * a.dim]
    inner.copy_(torch.randn(inner.shape, dtype=torch.float64, generator=g))
    F = F.cuda()
    plan.box_solve(F)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.solves):
        plan.box_solve(F)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / a.solves * 1e3
    cycles, rel = plan.box_stats()
    print(json.dumps({"dim": a.dim, "N": a.N, "solver": a.solver, "eps": a.eps, "ms_per_box_solve": ms,
                      "corrections": cycles, "rel_residual": rel,
                      "tile_lines": {"N": kfbi.tile_lines(a.dim, a.N), "N/2": kfbi.tile_lines(a.dim, a.N // 2)}}),
          flush=True)


if __name__ == "__main__":
    main()

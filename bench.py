"""Benchmark: KFBI solves/s at 1e-8 relative GMRES residual on one MI355X,
plain FP64 against FP32 multigrid + learned warm start.

Workload (N=1): the learned-start workload, 3D fourth-order interface
problems on a 128^3 grid over [-1, 1]^3: random ellipsoids (semi-axes
U(0.3, 0.7), random rotation), beta 1/100, kappa 0, zero source and box
data, random Fourier jumps (8 modes, N(0, 1) coefficients), held-out seeds
from 1,000,000 on (the network never saw them).  One step is one whole
solve of one held-out problem that its plan has not solved before: set-up
(geometry and collocation, S0 + S1) of the new geometry, the learned
prediction of the initial density (mixed form), the BIE right-hand side,
GMRES over the simple-interface-problem operator (S2-S6) to |r| <= 1e-8 |b|,
the true residual of a fresh full-accuracy FP64 matvec, and the final grid
solve (S7).  The jump data are resident in HBM before the timed region.

  value (headline): the mixed + learned form, solves/s: FP32 multigrid
      V-cycles in FP64 defect correction to tol / 10, the inner tolerance
      relaxed inside GMRES (inexact Krylov), learned initial density;
  config.plain_fp64_solves_per_s: FP64 multigrid to 1e-12, zero start, on
      the same held-out problems (on a plan of its own);
  config.mixed_learned_over_plain: their ratio (the metric's comparison);
  forms.ellipsoid128_ingredients: each ingredient alone on the same
      problems, with the controls of the start: zero, the learned density and
      psi0 = g2 / (beta_in + beta_out).

Prints one JSON line (rank 0, N=1 only).  The roofline object reports the
exact coarse-grid solve's sine-transform pass (the kernel with the most time
in both forms), timed with HIP events on the plan's stream after the timed
region; cpu_baseline times the FP64 NumPy oracle on this host on one
held-out problem of the same workload.
"""
import os

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import argparse  # noqa: E402
import contextlib  # noqa: E402
import gc  # noqa: E402
import json  # noqa: E402
import platform  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

METRIC = "KFBI solves/s at 1e-8 rel residual: plain FP64 vs FP32-MG+learned warm start"
HBM_PEAK_GBS = 8000.0
HELDOUT0 = 1_000_000
# mixed form: inner tolerance tol * EPS_FRAC, relaxed inside GMRES by RELAX
EPS_FRAC = 0.1
RELAX = 3.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed held-out problems per form")
    ap.add_argument("--warmup", type=int, default=2, help="untimed held-out problems per form first")
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--workers", type=int, default=1,
                    help="also time both forms with this many host threads, each with its own plan and stream")
    ap.add_argument("--cpu-suite", action="store_true",
                    help="only time the oracle on every workload (long; one JSON line)")
    ap.add_argument("--form", default=None,
                    choices=("star512", "torus_sphere128", "torus_sphere256", "batch512_random_stars", "widened_rows",
                             "mg_smoothing_sweep_roofline_256"),
                    help="only this entry of `forms` (for profiling; one JSON line)")
    return ap.parse_args()


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "numpy": np.__version__}


# ---------------------------------------------------------------- oracle timings
def oracle_solve_config5(seed, N, tol):
    from oracle import kfbi as okfbi
    from paper_2309_05965_amd import workloads as W
    prob, geom, jmp = W.config5(seed, N)
    t0 = time.perf_counter()
    pl = okfbi.Plan(prob)
    data = W.jump_data(prob, jmp, pl.geo["surf"]["pos"])
    r = pl.solve(data, tol=tol)
    return time.perf_counter() - t0, r["iters"], r["true_rel_res"]


def oracle_solve_manufactured(prob, sol, tol):
    from oracle import kfbi as okfbi
    from paper_2309_05965_amd import workloads as W
    t0 = time.perf_counter()
    pl = okfbi.Plan(prob)
    s = pl.geo["surf"]
    data = W.make_data(prob, sol, s["pos"], s["nrm"], s["iface"], pl.geo["st"]["pde_pts"], pl.geo["dofs"]["iface"])
    r = pl.solve(data, tol=tol)
    return time.perf_counter() - t0, r["iters"], r["true_rel_res"]


def first_resolved_seeds(count, N, start=HELDOUT0):
    """The first `count` held-out seeds whose geometry the oracle resolves
    on the N^3 grid (the same rule the device applies)."""
    from oracle import geometry
    from paper_2309_05965_amd import workloads as W
    out, s = [], start
    while len(out) < count:
        try:
            geometry.build(W.config5(s, N)[0])
            out.append(s)
        except geometry.GeometryError:
            pass
        s += 1
    return out


def cpu_baseline(N, tol):
    """The oracle as it stands, one thread, one whole solve of the first
    resolvable held-out problem of the headline workload (zero start)."""
    seed = first_resolved_seeds(1, N)[0]
    el, its, tr = oracle_solve_config5(seed, N, tol)
    out = {"value": 1.0 / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": "1 whole solve (geometry, collocation, data, GMRES to %g, final solve) of held-out seed %d "
                     "of the 128^3 ellipsoid workload, %.1f s, %d iterations, true residual %.1e, NumPy/SciPy "
                     "FP64, 1 thread" % (tol, seed, el, its, tr)}
    out.update(cpu_info())
    return out


def cpu_suite(tol):
    """Oracle timings of every workload (one thread per solve; the batch
    over a process pool of all host cores).  Long: run on its own."""
    import multiprocessing as mp
    from paper_2309_05965_amd import workloads as W
    res = {"host": cpu_info(), "tol": tol}
    for name, mk in (("config1_ellipse64", lambda: W.config1(64)), ("config2_star512", lambda: W.config2(512)),
                     ("config3_torus_sphere128", lambda: W.config3(128))):
        times, its = [], []
        for _ in range(3 if name != "config3_torus_sphere128" else 1):
            prob, sol = mk()
            el, it, tr = oracle_solve_manufactured(prob, sol, tol)
            times.append(el)
            its.append(it)
        res[name] = {"median_s": float(np.median(times)), "solves_per_s": 1.0 / float(np.median(times)),
                     "runs": len(times), "iters": its[-1], "true_rel_res": tr}
        print(name, res[name], flush=True)
    seeds = first_resolved_seeds(16, 128)
    t0 = time.perf_counter()
    with mp.Pool(min(16, os.cpu_count() or 1)) as pool:
        rows = pool.starmap(oracle_solve_config5, [(s, 128, tol) for s in seeds])
    el = time.perf_counter() - t0
    res["config5_ellipsoid128_16_heldout"] = {"wall_s": el, "solves_per_s": len(seeds) / el, "processes": min(16, os.cpu_count() or 1),
                                               "iters_mean": float(np.mean([r[1] for r in rows])),
                                               "solve_s_median": float(np.median([r[0] for r in rows]))}
    print("config5", res["config5_ellipsoid128_16_heldout"], flush=True)
    batch = W.config4_batch(512)
    t0 = time.perf_counter()
    with mp.Pool(min(16, os.cpu_count() or 1)) as pool:
        rows = pool.map(_oracle_batch_one, range(len(batch)))
    el = time.perf_counter() - t0
    ok = sum(1 for r in rows if r)
    res["config4_batch512"] = {"wall_s": el, "solved": ok, "solved_per_s": ok / el, "processes": min(16, os.cpu_count() or 1)}
    print("config4", res["config4_batch512"], flush=True)
    res["widened_2d"] = oracle_widened(tol)
    return res


def _oracle_batch_one(i):
    from oracle import geometry
    from paper_2309_05965_amd import workloads as W
    prob, sol = W.config4_batch(512)[i]
    try:
        oracle_solve_manufactured(prob, sol, 1e-8)
        return True
    except geometry.GeometryError:
        return False


# ---------------------------------------------------------------- GPU forms
@contextlib.contextmanager
def no_gc():
    """The timed regions run with Python's cyclic garbage collector off (as
    timeit does), after a full collection: with torch loaded a generation-2
    pass walks about 170,000 objects and stalls the host for about 35 ms,
    which would land on whichever solve happened to trigger it."""
    was = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


class HeldOut:
    """The first `count` held-out problems of the ellipsoid workload that
    the set-up resolves on the N^3 grid, with their jump data resident on
    the device (generated at the solver's own surface points, which a
    set-up reproduces bit for bit)."""

    def __init__(self, count, N, start=HELDOUT0):
        import torch
        from paper_2309_05965_amd import kfbi
        from paper_2309_05965_amd import workloads as W
        self.items = []
        plan = None
        s = start
        while len(self.items) < count:
            prob, geom, jmp = W.config5(s, N)
            try:
                if plan is None:
                    plan = kfbi.Plan(prob)
                else:
                    plan.setup(prob)
                self.items.append((s, prob, geom, jmp, kfbi.device_jump_data(plan, jmp)))
            except kfbi.KfbiError:
                if plan is not None:
                    plan.close()
                plan = None
            s += 1
        torch.cuda.synchronize()
        plan.close()
        self.seeds = [it[0] for it in self.items]


def run_form_workers(ho, warm, timed, tol, solver, eps, relax, learned_start, workers):
    """Solves/s of one form with `workers` host threads, each with a plan
    and a model of its own on a stream of its own, taking every workers-th
    held-out problem (the library waits on the host inside a solve, so the
    threads overlap one solve's device work with another's host waits).
    Returns (solves/s, iterations, true residuals)."""
    import threading
    import torch
    from paper_2309_05965_amd import kfbi, warmstart
    items = ho.items[:warm + timed]
    streams = [torch.cuda.Stream() for _ in range(workers)]
    plans, models = [], []
    for w in range(workers):
        with torch.cuda.stream(streams[w]):
            pl = kfbi.Plan(items[0][1])
        pl.set_box_solver(solver, eps_in=eps, max_cycles=16)
        pl.set_box_relaxation(relax)
        plans.append(pl)
        models.append(warmstart.load_pretrained() if learned_start else None)
    errors = []

    def worker(w, idx, out):
        try:
            torch.cuda.set_stream(streams[w])
            for i in idx:
                _, prob, geom, jmp, data = items[i]
                plans[w].setup(prob)
                la = warmstart.learned_args(models[w], geom, jmp) if learned_start else None
                _, _, info = plans[w].solve(data, tol=tol, learned=la)
                out.append(info)
            streams[w].synchronize()
        except Exception as e:   # reported after the join
            errors.append(e)

    def run(first, count):
        outs = [[] for _ in range(workers)]
        ths = [threading.Thread(target=worker, args=(w, [first + i for i in range(count) if i % workers == w], outs[w]))
               for w in range(workers)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        if errors:
            raise errors[0]
        return [x for o in outs for x in o]

    run(0, warm)
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        infos = run(warm, timed)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    for pl in plans:
        pl.close()
    return timed / el, [i["iters"] for i in infos], [i["true_rel_res"] for i in infos]


def run_form(ho, warm, timed, tol, solver, eps, relax, learned_start, keep_u=False):
    """Solves/s of one form over held-out problems: a plan of its own, the
    first `warm` problems untimed, then `timed` problems, each solved once.
    Returns (solves/s, iterations, true residuals, densities, solutions)."""
    import torch
    from paper_2309_05965_amd import kfbi, learned, warmstart
    model = warmstart.load_pretrained() if learned_start is True else None
    items = ho.items[:warm + timed]
    plan = kfbi.Plan(items[0][1])
    plan.set_box_solver(solver, eps_in=eps, max_cycles=16)
    plan.set_box_relaxation(relax)
    n = plan.n_nodes
    U = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(timed)] if keep_u else None
    psis, its, trs = [], [], []

    def one(i, it):
        _, prob, geom, jmp, data = it
        plan.setup(prob)
        la = warmstart.learned_args(model, geom, jmp) if learned_start is True else None
        # the control start psi0 = g2 / (beta_in + beta_out) at the unknowns
        psi0 = None
        if learned_start == "g2":
            psi0 = data["g2"][plan.export("dof_surf").long()] / (prob["beta_in"] + prob["beta_out"])
        psi, _, info = plan.solve(data, tol=tol, learned=la, psi0=psi0,
                                  u_out=U[i] if (keep_u and i >= 0) else None)
        return psi, info

    for it in items[:warm]:
        one(-1, it)
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        for i, it in enumerate(items[warm:]):
            psi, info = one(i, it)
            psis.append(psi)
            its.append(info["iters"])
            trs.append(info["true_rel_res"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    plan.close()
    return timed / el, its, trs, psis, U


# HBM traffic of an active coarse solve on the 64^3 coarse grid of a 128^3
# box with the FP32 inner cycle, per launch averaged over its five passes
# (the first restricts the fine residual as it loads; FETCH_SIZE x 2 +
# WRITE_SIZE x 1 per dispatch, the factors read off a plain 256 MiB copy;
# profiles/mg_kernels_torus128_256_hbm_counters.md)
COARSE_PASS_TRAFFIC_128 = 5.755e6


def coarse_pass_roofline(prob, N, solver):
    """Average duration of a pass of the multigrid's exact coarse solve (the
    kernel that takes the most time in both forms; HIP events on the plan's
    stream around the five passes of every cycle of eager box solves, every
    correction active).  Algorithmic bytes per coarse solve: one FP64 read
    and one FP64 write of each interior coarse node in each of the last four
    passes; the first pass forms the coarse right-hand side from the fine
    residual as it loads (one read of each interior fine node in the inner
    precision, one FP64 write of each interior coarse node); reported per
    launch (the solve's total over its five launches)."""
    import torch
    from paper_2309_05965_amd import kfbi
    plan = kfbi.Plan(prob)
    plan.set_box_solver(solver, eps_in=1e-30, max_cycles=8)     # all 8 corrections active
    F = torch.randn(plan.n_nodes, dtype=torch.float64, device="cuda")
    plan.box_solve(F)
    plan.profile(3)
    for _ in range(10):
        plan.box_solve(F)
    ivals, launches, ms = plan.timing()
    plan.profile(False)
    plan.close()
    nc = N // 2
    inner = 4 if solver == "mg32" else 8
    bytes_per_launch = (4 * 16 * (nc - 1) ** 3 + inner * (N - 1) ** 3 + 8 * (nc - 1) ** 3) / 5
    avg_s = ms / 1e3 / launches
    achieved = bytes_per_launch / avg_s / 1e9
    return {"kernel": "k_dst coarse sine-transform passes, %d^3 coarse grid of the %d^3 multigrid (FP64; the "
                      "first restricts the fine residual on load)" % (nc, N),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": COARSE_PASS_TRAFFIC_128 if (N == 128 and solver == "mg32") else None,
            "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_per_launch,
            "timing": "HIP events around the %d coarse solves (%d launches) of 10 eager box solves after the "
                      "timed region" % (ivals, launches)}


def sweep_roofline_256():
    """The finest-level smoothing sweep of the multigrid at 256^3 (torus +
    sphere box, 2.5D-blocked sweeps): HIP events on the plan's stream around
    the two post-smoothing steps of every cycle of eager box solves (every
    correction active).  Algorithmic bytes per launch: u and f read, u'
    written, 4 B each in FP32 and 8 B in FP64, per interior node."""
    import torch
    from paper_2309_05965_amd import kfbi
    from paper_2309_05965_amd import workloads as W
    N = 256
    prob, _ = W.config3(N)
    plan = kfbi.Plan(prob)
    out = {}
    for solver, b in (("mg32", 12), ("mg64", 24)):
        plan.set_box_solver(solver, eps_in=1e-30, max_cycles=4)
        F = torch.randn(plan.n_nodes, dtype=torch.float64, device="cuda")
        plan.box_solve(F)
        plan.profile(2)
        for _ in range(3):
            plan.box_solve(F)
        ivals, launches, ms = plan.timing()
        plan.profile(False)
        bytes_per_launch = b * (N - 1) ** 3
        avg_s = ms / 1e3 / launches
        achieved = bytes_per_launch / avg_s / 1e9
        out["fp32" if solver == "mg32" else "fp64"] = {
            "kernel": "k_sweep3 smoothing step, %d^3 (%s)" % (N, "FP32" if solver == "mg32" else "FP64"),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_per_launch,
            "timing": "HIP events around %d launches in %d events of 3 eager box solves" % (launches, ivals)}
    plan.close()
    return out


def forms_config5_ingredients(ho, warm, timed, tol):
    """Each ingredient of the mixed form alone, on the same held-out problems
    (a plan per form, each problem solved once per plan)."""
    out = {}
    for name, solver, eps, relax, ls in (
            ("fp32_mg_relaxed_zero_start", "mg32", EPS_FRAC * tol, RELAX, False),
            ("fp64_mg_relaxed_zero_start", "mg64", EPS_FRAC * tol, RELAX, False),
            ("fp32_mg_relaxed_g2_start", "mg32", EPS_FRAC * tol, RELAX, "g2"),
            ("fp32_mg_unrelaxed_learned_start", "mg32", EPS_FRAC * tol, 0.0, True),
            ("fp64_fft_zero_start", "fft", 1e-12, 0.0, False),
            ("fp64_fft_learned_start", "fft", 1e-12, 0.0, True)):
        v, its, trs, _, _ = run_form(ho, warm, timed, tol, solver, eps, relax, ls)
        out[name] = {"solves_per_s": v, "iters_mean": float(np.mean(its)), "true_rel_res_max": float(np.max(trs))}
    return out


def forms_star512(tol, steps=10):
    """The 2D fourth-order star (512^2, beta 1000/1), FP64 FFT box solve,
    one repeated problem, set-up included (the paper's own solver)."""
    import torch
    from paper_2309_05965_amd import kfbi
    from paper_2309_05965_amd import workloads as W
    prob, sol = W.config2(512)
    plan = kfbi.Plan(prob)
    data = kfbi.device_data(plan, prob, sol)
    u = torch.empty(plan.n_nodes, dtype=torch.float64, device="cuda")
    for _ in range(3):
        plan.setup(prob)
        plan.solve(data, tol=tol, u_out=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.setup(prob)
        _, _, info = plan.solve(data, tol=tol, u_out=u)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    reg = plan.export("region").cpu().numpy().reshape(513, 513)
    err = float(np.max(np.abs(u.cpu().numpy() - W.exact_solution(prob, sol, reg).ravel())))
    plan.close()
    return {"fp64_fft_solves_per_s": steps / el, "iters": info["iters"], "max_error_vs_exact": err}


def forms_config3(tol, N):
    """Torus + concentric sphere (gap 2h, beta 1/100, 4th order): FP64 FFT
    and the mixed FP32-multigrid form, one repeated problem, set-up
    included; maximum error against the exact solution."""
    import torch
    from paper_2309_05965_amd import kfbi
    from paper_2309_05965_amd import workloads as W
    prob, sol = W.config3(N)
    plan = kfbi.Plan(prob)
    data = kfbi.device_data(plan, prob, sol)
    reg = plan.export("region").cpu().numpy().reshape((N + 1,) * 3)
    ue = W.exact_solution(prob, sol, reg).ravel()
    u = torch.empty(plan.n_nodes, dtype=torch.float64, device="cuda")
    out = {"n_dof": int(plan.n_dof)}
    reps = 5 if N <= 128 else 2
    for name, solver, eps, relax in (("fp64_fft", "fft", 1e-12, 0.0), ("fp32_mg_relaxed", "mg32", EPS_FRAC * tol, RELAX),
                                     ("fp64_mg_eps1e-12", "mg64", 1e-12, 0.0)):
        plan.set_box_solver(solver, eps_in=eps, max_cycles=16)
        plan.set_box_relaxation(relax)
        for _ in range(2):
            plan.setup(prob)
            plan.solve(data, tol=tol, u_out=u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.setup(prob)
            _, _, info = plan.solve(data, tol=tol, u_out=u)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"solves_per_s": reps / el, "iters": info["iters"], "true_rel_res": info["true_rel_res"],
                     "max_error_vs_exact": float(np.max(np.abs(u.cpu().numpy() - ue)))}
    plan.close()
    return out


def widened_2d():
    """2D problems of the widened rows, small enough for the oracle: the
    paper's Dirichlet ellipse, a Neumann problem on it, a two-density
    Poisson / modified-Helmholtz ellipse and the workload star given by its
    node samples, all at 256^2."""
    from paper_2309_05965_amd import workloads as W
    neu, u1 = W.e1_dirichlet(256)
    neu = dict(neu, bie="neumann")
    td = W.td_problem(2, 4, 256, -1.0, 1.0, 1.0, 4.0, 0.0, 2.5, [W.ellipse2d(0.05, -0.02, 0.6, 0.45, theta=0.3)])
    star, ssol = W.config2(256)
    return [("dirichlet_ellipse256", W.e1_dirichlet(256)), ("neumann_ellipse256", (neu, u1)),
            ("two_density_ellipse256", (td, {0: W.f_sin_sin, 1: W.f_exp_cos})),
            ("star256_sampled_quintic", (W.with_sampled(star, W.H_star(0.5, 0.3, 5), 5), ssol))]


def oracle_widened(tol):
    """The oracle's whole solves (set-up included) of the 2D widened problems,
    one thread each."""
    from oracle import bvp, kfbi as okfbi, twodensity
    from paper_2309_05965_amd import workloads as W
    out = {}
    for name, (prob, sol) in widened_2d():
        t0 = time.perf_counter()
        bie = prob.get("bie", "interface")
        if bie in ("dirichlet", "neumann"):
            pl = bvp.BVPPlan(prob)
            s = pl.geo["surf"]
            res = pl.solve(W.make_bvp_data(prob, sol, s["pos"], s["nrm"], pl.geo["st"]["pde_pts"]), tol=tol)
        elif bie == "two_density":
            pl = twodensity.TwoDensityPlan(prob)
            s = pl.geo["surf"]
            res = pl.solve(W.make_td_data(prob, sol, s["pos"], s["nrm"], s["iface"], pl.geo["st"]["pde_pts"],
                                          pl.geo["dofs"]["iface"]), tol=tol)
        else:
            pl = okfbi.Plan(prob)
            s = pl.geo["surf"]
            res = pl.solve(W.make_data(prob, sol, s["pos"], s["nrm"], s["iface"], pl.geo["st"]["pde_pts"],
                                       pl.geo["dofs"]["iface"]), tol=tol)
        el = time.perf_counter() - t0
        out[name] = {"seconds": el, "solves_per_s": 1.0 / el, "iters": res["iters"]}
        print(name, out[name], flush=True)
    return out


def forms_widened(tol, reps=5):
    """The widened rows on repeated problems (FFT box solver, GMRES to tol):
    the interior Neumann problem in the torus and the two-density
    three-sphere problem at 128^3, the molecular surface at contrast 1e4:1,
    and the torus of the 3D workload given only by its node samples next to
    the same torus given analytically.  Solve time with the plan set up and
    the data resident; the set-up (S0 + S1) timed separately; maximum error
    against the exact solution on the nodes of the solution's regions."""
    import torch
    from paper_2309_05965_amd import kfbi
    from paper_2309_05965_amd import workloads as W
    cases = dict(widened_2d())
    torus = W.problem(3, 4, 128, -1.0, 1.0, 1.0, 100.0, 0.0, [W.torus3d(0.0, 0.0, 0.0, 0.6, 0.25)])
    cases.update({
        "neumann_torus128": W.e3_neumann(128),
        "two_density_three_spheres128": W.e7_heterogeneous(128),
        "molecule128_contrast1e4": W.e5_molecule(128, 1e4),
        "torus128_analytic": (torus, {0: W.f_exp3, 1: W.f_sin3}),
        "torus128_sampled_quintic": (W.with_sampled(torus, W.H_torus(0.6, 0.25), 5), {0: W.f_exp3, 1: W.f_sin3}),
    })
    out = {}
    for name, (prob, sol) in cases.items():
        bie = prob.get("bie", "interface")
        plan = kfbi.Plan(prob)
        if bie in ("dirichlet", "neumann"):
            data = kfbi.device_bvp_data(plan, prob, sol)
        elif bie == "two_density":
            data = kfbi.device_td_data(plan, prob, sol)
        else:
            data = kfbi.device_data(plan, prob, sol)
        u = torch.empty(plan.n_nodes, dtype=torch.float64, device="cuda")
        plan.solve(data, tol=tol, u_out=u, max_iter=300)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, _, info = plan.solve(data, tol=tol, u_out=u, max_iter=300)
        torch.cuda.synchronize()
        t_solve = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(2):
            plan.setup(prob)
        torch.cuda.synchronize()
        t_setup = (time.perf_counter() - t0) / 2
        reg = plan.export("region").cpu().numpy().ravel()
        un = u.cpu().numpy()
        if bie in ("dirichlet", "neumann"):
            ue = W.bvp_exact(prob, sol).ravel()
            m = reg > 0
            d = (un - ue)[m]
            err = float(np.max(np.abs(d - d.mean()))) if bie == "neumann" else float(np.max(np.abs(d)))
        else:
            ue = W.exact_solution(prob, sol, reg.reshape((prob["N"] + 1,) * prob["dim"])).ravel()
            err = float(np.max(np.abs(un - ue)))
        out[name] = {"solves_per_s": 1.0 / t_solve, "setup_ms": 1e3 * t_setup, "iters": info["iters"],
                     "unknowns": int(plan.n_unknowns), "true_rel_res": info["true_rel_res"],
                     "max_error_vs_exact": err}
        plan.close()
        torch.cuda.empty_cache()
    return out


def tile_lines_of(dim, n):
    from paper_2309_05965_amd import kfbi
    return kfbi.tile_lines(dim, n)


def forms_batch(workers=(1, 8)):
    """The 512-problem batch of random stars (N in {64, 128, 256, 512},
    beta_in log-uniform 1e-2..1e2): solved problems per second over the
    whole batch, set-up and data generation included (stars the grid does
    not resolve fail in set-up, as the oracle's set-up reports them, and are
    not counted as solved).  Set up, then solve (a plan per problem, the data
    generated at every plan's query points) and streaming (a plan per grid
    shape per worker, the data from the generator's callback)."""
    import torch
    from paper_2309_05965_amd import kfbi
    from paper_2309_05965_amd import manufactured as M
    from paper_2309_05965_amd import workloads as W
    probs = [p for p, _ in W.config4_batch(512)]
    gen = M.BatchData(probs, ["star2d"] * len(probs))
    out = {}
    for w in workers:
        b = kfbi.Batch(probs, workers=w)
        b.solve_stream(gen.fn, gen.ctx, tol=1e-8, raise_on_fail=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _ = b.solve_stream(gen.fn, gen.ctx, tol=1e-8, raise_on_fail=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ok = sum(1 for i in info if i["status"] == 0)
        out["stream_workers_%d" % w] = {"solved_per_s": ok / el, "solved": ok, "unresolved": len(probs) - ok,
                                        "wall_s": el}
        b.close()
        for rep in range(2):
            b = kfbi.Batch(probs, workers=w)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.setup()
            t1 = time.perf_counter()
            plans = [b.plan(i) for i in range(len(probs))]
            data = [M.plan_data(pl, "star2d") if pl is not None else None for pl in plans]
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            _, info, _ = b.solve(data, tol=1e-8, raise_on_fail=False)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            ok = sum(1 for i in info if i["status"] == 0)
            if rep == 1:
                out["setup_then_solve_workers_%d" % w] = {
                    "solved_per_s": ok / (t3 - t0), "solved": ok, "wall_s": t3 - t0, "setup_s": t1 - t0,
                    "data_s": t2 - t1, "solve_s": t3 - t2}
            del plans, data
            b.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the method has no multi-GPU path in this build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    if args.cpu_suite:
        print(json.dumps(cpu_suite(args.tol)), flush=True)
        return
    import torch
    torch.cuda.set_device(0)
    # plans live on a stream of their own (a caller's non-default stream is
    # used for the solve as it is; on the default stream the library orders
    # a private stream before and after every solve with events)
    torch.cuda.set_stream(torch.cuda.Stream())
    # the GPU phases run with the cyclic collector off (collections between
    # phases only; see no_gc)
    gc.collect()
    gc.disable()
    if args.form:
        run = {"star512": lambda: forms_star512(args.tol), "torus_sphere128": lambda: forms_config3(args.tol, 128),
               "torus_sphere256": lambda: forms_config3(args.tol, 256), "batch512_random_stars": forms_batch,
               "mg_smoothing_sweep_roofline_256": sweep_roofline_256,
               "widened_rows": lambda: forms_widened(args.tol)}[args.form]
        print(json.dumps({"forms": {args.form: run()}}), flush=True)
        return
    N, tol = args.N, args.tol
    W_, K = args.warmup, args.steps
    ho = HeldOut(W_ + K, N)
    seeds = ho.seeds

    mixed, its_m, trs_m, psi_m, U_m = run_form(ho, W_, K, tol, "mg32", EPS_FRAC * tol, RELAX, True, keep_u=True)
    plain, its_p, trs_p, psi_p, U_p = run_form(ho, W_, K, tol, "mg64", 1e-12, 0.0, False, keep_u=True)
    du = max(float(((a - b).abs().max() / b.abs().max()).item()) for a, b in zip(U_m, U_p))
    dpsi = max(float(((a - b).norm() / b.norm()).item()) for a, b in zip(psi_m, psi_p))
    del U_m, U_p
    torch.cuda.empty_cache()
    roof = coarse_pass_roofline(ho.items[0][1], N, "mg32")

    out = {
        "metric": METRIC,
        "value": mixed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W_,
        "ms_per_step": 1e3 / mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "3D 4th-order KFBI, learned-start workload: random ellipsoids (axes U(0.3,0.7), random "
                        "rotation), %d^3 grid on [-1,1]^3, beta_in/out 1/100, kappa 0, zero source and box data, "
                        "random Fourier jumps (8 modes), held-out seeds %d..%d, each solved once per form, set-up "
                        "and prediction inside the timed solve, GMRES tol %g" % (N, seeds[W_], seeds[-1], tol),
            "mixed_form": "FP32 multigrid V(2,2) in FP64 defect correction to %g, relaxed inside GMRES (factor %g), "
                          "learned initial density (bf16 MLP)" % (EPS_FRAC * tol, RELAX),
            "plain_form": "FP64 multigrid V(2,2) in FP64 defect correction to 1e-12, zero start",
            "plain_fp64_solves_per_s": plain,
            "mixed_learned_over_plain": mixed / plain,
            "gmres_iters_mean": {"mixed": float(np.mean(its_m)), "plain": float(np.mean(its_p))},
            "true_rel_res_max": {"mixed": float(np.max(trs_m)), "plain": float(np.max(trs_p))},
            "mixed_vs_plain_max_rel_diff": {"u": du, "psi_l2": dpsi},
            "sine_transform_tile_lines": {"3d_%d" % n: tile_lines_of(3, n) for n in (N // 2, N)},
        },
        "roofline": roof,
    }
    if args.workers > 1:
        wm = run_form_workers(ho, W_, K, tol, "mg32", EPS_FRAC * tol, RELAX, True, args.workers)
        wp = run_form_workers(ho, W_, K, tol, "mg64", 1e-12, 0.0, False, args.workers)
        out["config"]["workers_%d" % args.workers] = {
            "mixed_solves_per_s": wm[0], "plain_fp64_solves_per_s": wp[0], "mixed_learned_over_plain": wm[0] / wp[0],
            "true_rel_res_max": {"mixed": float(np.max(wm[2])), "plain": float(np.max(wp[2]))}}
    gc.collect()
    if not args.no_forms:
        out["forms"] = {
            "ellipsoid128_ingredients": forms_config5_ingredients(ho, W_, min(K, 8), tol),
            "star512": forms_star512(tol),
            "torus_sphere128": forms_config3(tol, 128),
            "torus_sphere256": forms_config3(tol, 256),
            "mg_smoothing_sweep_roofline_256": sweep_roofline_256(),
            "batch512_random_stars": forms_batch(),
            "widened_rows": forms_widened(tol),
        }
    gc.enable()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, tol)
        # the oracle beside the widened rows' GPU solves (forms.widened_rows, the 2D problems)
        out["cpu_baseline"]["widened_2d"] = oracle_widened(tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

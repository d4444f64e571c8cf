"""Benchmark of the p-multigrid pressure Poisson path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the paper's time-stepping configuration): Nx = 256 Fourier x Nz = 17 Chebyshev, flat
bed h = 1, periodic L = 2 pi, second-order Stokes wave kh = 1, H/L = 0.05. One step is one pass of
the hot path: set the geometry of the stage (sigma-metrics and smoother block inverses) and solve
the pressure Poisson problem to relative residual 1e-10 with FGMRES preconditioned by one
p-multigrid V-cycle per iteration. The headline value is mixed precision (float32 V-cycle inside a
float64 outer iteration); the float64 plan is timed alongside, with the difference of the two
solutions.

Prints ONE JSON line (rank 0). See the design notes for the work model behind `roofline`.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


# ----------------------------------------------------------------------------- work model
def level_rows(nz):
    out = [nz]
    while out[-1] > 3:
        out.append((out[-1] + 1) // 2)
    return out


def apply_flops(nx, nz):
    """Algorithmic flops of one operator apply on an nz x nx level: three D_sigma contractions
    (2 nz per point each), two D_x passes (packed complex FFT pairs, 5 log2 nx + 3 per point each)
    and the pointwise metric terms (~18 per point)."""
    return nx * nz * (6 * nz + 10 * math.log2(nx) + 24)


def vcycle_flops(nx, nz, nu1=1, nu2=1, coarse_pairs=4):
    tot = 0.0
    rows = level_rows(nz)
    for li, r in enumerate(rows):
        n = nx * r
        a = apply_flops(nx, r)
        colstep = 2 * r * n + a
        modestep = a + n * (5 * math.log2(nx) + 2 * r + 2)
        pairs = coarse_pairs if li == len(rows) - 1 else nu1 + nu2
        tot += pairs * (colstep + modestep) - a          # first column step starts from zero
        if li < len(rows) - 1:
            tot += a + 2 * n * ((r + 1) // 2) + 2 * n * ((r + 1) // 2)   # residual, R, P
    return tot


def solve_flops(nx, nz, iters):
    n = nx * nz
    per_it = vcycle_flops(nx, nz) + apply_flops(nx, nz) + sum(4 * n * (j + 2) for j in range(1))
    arnoldi = sum(4.0 * n * (j + 2) for j in range(iters))
    return iters * per_it + arnoldi + 2 * apply_flops(nx, nz)


def solve_bytes(nx, nz, iters, ws):
    """Algorithmic bytes of one solve: each kernel phase reads its inputs once and writes its
    outputs once; ws = word size of the V-cycle (8 float64, 4 mixed)."""
    n = nx * nz
    nl = sum(nx * r for r in level_rows(nz))
    tot = 24 * n
    for j in range(iters):
        tot += 16 * n + (2 * j + 4) * 8 * n + 19 * ws * nl + ws * n
    return tot + (iters * ws + 16) * n


# ----------------------------------------------------------------------------- helpers
def _plan(pr, precision):
    import torch

    from paper_2406_00991_amd import pmgw
    plan = pmgw.Plan([pr["nx"]], [pr["nz"]], [pr["L"]], precision=precision)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                 device="cuda")
    return plan, dev(pr["h"]), dev(pr["eta_old"]), dev(pr["eta_new"]), dev(pr["b"])


def _time_steps(plan, h, eo, en, b, steps, warmup, rtol):
    import torch
    p = plan.field()
    for _ in range(warmup):
        plan.set_geometry(h, eo, en)
        p.zero_()
        plan.solve(b, p=p, rtol=rtol, maxit=100, sync=False)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        plan.set_geometry(h, eo, en)
        p.zero_()
        ev[k][0].record()
        plan.solve(b, p=p, rtol=rtol, maxit=100, sync=False)
        ev[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    solve_ms = float(np.mean([a.elapsed_time(c) for a, c in ev]))
    info = plan.solve(b, p=p.zero_(), rtol=rtol, maxit=100)[1]
    return wall, solve_ms, info, p


def cpu_baseline(pr, budget_s=12.0):
    """The oracle as it stands: FGMRES with its own dense-step V-cycle, on the host's cores."""
    from oracle import krylov
    from oracle import operator as op
    from oracle import pmg
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    go = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    gn = op.Geometry(pr["h"], pr["eta_new"], pr["L"])
    n_done, t0 = 0, time.perf_counter()
    while True:
        H = pmg.Hierarchy(pr["nx"], pr["nz"] - 1, go, gn, pmg.PmgOptions())
        krylov.fgmres(lambda v: op.apply(v, go, gn), pr["b"], H, rtol=1e-10)
        n_done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=n_done / dt, unit="solves/s", cores=cores, kind="oracle",
                sample=f"{n_done} solves of the {pr['nx']}x{pr['nz']} problem (setup + FGMRES "
                       f"to 1e-10), NumPy/SciPy float64")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (tanks shard across GPUs "
              "without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2406_00991_amd import workloads as wl
    torch.cuda.set_device(0)
    pr = wl.stokes_rest_problem(256, 17)
    rtol = 1e-10
    res = {}
    for prec in ("mixed", "fp64"):
        plan, h, eo, en, b = _plan(pr, prec)
        wall, solve_ms, info, p = _time_steps(plan, h, eo, en, b, args.steps, args.warmup, rtol)
        res[prec] = dict(wall=wall, solve_ms=solve_ms, iters=info[0][0], relres=info[0][2],
                         p=p.cpu().numpy())
    mix, f64 = res["mixed"], res["fp64"]
    delta = float(np.linalg.norm(mix["p"] - f64["p"]) / np.linalg.norm(f64["p"]))
    nx, nz = pr["nx"], pr["nz"]
    it = mix["iters"]
    flops = solve_flops(nx, nz, it)
    byts = solve_bytes(nx, nz, it, 4)
    t_s = mix["solve_ms"] * 1e-3
    achieved = flops / t_s / 1e12
    out = {
        "metric": "Poisson solves/s at rel. residual 1e-10 (mixed float32 V-cycle / float64 "
                  "FGMRES)",
        "value": args.steps / mix["wall"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mix["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "stokes-wave pressure solve, Nx=256 x Nz=17, flat bed h=1, "
                               "kh=1, H/L=0.05, first stage from rest, one tank",
                   "precision": "mixed", "rtol": rtol},
        "fp64": {"value": args.steps / f64["wall"], "unit": "solves/s",
                 "ms_per_step": 1e3 * f64["wall"] / args.steps, "iters": f64["iters"],
                 "relres": f64["relres"]},
        "mixed": {"iters": mix["iters"], "relres": mix["relres"],
                  "rel_diff_vs_fp64": delta},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_solve<float,17> (one workgroup per tank)",
                     "launch_ms": mix["solve_ms"], "flops_per_launch": flops,
                     "alg_bytes_per_launch": byts,
                     "alg_GBps": byts / t_s / 1e9,
                     "cus_used": 1,
                     "frac_of_one_cu": achieved / (FP32_PEAK_TFLOPS / 256)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pr)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

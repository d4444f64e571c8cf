"""Benchmark of the hybrid-spectral time-stepping hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload: RK4 time stepping of a second-order Stokes wave, Nx = 256 Fourier x Nz = 17 Chebyshev
points, flat bed h = 1, periodic L = 2 pi, kh = 1, H/L = 0.05, dt from CFL 0.5 on the linear
phase speed. One step is one time step of the low-storage scheme: five stages, each with the
kinematic surface update, the sigma-metrics of the new surface and the smoother block inverses,
the forcing, the pressure Poisson solve (FGMRES to relative residual 1e-10, one p-multigrid
V-cycle per iteration, warm-started from the previous stage's pressure), the projection and the
filters. The headline value is Poisson solves per second in mixed precision (float32 V-cycle
inside a float64 outer iteration); the float64 plan runs the same steps alongside, and the
difference of the two final states is reported.

Prints ONE JSON line. `roofline` covers the dominant kernel (the solve kernel): algorithmic bytes
per launch from the work model below over its mean launch duration, timed with HIP events on the
plan's stream inside the timed region.
"""
import argparse
import hashlib
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_solve_stokes256x17_traffic.json")


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


def vcycle_flops(nx, nz, nu1=1, nu2=1, coarse_pairs=1):
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
    per_it = vcycle_flops(nx, nz) + apply_flops(nx, nz)
    arnoldi = sum(4.0 * n * (j + 2) for j in range(int(round(iters))))
    return iters * per_it + arnoldi + 2 * apply_flops(nx, nz)


def solve_bytes(nx, nz, iters, ws):
    """Algorithmic bytes of one solve: each phase reads its inputs once and writes its outputs
    once; per iteration j the Arnoldi step streams (2j + 4) float64 vectors, the V-cycle 19 words
    per point of every level, and the preconditioned vector one; ws = word size of the V-cycle
    (8 float64, 4 mixed)."""
    n = nx * nz
    nl = sum(nx * r for r in level_rows(nz))
    tot = 24 * n
    for j in range(int(round(iters))):
        tot += 16 * n + (2 * j + 4) * 8 * n + 19 * ws * nl + ws * n
    return tot + (iters * ws + 16) * n


def kernel_source_hash():
    """Hash of the 2D library's HIP sources (every file but the 3D tanks' pmgw3d*); the stored
    HBM counter readings of the 2D solve kernel are used only while it matches."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2406_00991_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp")) and not name.startswith("pmgw3d"):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def stored_traffic(kernel, precision):
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}/{precision}")
    return None if ent is None else float(ent["bytes_per_launch"])


# ----------------------------------------------------------------------------- GPU run
class Tank:
    """Device state of one tank and the stage loop through the C ABI."""

    def __init__(self, wave, precision, capacity, opts=None):
        import torch

        from paper_2406_00991_amd import pmgw
        self.pmgw = pmgw
        self.wave = wave
        self.plan = pmgw.Plan([wave["nx"]], [wave["nz"]], [wave["L"]], precision=precision,
                              opts=opts)
        dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                     device="cuda")
        self.h, self.u, self.w, self.eta = (dev(wave[k]) for k in ("h", "u", "w", "eta"))
        self.Ku = torch.zeros_like(self.u)
        self.Kw = torch.zeros_like(self.u)
        self.Keta = torch.zeros_like(self.eta)
        self.p = torch.zeros_like(self.u)
        self.info = pmgw.info_buffer(capacity)      # one record per stage
        self.nstage = 0

    def step(self, dt, rtol):
        for k in range(1, 6):
            rec = self.info[2 * self.nstage: 2 * self.nstage + 2]
            self.pmgw.rk4_stage(self.plan, k, dt, self.h, self.u, self.w, self.eta, self.Ku,
                                self.Kw, self.Keta, self.p, rtol=rtol, maxit=100, info_dev=rec)
            self.nstage += 1

    def infos(self, first, count):
        return self.pmgw.read_info(self.info[2 * first: 2 * (first + count)])


def run_precision(wave, precision, steps, warmup, rtol, guess=0, correct=0):
    """RK4 stepping of one tank; guess = opts.guess_steps (0: each solve starts from the previous
    stage's pressure), correct = opts.guess_correct."""
    import torch

    from paper_2406_00991_amd import pmgw
    opts = pmgw.default_opts(guess_steps=guess, guess_correct=correct) if guess else None
    T = Tank(wave, precision, 5 * (steps + warmup), opts)
    dt = wave["dt"]
    for _ in range(warmup):
        T.step(dt, rtol)
    torch.cuda.synchronize()
    T.pmgw.profile_start(T.plan, 5 * steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        T.step(dt, rtol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, tot_ms, max_ms = T.pmgw.profile_read(T.plan)
    T.pmgw.profile_start(T.plan, 0)
    infos = T.infos(5 * warmup, 5 * steps)
    return dict(wall=wall, launches=launches, solve_ms=tot_ms / max(launches, 1), max_ms=max_ms,
                iters=float(np.mean([i["iters"] for i in infos])),
                iters_each=[int(i["iters"]) for i in infos],
                max_iters=int(max(i["iters"] for i in infos)),
                relres=float(max(i["relres"] for i in infos)),
                status=sorted({i["status"] for i in infos}),
                u=T.u.cpu().numpy(), w=T.w.cpu().numpy(), eta=T.eta.cpu().numpy(),
                p=T.p.cpu().numpy())


def run_batch(seed, ntanks, reps, rtol):
    """The batched workload: ntanks tanks of uneven (Nx, Nz), first-stage problems, one mixed
    plan; `reps` timed batched solves (one poisson_solve call each, zero initial guess) in the
    configuration the per-class tuner picks for this batch (searched here, on this device, on
    these problems), with the library's default configuration timed beside it."""
    import torch

    from paper_2406_00991_amd import autotune
    from paper_2406_00991_amd import pmgw
    from paper_2406_00991_amd import workloads as wl
    tanks = wl.batch(seed, ntanks)
    nx, nz, L = ([t[k] for t in tanks] for k in ("nx", "nz", "L"))
    cat = lambda key: torch.tensor(np.concatenate([np.asarray(t[key]).ravel() for t in tanks]),
                                   dtype=torch.float64, device="cuda")
    h, eo, en, b = cat("h"), cat("eta_old"), cat("eta_new"), cat("b")
    t_default = autotune.time_batch(nx, nz, L, h, eo, en, b, "mixed", pmgw.default_opts(),
                                    rtol, reps)
    t0 = time.perf_counter()
    choice, log = autotune.tune(nx, nz, L, h, eo, en, b, "mixed", rtol, reps=2, cache=False)
    t_search = time.perf_counter() - t0
    plan = pmgw.Plan(nx, nz, L, precision="mixed", opts=pmgw.default_opts(**choice))
    plan.set_geometry(h, eo, en)
    p = plan.field()
    pmgw.poisson_solve(plan, b, p, rtol=rtol, maxit=200, sync=False)
    torch.cuda.synchronize()
    pmgw.profile_start(plan, reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        p.zero_()
        pmgw.poisson_solve(plan, b, p, rtol=rtol, maxit=200, sync=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, tot_ms, _ = pmgw.profile_read(plan)
    info = pmgw.poisson_solve(plan, b, p.zero_(), rtol=rtol, maxit=200)
    its = [i[0] for i in info]
    byts = sum(solve_bytes(t["nx"], t["nz"], k, 4) for t, k in zip(tanks, its))
    t_launch = tot_ms / max(launches, 1) * 1e-3
    rows = pmgw.CLASS_ROWS
    present = sorted({t["nz"] for t in tanks})
    return {"workload": f"{ntanks} tanks, seed {seed}, Nx in {{64,128,256,512}}, "
                        "Nz in {9,17,33}, first-stage problems, mixed precision, rtol 1e-10",
            "value": ntanks * reps / wall, "unit": "tank-solves/s",
            "mean_batch_ms": tot_ms / max(launches, 1), "points": int(sum(t["nx"] * t["nz"] for t in tanks)),
            "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
            "status": sorted({i[1] for i in info}),
            "tuned": {"class_threads": {r: choice["class_threads"][rows.index(r)] for r in present},
                      "class_resident": {r: ["default", "lds", "global"][
                          choice["class_resident"][rows.index(r)]] for r in present},
                      "default_config_batch_ms": t_default, "search_s": t_search,
                      "search": [{"rows": r, "threads": t, "cycle": ["default", "lds", "global"][c],
                                  "batch_ms": ms} for r, t, c, ms in log]},
            "roofline": {"bound": "hbm", "achieved": byts / t_launch / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": byts / t_launch / 1e9 / HBM_PEAK_GBS,
                         "alg_bytes_per_batch": byts}}


# ----------------------------------------------------------------------------- bar workload
def run_bar(seeds, reps, rtol):
    """The 1024 x 33 trapezoidal bar, first-stage problem from rest, one tank per seed, in the
    mixed and the float64 plan: mean launch time of one solve from zero (HIP events on the plan's
    stream, `reps` solves per seed after one warm-up), solves/s = 1 / that time, iterations, and
    the solve kernel's algorithmic bytes over its launch time against the HBM peak."""
    import torch

    from paper_2406_00991_amd import pmgw
    from paper_2406_00991_amd import workloads as wl
    out = {"workload": f"trapezoidal bar, Nx=1024 x Nz=33, depth 0.4 to 0.1 (slopes 1:20, 1:10), "
                       f"seeded monochromatic wave plus 1% noise, first-stage problem from rest, "
                       f"seeds {seeds[0]}..{seeds[-1]}, one tank per solve, rtol {rtol:g}"}
    for precision, ws in (("mixed", 4), ("fp64", 8)):
        ms, its, byts = [], [], []
        for seed in seeds:
            pr = wl.bar(seed, 1024, 33)
            plan = pmgw.Plan([1024], [33], [pr["L"]], precision=precision)
            dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                         device="cuda")
            plan.set_geometry(dev(pr["h"]), dev(pr["eta_old"]), dev(pr["eta_new"]))
            b, p = dev(pr["b"]), plan.field()
            info = pmgw.poisson_solve(plan, b, p, rtol=rtol, maxit=300)
            pmgw.profile_start(plan, reps)
            for _ in range(reps):
                p.zero_()
                pmgw.poisson_solve(plan, b, p, rtol=rtol, maxit=300, sync=False)
            n, tot, _ = pmgw.profile_read(plan)
            pmgw.profile_start(plan, 0)
            ms.append(tot / max(n, 1))
            its.append(info[0][0])
            byts.append(solve_bytes(1024, 33, info[0][0], ws))
        t = float(np.mean(ms)) * 1e-3
        alg = float(np.mean(byts))
        out[precision] = {"value": 1.0 / t, "unit": "solves/s", "mean_launch_ms": 1e3 * t,
                          "launch_ms_per_seed": ms, "iters": its,
                          "roofline": {"bound": "hbm", "achieved": alg / t / 1e9,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": alg / t / 1e9 / HBM_PEAK_GBS,
                                       "alg_bytes_per_launch": alg}}
    out["mixed_speedup"] = out["fp64"]["mean_launch_ms"] / out["mixed"]["mean_launch_ms"]
    return out


# ----------------------------------------------------------------------------- 3D tank
def run_tank3d(nx=64, ny=64, nz=17, reps=3, rtol=1e-10):
    """A 3D tank (x, y periodic Fourier, sigma Chebyshev; float64): the manufactured problem on a
    sloped bed under a moving wavy surface, solved from zero; mean of `reps` solves timed with
    events on the plan's stream."""
    import torch

    from paper_2406_00991_amd import pmgw
    from paper_2406_00991_amd import workloads as wl
    pr = wl.manufactured3d(nx, ny, nz)
    plan = pmgw.Plan3([nx], [ny], [nz], [pr["Lx"]], [pr["Ly"]])
    dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                 device="cuda")
    plan.set_geometry(dev(pr["h"]), dev(pr["eta_old"]), dev(1.05 * pr["eta_new"]))
    b = dev(pr["b"])
    _, info = plan.solve(b, rtol=rtol)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        plan.solve(b, plan.field(), rtol=rtol)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"workload": f"3D tank {nx}x{ny}x{nz}, sloped bed, moving surface, float64, rtol {rtol:g}",
            "value": 1e3 / ms, "unit": "solves/s", "mean_solve_ms": ms, "iters": info[0][0],
            "relres": info[0][2], "cus_used": 1}


def run_stokes_layer(precision, warmup=2, rtol=1e-10):
    """The oscillatory boundary layer (linearised model, no-slip bed, 64 x 33, filters off): one
    wave period of RK4 steps after `warmup` steps, timed like the headline, and the near-bed
    velocity against the closed-form Stokes layer at the end."""
    import torch

    from paper_2406_00991_amd import pmgw
    from paper_2406_00991_amd import workloads as wl
    t = wl.stokes_layer()
    opts = pmgw.default_opts(nu_visc=t["nu"], filt_fx=1.0, filt_fz=1.0, linear=1, no_slip=1)
    steps = int(round(t["T"] / t["dt"]))
    T = Tank(t, precision, 5 * (steps + warmup), opts)
    for _ in range(warmup):
        T.step(t["dt"], rtol)
    torch.cuda.synchronize()
    T.pmgw.profile_start(T.plan, 5 * steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        T.step(t["dt"], rtol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, tot_ms, _ = T.pmgw.profile_read(T.plan)
    T.pmgw.profile_start(T.plan, 0)
    infos = T.infos(5 * warmup, 5 * steps)
    ue, _, _ = t["exact"]((warmup + steps) * t["dt"])
    near = t["zeta"][:, 0] < 6 * t["delta1"]
    u = T.u.cpu().numpy().reshape(t["nz"], t["nx"])
    return {"value": 5 * steps / wall, "unit": "solves/s", "ms_per_step": 1e3 * wall / steps,
            "steps": steps, "mean_launch_ms": tot_ms / max(launches, 1),
            "mean_iters": float(np.mean([i["iters"] for i in infos])),
            "status": sorted({i["status"] for i in infos}),
            "closed_form_err": float(np.abs(u[near] - ue[near]).max() / t["U0m"])}


def run_bar_flume(steps=12, warmup=2, rtol=1e-10, guess=4, correct=0):
    """The submerged-bar flume (1024 x 33, float64: on this bed the float32 cycle is near its
    stability edge; zones of one wavelength, stream-function wave
    H = 0.02 m, T = 2.02 s ramped in from still water, as the experiment starts): `steps` RK4
    steps after `warmup`, each followed by the target evaluation and the relaxation; solves/s
    over the whole stepping. These first steps have near-zero right-hand sides and take about
    twice the FGMRES iterations of the developed flow."""
    import torch

    from paper_2406_00991_amd import pmgw
    from paper_2406_00991_amd import workloads as wl
    fl = wl.bar_flume()
    T = Tank(fl, "fp64", 5 * (steps + warmup),
             pmgw.default_opts(guess_steps=guess, guess_correct=correct))
    dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                 device="cuda")
    r, S, coef = dev(fl["r"]), dev(fl["S"]), dev(fl["coef"])
    ut, wt, et = T.plan.field(), T.plan.field(), torch.zeros_like(T.eta)
    mass0 = float(T.eta.sum())

    def step(n):
        T.step(fl["dt"], rtol)
        t = (n + 1) * fl["dt"]
        pmgw.stream_target(T.plan, coef, fl["nmodes"], t, wl.ramp_in(t, fl["T"]), S, ut, wt, et)
        pmgw.relax(T.plan, r, ut, wt, et, T.u, T.w, T.eta)

    for n in range(warmup):
        step(n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(warmup, warmup + steps):
        step(n)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = T.infos(5 * warmup, 5 * steps)
    return {"workload": "submerged-bar flume, Nx=1024 x Nz=33, L = 10 incident wavelengths "
                        "(37.4 m), depth 0.4 m to 0.1 m over the bar, generation and absorption "
                        "zones of one wavelength, stream-function wave H=0.02 m, T=2.02 s "
                        "ramped in over two periods from still water, float64, rtol 1e-10, steps "
                        f"{warmup + 1}..{warmup + steps} from rest, relaxation after each step; "
                        f"initial guess opts.guess_steps {guess}, guess_correct {correct}",
            "value": 5 * steps / wall, "unit": "solves/s", "ms_per_step": 1e3 * wall / steps,
            "mean_iters": float(np.mean([i["iters"] for i in infos])),
            "max_iters": int(max(i["iters"] for i in infos)),
            "status": sorted({i["status"] for i in infos}),
            "mean_eta_change": (float(T.eta.sum()) - mass0) / fl["nx"]}


# ----------------------------------------------------------------------------- oracle timing
def _cores():
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def _oracle_stages(wave, budget_s):
    """The oracle's RK stages with its p-multigrid FGMRES solve (warm-started, 1e-10) from the
    bench's initial state, for about budget_s seconds: (stages done, seconds)."""
    from oracle import krylov
    from oracle import lserk
    from oracle import operator as op
    from oracle import pmg

    def solve(b, g_old, g_new, p0):
        H = pmg.Hierarchy(b.shape[1], b.shape[0] - 1, g_old, g_new, pmg.PmgOptions())
        return krylov.fgmres(lambda v: op.apply(v, g_old, g_new), b, H, x0=p0, rtol=1e-10)[0]

    s = lserk.State.rest_registers(wave["u"], wave["w"], wave["eta"])
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        lserk.stage(n % 5 + 1, wave["dt"], wave["h"], wave["L"], s, solve)
        n += 1
    return n, time.perf_counter() - t0


def _dense_solve_s(nx, nz):
    """Definition mode: seconds for one dense LU solve of the manufactured problem's operator
    (assembly excluded), the median of 3 after one warm-up."""
    from oracle import operator as op
    from paper_2406_00991_amd import workloads as wl
    import scipy.linalg as sla
    pr = wl.manufactured(nx, nz)
    g = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    A = op.assemble(nx, nz - 1, g, g)
    b = pr["b"].ravel()
    ts = []
    for _ in range(4):
        t0 = time.perf_counter()
        sla.lu_solve(sla.lu_factor(A), b)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts[1:]))


def cpu_baseline(wave, budget_s=12.0, budget_1t_s=6.0):
    """The oracle as it stands, on the host's cores (BLAS threads pinned to the core count with
    threadpoolctl; the FFTs are single-threaded): its RK stage with the p-multigrid FGMRES solve,
    from the same initial state, for about budget_s seconds. Beside it: the same with one BLAS
    thread, and the definition mode (dense LU) at 32 x 9 and 256 x 17."""
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = _cores()
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                       "")
    except OSError:
        pass
    with threadpool_limits(limits=cores):
        n, el = _oracle_stages(wave, budget_s)
        lu_c1 = _dense_solve_s(32, 9)
        lu_c2 = _dense_solve_s(256, 17)
    with threadpool_limits(limits=1):
        n1, el1 = _oracle_stages(wave, budget_1t_s)
    blas = sorted({f"{d.get('internal_api')}" for d in threadpool_info()})
    return dict(value=n / el, unit="solves/s", cores=cores, kind="oracle",
                sample=f"the first {n} RK stages (one pressure solve each) of the "
                       f"{wave['nx']}x{wave['nz']} Stokes-wave run, NumPy/SciPy float64, "
                       f"{el:.1f} s",
                cpu=cpu, blas=blas,
                one_thread={"value": n1 / el1, "unit": "solves/s",
                            "sample": f"the first {n1} RK stages, {el1:.1f} s, 1 BLAS thread"},
                dense_lu_s={"32x9": lu_c1, "256x17": lu_c2})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-tank batched solve reported beside the headline")
    ap.add_argument("--no-bar", action="store_true",
                    help="skip the 1024 x 33 bar solves reported beside the headline")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3D tank solve reported beside the headline")
    ap.add_argument("--guess-steps", type=int, default=4,
                    help="opts.guess_steps of the stepping plans: each stage's solve starts from "
                         "that stage's pressure extrapolated over this many previous steps "
                         "(0: from the previous stage's pressure)")
    ap.add_argument("--guess-correct", type=int, default=1,
                    help="opts.guess_correct of the stepping plans (with --guess-steps): add the "
                         "previous stage's extrapolation error to the extrapolation")
    ap.add_argument("--no-prev", action="store_true",
                    help="skip the stepping with each solve started from the previous stage's "
                         "pressure (reported beside the headline)")
    ap.add_argument("--no-flume", action="store_true",
                    help="skip the submerged-bar flume stepping reported beside the headline")
    ap.add_argument("--no-layer", action="store_true",
                    help="skip the oscillatory boundary-layer stepping reported beside the "
                         "headline")
    ap.add_argument("--calibrate-mib", type=int, default=0,
                    help="first run an elementwise negation of a float64 buffer of this size "
                         "(reads and writes it once), the known-traffic kernel that scales the "
                         "HBM counters of a profiled run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); tanks would shard across "
              "GPUs without communication", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2406_00991_amd import workloads as wl
    torch.cuda.set_device(0)
    if args.calibrate_mib > 0:
        src = torch.ones(args.calibrate_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    wave = wl.stokes_wave(256, 17)
    rtol = 1e-10
    gs = args.guess_steps
    gc = args.guess_correct if gs else 0
    res = {"mixed": run_precision(wave, "mixed", args.steps, args.warmup, rtol, gs, gc)}
    print(f"# mixed: {args.steps} steps in {res['mixed']['wall']:.3f} s", file=sys.stderr,
          flush=True)
    if not args.no_fp64:
        res["fp64"] = run_precision(wave, "fp64", args.steps, args.warmup, rtol, gs, gc)
        print(f"# fp64: {args.steps} steps in {res['fp64']['wall']:.3f} s", file=sys.stderr,
              flush=True)
    if gs and not args.no_prev:
        res["mixed_prev"] = run_precision(wave, "mixed", args.steps, args.warmup, rtol, 0)
        print(f"# mixed, previous-stage start: {args.steps} steps in "
              f"{res['mixed_prev']['wall']:.3f} s", file=sys.stderr, flush=True)
    mix = res["mixed"]
    nx, nz = wave["nx"], wave["nz"]
    solves = 5 * args.steps
    t_launch = mix["solve_ms"] * 1e-3
    # the mean of every timed solve's algorithmic bytes at its own iteration count
    byts = float(np.mean([solve_bytes(nx, nz, k, 4) for k in mix["iters_each"]]))
    flops = solve_flops(nx, nz, mix["iters"])
    achieved = byts / t_launch / 1e9
    # the mixed plan's 256 x 17 tank runs the solve kernel with the LDS-resident V-cycle
    kname = "k_solve<float,17,res>"
    out = {
        "metric": "Poisson solves/s at rel. residual 1e-10 (mixed float32 V-cycle / float64 "
                  "FGMRES), one per RK stage",
        "value": solves / mix["wall"],
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
        "config": {"workload": "RK4 time stepping of a second-order Stokes wave, Nx=256 x Nz=17, "
                               "flat bed h=1, L=2pi, kh=1, H/L=0.05, CFL 0.5, one tank, five "
                               "pressure solves per step, each to rel. residual 1e-10",
                   "precision": "mixed", "rtol": rtol, "dt": wave["dt"],
                   "initial_guess": (f"each stage's pressure extrapolated over its previous {gs} "
                                     "steps (opts.guess_steps)"
                                     + (", plus the previous stage's extrapolation error "
                                        "(opts.guess_correct)" if gc else "") if gs else
                                     "the previous stage's pressure")},
        "solve": {"launches": mix["launches"], "mean_launch_ms": mix["solve_ms"],
                  "max_launch_ms": mix["max_ms"], "mean_iters": mix["iters"],
                  "max_iters": mix["max_iters"], "max_relres": mix["relres"],
                  "status": mix["status"],
                  "share_of_step": mix["solve_ms"] * solves / (1e3 * mix["wall"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic(kname, "mixed"),
                     "kernel": "k_solve<float, 17, 256, false, true> (FGMRES with the "
                               "LDS-resident float32 V-cycle, one workgroup per tank)",
                     "alg_bytes_per_launch": byts, "launch_ms": mix["solve_ms"],
                     "flops_per_launch": flops,
                     "fp32_tflops": flops / t_launch / 1e12,
                     "fp32_frac_of_one_cu": flops / t_launch / 1e12 / (FP32_PEAK_TFLOPS / 256),
                     "cus_used": 1},
    }
    if "fp64" in res:
        f64 = res["fp64"]
        rd = lambda k: float(np.abs(mix[k] - f64[k]).max() / np.abs(f64[k]).max())
        out["fp64"] = {"value": solves / f64["wall"], "unit": "solves/s",
                       "ms_per_step": 1e3 * f64["wall"] / args.steps,
                       "mean_launch_ms": f64["solve_ms"], "mean_iters": f64["iters"],
                       "max_relres": f64["relres"], "status": f64["status"],
                       "mixed_speedup": f64["wall"] / mix["wall"]}
        out["mixed_vs_fp64_final_state"] = {k: rd(k) for k in ("u", "w", "eta", "p")}
    if "mixed_prev" in res:
        mp = res["mixed_prev"]
        rp = lambda k: float(np.abs(mix[k] - mp[k]).max() / np.abs(mp[k]).max())
        out["previous_stage_start"] = {
            "value": solves / mp["wall"], "unit": "solves/s",
            "ms_per_step": 1e3 * mp["wall"] / args.steps, "mean_launch_ms": mp["solve_ms"],
            "mean_iters": mp["iters"], "max_relres": mp["relres"], "status": mp["status"],
            "final_state_vs_headline": {k: rp(k) for k in ("u", "w", "eta", "p")}}
    if not args.no_batch:
        out["batched"] = run_batch(0, 512, 5, rtol)
        print(f"# batch: {out['batched']['value']:.0f} tank-solves/s", file=sys.stderr, flush=True)
    if not args.no_bar:
        out["bar"] = run_bar([0, 1, 2, 3, 4], 5, rtol)
        print(f"# bar: mixed {out['bar']['mixed']['value']:.0f} solves/s, fp64 "
              f"{out['bar']['fp64']['value']:.0f} solves/s", file=sys.stderr, flush=True)
    if not args.no_3d:
        out["tank3d"] = run_tank3d()
        print(f"# 3D tank: {out['tank3d']['value']:.1f} solves/s", file=sys.stderr, flush=True)
    if not args.no_layer:
        out["stokes_layer"] = {
            "workload": "oscillatory wave boundary layer: linearised model, no-slip bed, "
                        "Nx=64 x Nz=33, depth 0.1 m, H=0.02 m, kh=0.6725, nu=1e-6, 40 steps "
                        "per period, filters off, one tank, rtol 1e-10; closed_form_err = max "
                        "|u - u_Stokes-layer| / U_0m within 6 delta_1 of the bed",
            "fp64": run_stokes_layer("fp64"), "mixed": run_stokes_layer("mixed")}
        print(f"# boundary layer: fp64 {out['stokes_layer']['fp64']['value']:.0f} solves/s, "
              f"mixed {out['stokes_layer']['mixed']['value']:.0f} solves/s", file=sys.stderr,
              flush=True)
    if not args.no_flume:
        out["bar_flume"] = run_bar_flume(correct=gc)
        print(f"# bar flume: {out['bar_flume']['value']:.1f} solves/s", file=sys.stderr,
              flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wave)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

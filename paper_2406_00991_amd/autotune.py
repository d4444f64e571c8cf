"""Workgroup-size tuning of the batched solve.

The solve kernel runs one workgroup per tank. Fewer threads per workgroup make each tank slower
but let two workgroups share a CU (the kernel's register and LDS use allow one 256-thread or two
128-thread workgroups per CU), which pays off when a batch has more tanks than CUs. `tune` times
one batched solve of the caller's own problems for each candidate size on the device and keeps
the fastest; results are cached in a JSON file keyed by the batch's (Nx, Nz) histogram, the
precision and the device name.

The timing runs the library's solve (no work is skipped); the problems' geometry and right-hand
sides are the caller's, so the choice reflects their iteration counts too.
"""
import hashlib
import json
import os

from . import pmgw

CANDIDATES = (256, 128, 64)


def default_cache():
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2406_00991_amd",
                        "autotune.json")


def _key(nx, nz, precision, device_name):
    hist = {}
    for a, b in zip(nx, nz):
        hist[f"{a}x{b}"] = hist.get(f"{a}x{b}", 0) + 1
    blob = json.dumps(dict(hist=sorted(hist.items()), precision=precision, device=device_name),
                      sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()[:24]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(nx, nz, L, h, eta_old, eta_new, b, precision="mixed", rtol=1e-10, reps=2,
         candidates=CANDIDATES, cache=None, opts_kw=None):
    """Return (threads, timings) for a batch; h, eta_old, eta_new, b are packed device tensors
    as for Plan.set_geometry and poisson_solve. Timings are ms per batched solve (None when read
    from the cache)."""
    import torch
    cache = cache or default_cache()
    key = _key(nx, nz, precision, torch.cuda.get_device_name())
    store = _load(cache)
    if key in store:
        return int(store[key]["threads"]), None
    timings = {}
    for thr in candidates:
        plan = pmgw.Plan(nx, nz, L, precision=precision,
                         opts=pmgw.default_opts(threads=thr, **(opts_kw or {})))
        plan.set_geometry(h, eta_old, eta_new)
        p = plan.field()
        pmgw.poisson_solve(plan, b, p, rtol=rtol, maxit=200, sync=False)   # warm-up
        torch.cuda.synchronize()
        pmgw.profile_start(plan, reps)
        for _ in range(reps):
            p.zero_()
            pmgw.poisson_solve(plan, b, p, rtol=rtol, maxit=200, sync=False)
        n, tot, _ = pmgw.profile_read(plan)
        pmgw.profile_start(plan, 0)
        timings[thr] = tot / max(n, 1)
        del plan
    best = min(timings, key=timings.get)
    store[key] = dict(threads=int(best), timings_ms={str(k): v for k, v in timings.items()})
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(store, f, indent=1)
    os.replace(tmp, cache)
    return int(best), timings

"""Per-class launch tuning of the batched solve.

A batch runs one solve launch per finest-level class (3, 5, 9, 17, 33 rows), mixed-precision
classes split into the tanks whose V-cycle stays in LDS and the rest, and the launches run
concurrently, so the batch takes as long as its slowest launch, and the launches share the CUs.
Each class has its own candidate configurations:

- workgroup size 512, 256 or 128 threads with the V-cycle's fields in global memory (512 runs two
  wavefronts per SIMD for one wide tank; 128 lets two workgroups share a CU);
- for mixed-precision classes of at most 17 rows, the LDS-resident cycle (256 threads).

`tune` times the caller's own batch (its geometry and right-hand sides, one solve call per
repetition, no work skipped) and searches class by class, heaviest class first, keeping the
other classes at their current choice (one coordinate-descent pass). The result is the pair of
per-class option arrays (class_threads, class_resident) for pmgw_opts, cached in a JSON file
keyed by the batch's (Nx, Nz) histogram, the precision and the device name.
"""
import hashlib
import json
import os

from . import pmgw

THREADS = (512, 256, 128)


def default_cache():
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2406_00991_amd",
                        "autotune.json")


def _key(nx, nz, precision, device_name):
    hist = {}
    for a, b in zip(nx, nz):
        hist[f"{a}x{b}"] = hist.get(f"{a}x{b}", 0) + 1
    blob = json.dumps(dict(hist=sorted(hist.items()), precision=precision, device=device_name,
                           version=2), sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()[:24]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def candidates(rows, precision):
    """(threads, class_resident) pairs tried for a class with `rows` finest-level rows."""
    out = [(t, 2) for t in THREADS]
    if precision == "mixed" and rows <= 17:
        out.insert(0, (256, 1))
    return out


def time_batch(nx, nz, L, h, eta_old, eta_new, b, precision, opts, rtol=1e-10, reps=2):
    """Mean ms of one batched solve from zero (plan-stream events around each call)."""
    import torch
    plan = pmgw.Plan(nx, nz, L, precision=precision, opts=opts)
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
    return tot / max(n, 1)


def tune(nx, nz, L, h, eta_old, eta_new, b, precision="mixed", rtol=1e-10, reps=2, cache=None,
         opts_kw=None):
    """Return (choice, log) for a batch; h, eta_old, eta_new, b are packed device tensors as for
    Plan.set_geometry and poisson_solve. choice = {"class_threads": [5], "class_resident": [5]}
    (class order 3, 5, 9, 17, 33 rows; 0 = library default); log = list of
    (rows, threads, class_resident, ms) for every timed configuration, None when the choice
    came from the cache. cache=False disables the cache."""
    import torch
    key = _key(nx, nz, precision, torch.cuda.get_device_name())
    path = None if cache is False else (cache or default_cache())
    store = _load(path) if path else {}
    if key in store:
        return {k: list(store[key][k]) for k in ("class_threads", "class_resident")}, None
    ct, cr = [0] * 5, [0] * 5
    present = sorted({int(z) for z in nz}, reverse=True)
    log = []

    def run():
        o = pmgw.default_opts(class_threads=ct, class_resident=cr, **(opts_kw or {}))
        return time_batch(nx, nz, L, h, eta_old, eta_new, b, precision, o, rtol, reps)

    for rows in present:
        c = pmgw.CLASS_ROWS.index(rows)
        best = None
        for thr, res in candidates(rows, precision):
            ct[c], cr[c] = thr, res
            ms = run()
            log.append((rows, thr, res, ms))
            if best is None or ms < best[0]:
                best = (ms, thr, res)
        ct[c], cr[c] = best[1], best[2]
    choice = {"class_threads": ct, "class_resident": cr}
    if path:
        store[key] = dict(choice, log=log)
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(store, f, indent=1)
        os.replace(tmp, path)
    return choice, log

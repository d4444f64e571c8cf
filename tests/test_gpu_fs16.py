"""GPU parity of the float64 rows of 256 points, which run through the 16 x 16 register transform
(one 16-lane group per packed row pair, as many groups per round as the workgroup's FFT buffer
holds), against the CPU oracle.

The workgroup size sets the rounds: 256 threads fit the 9 row pairs of a 17-row level in one
round; 128 threads take two rounds, 64 threads three; 512 threads run the same code within 128
registers per lane. Row counts 3, 5, 9 and 17 give 2, 3, 5 and 9 pairs, each with a last pair
of one real row; 33 rows keep the radix-4 path. Bars as in test_gpu_poisson.py: apply 1e-12 of
max |A_oracle p|, float64 V-cycle 1e-12 relative, and the mixed-precision solve delta <= 1e-10.
The solves run with the bed-line step: on these sloped beds the plain smoother stalls at 9 rows
(the oracle's FGMRES too: relres 2.7e-11 after 100 iterations, against 10 with the step).
"""
import numpy as np
import pytest

from oracle import krylov
from oracle import operator as op
from oracle import pmg
from paper_2406_00991_amd import workloads as wl

from test_gpu_poisson import download, geoms, make_plan, mixed_geometry, upload2d

pytestmark = pytest.mark.gpu

ROWS = (3, 5, 9, 17, 33)
_REF = {}   # oracle solutions by row count, shared by the workgroup sizes


def problems():
    out = []
    for k, nz in enumerate(ROWS):
        p = mixed_geometry(wl.manufactured_sloped(256, nz), shift=0.1 * k)
        p["rnd"] = np.random.default_rng(40 + nz).standard_normal((nz, 256))
        out.append(p)
    return out


@pytest.mark.parametrize("threads", [64, 128, 256, 512])
def test_apply_and_vcycle_256_columns(threads):
    probs = problems()
    plan = make_plan(probs, "fp64", threads=threads)
    AP = download(plan, plan.apply(upload2d(probs, "rnd")))
    Z = download(plan, plan.vcycle(upload2d(probs, "b")))
    for pr, got_a, got_z in zip(probs, AP, Z):
        go, gn = geoms(pr)
        ref = op.apply(pr["rnd"], go, gn)
        ea = np.abs(got_a - ref).max() / np.abs(ref).max()
        H = pmg.Hierarchy(pr["nx"], pr["nz"] - 1, go, gn, pmg.PmgOptions())
        rz = H(pr["b"])
        ez = np.linalg.norm(got_z - rz) / np.linalg.norm(rz)
        print(f"threads {threads} 256x{pr['nz']}: apply {ea:.2e} vcycle {ez:.2e}", flush=True)
        assert ea <= 1e-12
        assert ez <= 1e-12


@pytest.mark.parametrize("threads", [64, 128, 256])
def test_mixed_solve_256_columns(threads):
    probs = [p for p in problems() if p["nz"] in (9, 17)]
    plan = make_plan(probs, "mixed", threads=threads, bed_line=1)
    P, info = plan.solve(upload2d(probs, "b"), rtol=1e-11, maxit=100)
    assert all(rec[1] == 0 for rec in info), info
    for pr, got in zip(probs, download(plan, P)):
        if pr["nz"] not in _REF:
            # the oracle's FGMRES with the bed-line cycle, run to its rounding floor (relres
            # ~5e-12 at 256 columns: the evaluation of b - A p, not the solution, limits it)
            go, gn = geoms(pr)
            H = pmg.Hierarchy(pr["nx"], pr["nz"] - 1, go, gn, pmg.PmgOptions(bed_line=True))
            _REF[pr["nz"]], _ = krylov.fgmres(lambda v: op.apply(v, go, gn), pr["b"], H,
                                              rtol=1e-14, restart=40, maxit=40)
        ref = _REF[pr["nz"]]
        delta = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"threads {threads} 256x{pr['nz']}: solve delta {delta:.2e}", flush=True)
        assert delta <= 1e-10

"""3D tanks (x, y periodic Fourier, sigma Chebyshev) on the GPU against the 3D oracle
(`oracle/operator3d.py`, `oracle/pmg3d.py`): the operator and the V-cycle at 1e-12 (float64,
fixed linear maps), the solve against the oracle's dense solution and against the closed-form
harmonic field."""
import math

import numpy as np
import pytest

from oracle import krylov
from oracle import operator3d as op3
from oracle import pmg
from oracle import pmg3d
from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _tank(nx, ny, nz, seed, move=True, Lx=2 * math.pi, Ly=3.0):
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * Lx / nx
    y = np.arange(ny) * Ly / ny
    X, Y = np.meshgrid(x, y)
    h = 1.0 - 0.1 * np.sin(X) * np.cos(2 * math.pi * Y / Ly) + 0.05 * np.cos(2 * math.pi * Y / Ly)
    eo = 0.04 * np.cos(X + 0.3) * np.cos(2 * math.pi * Y / Ly)
    en = eo * 1.1 + (0.01 * np.sin(2 * math.pi * Y / Ly) if move else 0.0)
    return dict(nx=nx, ny=ny, nz=nz, Lx=Lx, Ly=Ly, h=h, eta_old=eo, eta_new=en,
                b=rng.standard_normal((nz, ny, nx)))


def _m3(nx, ny, nz):
    pr = wl.manufactured3d(nx, ny, nz)
    return pr


CASES = {
    "manufactured_16x16x9": lambda: [_m3(16, 16, 9)],
    "rect_32x8x5": lambda: [_tank(32, 8, 5, 1)],
    "two_tanks": lambda: [_tank(16, 8, 9, 2), _tank(8, 16, 17, 3, Lx=4.0, Ly=2 * math.pi)],
}


def _plan(probs, **kw):
    import torch

    from paper_2406_00991_amd import pmgw
    plan = pmgw.Plan3([p["nx"] for p in probs], [p["ny"] for p in probs], [p["nz"] for p in probs],
                      [p["Lx"] for p in probs], [p["Ly"] for p in probs],
                      opts=pmgw.default_opts(**kw))
    cat = lambda key: torch.tensor(np.concatenate([np.asarray(p[key]).ravel() for p in probs]),
                                   dtype=torch.float64, device="cuda")
    plan.set_geometry(cat("h"), cat("eta_old"), cat("eta_new"))
    return plan, cat


def _geoms(p):
    return (op3.Geometry3(p["h"], p["eta_old"], p["Lx"], p["Ly"]),
            op3.Geometry3(p["h"], p["eta_new"], p["Lx"], p["Ly"]))


@pytest.mark.parametrize("case", sorted(CASES))
def test_apply3_parity(case):
    probs = CASES[case]()
    plan, cat = _plan(probs)
    out = plan.apply(cat("b"))
    for p, got in zip(probs, plan.split3d(out)):
        ref = op3.apply(p["b"], *_geoms(p))
        err = np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"{case} {p['nx']}x{p['ny']}x{p['nz']}: apply max rel err {err:.2e}", flush=True)
        assert err <= 1e-12


@pytest.mark.parametrize("case", sorted(CASES))
def test_vcycle3_parity(case):
    probs = CASES[case]()
    plan, cat = _plan(probs)
    out = plan.vcycle(cat("b"))
    for p, got in zip(probs, plan.split3d(out)):
        go, gn = _geoms(p)
        ref = pmg3d.Hierarchy3(p["nx"], p["ny"], p["nz"] - 1, go, gn)(p["b"])
        err = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"{case} {p['nx']}x{p['ny']}x{p['nz']}: vcycle rel err {err:.2e}", flush=True)
        assert err <= 1e-12


@pytest.mark.parametrize("case", sorted(CASES))
def test_solve3_parity(case):
    """FGMRES with the 3D V-cycle to 1e-12 (or 10 x the oracle's floor): status OK and within
    that of the oracle's dense solution."""
    probs = CASES[case]()
    plan, cat = _plan(probs)
    refs = [op3.solve_dense(p["b"], *_geoms(p)) for p in probs]
    floor = max(op3.relres(r, p["b"], *_geoms(p)) for r, p in zip(refs, probs))
    rtol = max(1e-12, 10 * floor)
    x, info = plan.solve(cat("b"), rtol=rtol, maxit=60)
    for p, got, inf, ref in zip(probs, plan.split3d(x), info, refs):
        d = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"{case} {p['nx']}x{p['ny']}x{p['nz']}: iters {inf[0]}, relres {inf[2]:.1e}, "
              f"delta {d:.2e} (floor {floor:.1e})", flush=True)
        assert inf[1] == 0 and inf[2] <= rtol and inf[0] <= 15
        assert d <= max(1e-11, 100 * floor)


def test_solve3_reproduces_the_harmonic_field():
    """16 x 16 x 17 manufactured problem: the solve reaches 1e-12 and the closed form within the
    discretisation error the oracle's dense solve has (3.8e-12 measured there)."""
    probs = [_m3(16, 16, 17)]
    plan, cat = _plan(probs)
    x, info = plan.solve(cat("b"), rtol=1e-12, maxit=60)
    got = plan.split3d(x)[0].cpu().numpy()
    err = np.abs(got - probs[0]["exact"]).max() / np.abs(probs[0]["exact"]).max()
    print(f"manufactured 16x16x17: iters {info[0][0]}, closed-form err {err:.2e}", flush=True)
    assert info[0][1] == 0 and err <= 1e-10


def test_solve3_64x32x17_against_oracle_fgmres():
    """A larger tank, beyond the dense solve: the GPU solve at 1e-12 against the oracle's
    p-multigrid FGMRES at 1e-12 (both from zero), within 1e-10; iteration counts printed."""
    probs = [_tank(64, 32, 17, 7)]
    p = probs[0]
    go, gn = _geoms(p)
    plan, cat = _plan(probs)
    x, info = plan.solve(cat("b"), rtol=1e-12, maxit=60)
    ref, inf = krylov.fgmres(lambda v: op3.apply(v, go, gn), p["b"],
                             pmg3d.Hierarchy3(p["nx"], p["ny"], p["nz"] - 1, go, gn), rtol=1e-12)
    d = np.linalg.norm(plan.split3d(x)[0].cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"64x32x17: GPU iters {info[0][0]} relres {info[0][2]:.1e}; oracle iters {inf['iters']} "
          f"relres {inf['relres']:.1e}; delta {d:.2e}", flush=True)
    assert info[0][1] == 0 and inf["converged"]
    assert d <= 1e-10

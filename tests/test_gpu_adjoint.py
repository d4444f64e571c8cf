"""GPU parity of the adjoint Poisson path (C ABI through the binding) against the CPU oracle.

- pmgw_adjoint_apply against the oracle's matrix-free transpose (itself pinned to the dense
  transpose): <= 1e-12 relative, float64.
- pmgw_adjoint_vcycle is the transpose of pmg_vcycle: <M a, b> = <a, M^T b> to 1e-12 relative in
  float64 plans (both are fixed linear maps), 1e-4 in mixed plans (float32 cycles).
- pmgw_adjoint_solve against the oracle's dense transposed LU: delta <= 1e-10 relative (solves
  stop at 1e-12 relative residual; the operator's condition number is ~1e3-1e4 here).
"""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import operator as op
from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def mixed_geometry(p, shift=0.3, scale=1.2):
    q = dict(p)
    x = np.arange(p["nx"]) * p["L"] / p["nx"]
    q["eta_new"] = p["eta_old"] * scale + 0.01 * np.cos(2 * math.pi * x / p["L"] + shift) * np.mean(p["h"])
    return q


CASES = {
    "c1_32x9": lambda: [wl.manufactured(32, 9)],
    "sloped_32x17_mixedgeo": lambda: [mixed_geometry(wl.manufactured_sloped(32, 17))],
    "batch_uneven": lambda: [mixed_geometry(wl.manufactured_sloped(64, 9)), wl.manufactured(16, 5),
                             mixed_geometry(wl.manufactured(128, 17), 1.0, 0.9)],
}


def make(problems, precision):
    from paper_2406_00991_amd import pmgw
    torch = _torch()
    plan = pmgw.Plan([p["nx"] for p in problems], [p["nz"] for p in problems],
                     [p["L"] for p in problems], precision=precision)
    cat = lambda key: torch.tensor(np.concatenate([p[key] for p in problems]),
                                   dtype=torch.float64, device="cuda")
    plan.set_geometry(cat("h"), cat("eta_old"), cat("eta_new"))
    return pmgw, plan


def rand(problems, seed):
    torch = _torch()
    rng = np.random.default_rng(seed)
    arrs = [rng.standard_normal((p["nz"], p["nx"])) for p in problems]
    return arrs, torch.tensor(np.concatenate([a.ravel() for a in arrs]), dtype=torch.float64,
                              device="cuda")


def geoms(p):
    return op.Geometry(p["h"], p["eta_old"], p["L"]), op.Geometry(p["h"], p["eta_new"], p["L"])


@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_apply_parity(case):
    probs = CASES[case]()
    pmgw, plan = make(probs, "fp64")
    lams, lam = rand(probs, 1)
    out = plan.field()
    pmgw.adjoint_apply(plan, lam, out)
    for p, l, got in zip(probs, lams, plan.split2d(out)):
        want = adj.apply_T(l, *geoms(p))
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-4)])
@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_vcycle_is_transpose(case, precision, tol):
    probs = CASES[case]()
    pmgw, plan = make(probs, precision)
    _, a = rand(probs, 2)
    _, b = rand(probs, 3)
    Ma, MTb = plan.field(), plan.field()
    pmgw.pmg_vcycle(plan, a, Ma)
    pmgw.adjoint_vcycle(plan, b, MTb)
    for x, y, u, v in zip(plan.split2d(Ma), plan.split2d(b), plan.split2d(a), plan.split2d(MTb)):
        lhs = float((x * y).sum())
        rhs = float((u * v).sum())
        assert abs(lhs - rhs) <= tol * max(abs(lhs), float(x.abs().sum() * y.abs().max()) * 1e-3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_solve_parity(case, precision):
    probs = CASES[case]()
    pmgw, plan = make(probs, precision)
    gs, g = rand(probs, 4)
    lam = plan.field()
    info = pmgw.adjoint_solve(plan, g, lam, rtol=1e-12, maxit=200)
    for p, gi, got, inf in zip(probs, gs, plan.split2d(lam), info):
        assert inf[1] == 0 and inf[2] <= 1e-12
        want = adj.solve_T_dense(gi, *geoms(p))
        got = got.cpu().numpy()
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_adjoint_solve_full_size_stokes():
    """The 256 x 17 Stokes-wave geometry with distinct old and new surfaces, mixed precision."""
    pr = mixed_geometry(wl.stokes_rest_problem(256, 17), 0.7, 1.1)
    pmgw, plan = make([pr], "mixed")
    gs, g = rand([pr], 5)
    lam = plan.field()
    info = pmgw.adjoint_solve(plan, g, lam, rtol=5e-12, maxit=200)
    assert info[0][1] == 0
    want = adj.solve_T_dense(gs[0], *geoms(pr))
    got = plan.split2d(lam)[0].cpu().numpy()
    assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(want)

"""poisson_solve_noalloc (geometry and solve in the library's static scratch array) against the
workspace path, pmgw_set_geometry + poisson_solve on a bound workspace, through the C ABI.

Both paths run the same kernels on the same inputs, so the solutions must agree to the float64
parity bar of the solve tests (here they are expected to be identical). Two calls in a row share
the device's one scratch array: the second with a smaller tank (so it reads tables and vectors that
the first call left behind at other offsets), then the first plan again (its tables were
overwritten and must be copied back in)."""
import numpy as np
import pytest

from oracle import operator as op
from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64, device="cuda")


def _workspace_solution(pr, precision, rtol):
    from paper_2406_00991_amd import pmgw
    plan = pmgw.Plan([pr["nx"]], [pr["nz"]], [pr["L"]], precision=precision)
    plan.set_geometry(_dev(pr["h"]), _dev(pr["eta_old"]), _dev(pr["eta_new"]))
    p, info = plan.solve(_dev(pr["b"]), rtol=rtol, maxit=200)
    return p.cpu().numpy(), info


def _noalloc_solution(plan, pr, rtol):
    from paper_2406_00991_amd import pmgw
    p = plan.field()
    info = pmgw.poisson_solve_noalloc(plan, _dev(pr["h"]), _dev(pr["eta_old"]),
                                      _dev(pr["eta_new"]), _dev(pr["b"]), p, rtol=rtol, maxit=200)
    return p.cpu().numpy(), info


def _check(pr, got, ginfo, ref, rinfo, rtol):
    delta = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    g = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    gn = op.Geometry(pr["h"], pr["eta_new"], pr["L"])
    rr = op.relres(got.reshape(pr["nz"], pr["nx"]), pr["b"], g, gn)
    print(f"{pr['nx']}x{pr['nz']}: iters {ginfo[0][0]} vs {rinfo[0][0]}, delta {delta:.2e}, "
          f"relres (oracle operator) {rr:.2e}", flush=True)
    assert ginfo[0][1] == 0 and rinfo[0][1] == 0
    assert ginfo[0][0] == rinfo[0][0]
    assert delta <= 1e-12
    assert rr <= 10 * rtol


def test_noalloc_matches_workspace_path_on_two_calls_in_a_row():
    from paper_2406_00991_amd import pmgw
    big = wl.stokes_rest_problem(256, 17)
    small = wl.manufactured_sloped(32, 9)
    pb = pmgw.Plan([big["nx"]], [big["nz"]], [big["L"]], precision="mixed", allocate=False)
    ps = pmgw.Plan([small["nx"]], [small["nz"]], [small["L"]], precision="fp64", allocate=False)
    assert pb.ws is None and ps.ws is None
    cases = [(pb, big, "mixed", 1e-10), (ps, small, "fp64", 1e-12), (pb, big, "mixed", 1e-10)]
    for plan, pr, prec, rtol in cases:
        ref, rinfo = _workspace_solution(pr, prec, rtol)
        got, ginfo = _noalloc_solution(plan, pr, rtol)
        _check(pr, got, ginfo, ref, rinfo, rtol)


def test_noalloc_batch_and_oversize_plan():
    """A small multi-class batch (its classes run one after another) matches the workspace path
    tank by tank; a plan larger than the array is refused before anything is launched."""
    import torch

    from paper_2406_00991_amd import pmgw
    tanks = wl.batch(2, 6, nx_choices=(32, 64), nz_choices=(9, 17))
    cat = lambda key: torch.tensor(np.concatenate([np.asarray(t[key]).ravel() for t in tanks]),
                                   dtype=torch.float64, device="cuda")
    args = [[t["nx"] for t in tanks], [t["nz"] for t in tanks], [t["L"] for t in tanks]]
    ref_plan = pmgw.Plan(*args, precision="mixed")
    ref_plan.set_geometry(cat("h"), cat("eta_old"), cat("eta_new"))
    ref, rinfo = ref_plan.solve(cat("b"), rtol=1e-10, maxit=200)
    plan = pmgw.Plan(*args, precision="mixed", allocate=False)
    got = plan.field()
    ginfo = pmgw.poisson_solve_noalloc(plan, cat("h"), cat("eta_old"), cat("eta_new"), cat("b"),
                                       got, rtol=1e-10, maxit=200)
    for a, b_, ia, ib in zip(plan.split2d(got), plan.split2d(ref), ginfo, rinfo):
        a, b_ = a.cpu().numpy(), b_.cpu().numpy()
        assert ia[1] == 0 and ib[1] == 0 and ia[0] == ib[0]
        assert np.linalg.norm(a - b_) / np.linalg.norm(b_) <= 1e-12
    huge = pmgw.Plan([1024, 1024], [33, 33], [10.0, 10.0], precision="fp64", allocate=False)
    assert huge.workspace_bytes > 48 << 20
    z1, z2 = torch.zeros(huge.n1d, dtype=torch.float64, device="cuda"), huge.field()
    with pytest.raises(pmgw.PmgwError) as ei:
        pmgw.poisson_solve_noalloc(huge, z1, z1, z1, z2, huge.field())
    assert ei.value.code == pmgw.EWORKSPACE

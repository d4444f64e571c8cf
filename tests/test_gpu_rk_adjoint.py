"""GPU parity of the discrete adjoint of the time stepping (rk4_stage_adjoint, the checkpointed
reverse sweep and the autograd Function) against the CPU oracle and finite differences.

- One reverse stage against the oracle's (dense-LU solves): the GPU recomputes the stage's
  pressure and solves the adjoint system iteratively to 1e-13, so the input adjoints and the
  depth gradient agree to 1e-9 relative (max norm).
- The depth gradient of a surface probe after whole steps against the oracle's: 1e-8 relative,
  over 2 steps (checkpoint 1) and over 10 steps of a 32 x 9 sloped-bed wave with checkpoints
  every 3 steps (segments of 3, 3, 3 and 1 steps).
- The 256 x 17 Stokes wave, 100 steps, probe at x = 0.75 L, checkpoints every 10 steps, float64:
  the adjoint gradient through torch.autograd against central differences (step 1e-6) of the GPU
  forward run in ALL 256 depth components, computed as one batched plan of 512 tanks (each tank
  one perturbed depth h +- 1e-6 e_i, stepped together), solves at 1e-12 (above this grid's
  rounding floor of ~4e-13). The bound is stated and measured in the test.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import lserk
from oracle import spectral as sp
from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("u", "w", "eta", "Ku", "Kw", "Keta")


def _torch():
    import torch
    return torch


def sloped(nx, nz, amp=0.05, steep=0.03):
    wv = dict(wl.stokes_wave(nx, nz, steep=steep))
    wv["h"] = wv["h"] + amp * np.sin(sp.x_nodes(nx, wv["L"]))
    return wv


def random_stage_input(wv, seed):
    rng = np.random.default_rng(seed)
    nz, nx = wv["u"].shape
    su = np.abs(wv["u"]).max()
    st = lserk.State.rest_registers(wv["u"], wv["w"], wv["eta"])
    st.Ku = 0.1 * su * rng.standard_normal((nz, nx))
    st.Kw = 0.1 * su * rng.standard_normal((nz, nx))
    st.Keta = 0.01 * rng.standard_normal(nx)
    bar = dict(u=rng.standard_normal((nz, nx)), w=rng.standard_normal((nz, nx)),
               eta=rng.standard_normal(nx), Ku=rng.standard_normal((nz, nx)),
               Kw=rng.standard_normal((nz, nx)), Keta=rng.standard_normal(nx))
    return st, bar


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run_stage_adjoint(tanks, k, precision="fp64"):
    from paper_2406_00991_amd import pmgw
    torch = _torch()
    plan = pmgw.Plan([t["wv"]["nx"] for t in tanks], [t["wv"]["nz"] for t in tanks],
                     [t["wv"]["L"] for t in tanks], precision=precision)
    dev = lambda arrs: torch.tensor(np.concatenate([np.asarray(a).ravel() for a in arrs]),
                                    dtype=torch.float64, device="cuda")
    h = dev([t["wv"]["h"] for t in tanks])
    st = {q: dev([getattr(t["st"], q) for t in tanks]) for q in KEYS}
    bar = {q: dev([t["bar"][q] for t in tanks]) for q in KEYS}
    hbar = torch.zeros_like(h)
    pmgw.rk4_stage_adjoint(plan, k, min(t["wv"]["dt"] for t in tanks), h, st, bar, hbar,
                           rtol=1e-13, maxit=300)
    out = []
    for i in range(len(tanks)):
        got = {}
        for q in KEYS:
            parts = plan.split1d(bar[q]) if q in ("eta", "Keta") else plan.split2d(bar[q])
            got[q] = parts[i].cpu().numpy()
        got["h"] = plan.split1d(hbar)[i].cpu().numpy()
        out.append(got)
    return out


@pytest.mark.parametrize("k,nx,nz", [(1, 16, 9), (3, 16, 9), (2, 32, 17), (5, 64, 9)])
def test_stage_adjoint_parity(k, nx, nz):
    wv = sloped(nx, nz)
    st, bar = random_stage_input(wv, 20 + k)
    got = run_stage_adjoint([dict(wv=wv, st=st, bar=bar)], k)[0]
    t = adj.stage_tape(k, wv["dt"], wv["h"], wv["L"], st)
    ref, href = adj.stage_T(t, bar, wv["h"], wv["L"])
    for q in KEYS:
        assert relerr(got[q], ref[q]) <= 1e-9, q
    assert relerr(got["h"], href) <= 1e-9


def test_stage_adjoint_batched_uneven():
    tanks = []
    for i, (nx, nz) in enumerate([(32, 9), (16, 5), (64, 17)]):
        wv = sloped(nx, nz, amp=0.03 + 0.01 * i)
        st, bar = random_stage_input(wv, 40 + i)
        tanks.append(dict(wv=wv, st=st, bar=bar))
    dt = min(t["wv"]["dt"] for t in tanks)
    got = run_stage_adjoint(tanks, 4)
    for t, g in zip(tanks, got):
        wv = t["wv"]
        tp = adj.stage_tape(4, dt, wv["h"], wv["L"], t["st"])
        ref, href = adj.stage_T(tp, t["bar"], wv["h"], wv["L"])
        for q in KEYS:
            assert relerr(g[q], ref[q]) <= 1e-9, q
        assert relerr(g["h"], href) <= 1e-9


def _plan_state(wv, precision="fp64"):
    from paper_2406_00991_amd import autograd as ag
    from paper_2406_00991_amd import pmgw
    torch = _torch()
    plan = pmgw.Plan([wv["nx"]], [wv["nz"]], [wv["L"]], precision=precision)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                 device="cuda")
    st0 = ag.initial_state(dev(wv["u"]), dev(wv["w"]), dev(wv["eta"]))
    return plan, dev(wv["h"]), st0, dev


def test_probe_gradient_matches_oracle():
    from paper_2406_00991_amd import autograd as ag
    torch = _torch()
    wv = sloped(16, 9)
    nsteps, probe = 2, 12
    plan, h, st0, dev = _plan_state(wv)
    geta = torch.zeros(16, dtype=torch.float64, device="cuda")
    geta[probe] = 1.0
    hbar, _ = ag.gradient(plan, h, st0, wv["dt"], nsteps, dict(eta=geta), checkpoint=1,
                          rtol=1e-13)
    ref = adj.probe_gradient(wv["h"], wv["L"], dict(u=wv["u"], w=wv["w"], eta=wv["eta"]),
                             wv["dt"], nsteps, probe)
    assert relerr(hbar.cpu().numpy(), ref) <= 1e-8


def test_probe_gradient_matches_oracle_ten_steps_checkpoint_3():
    """32 x 9, sloped bed, 10 steps with checkpoints every 3 steps (the last segment is one step):
    the checkpointed GPU sweep against the oracle's discrete adjoint, 1e-8 relative."""
    from paper_2406_00991_amd import autograd as ag
    torch = _torch()
    wv = sloped(32, 9)
    nsteps, probe = 10, 24
    plan, h, st0, dev = _plan_state(wv)
    geta = torch.zeros(32, dtype=torch.float64, device="cuda")
    geta[probe] = 1.0
    hbar, _ = ag.gradient(plan, h, st0, wv["dt"], nsteps, dict(eta=geta), checkpoint=3,
                          rtol=1e-13)
    ref = adj.probe_gradient(wv["h"], wv["L"], dict(u=wv["u"], w=wv["w"], eta=wv["eta"]),
                             wv["dt"], nsteps, probe)
    err = relerr(hbar.cpu().numpy(), ref)
    print(f"32x9, 10 steps, checkpoint 3: gradient rel err vs oracle {err:.2e}", flush=True)
    assert err <= 1e-8


def test_autograd_full_size_against_finite_differences():
    """Gradient of eta at x = 0.75 L after 100 steps of the 256 x 17 Stokes wave w.r.t. the 256
    nodal depths, through torch.autograd with checkpoints every 10 steps."""
    from paper_2406_00991_amd import autograd as ag
    torch = _torch()
    wv = wl.stokes_wave(256, 17)
    nsteps, probe = 100, 192
    plan, h, st0, dev = _plan_state(wv)
    hv = h.clone().requires_grad_(True)
    u, w, eta = ag.Rk4Steps.apply(hv, st0["u"], st0["w"], st0["eta"], plan, wv["dt"], nsteps,
                                  10, 1e-12)
    J = eta[probe]
    J.backward()
    g = hv.grad.detach().cpu().numpy()
    assert np.isfinite(g).all() and np.abs(g).max() > 0

    # central differences in all 256 components: one plan of 512 tanks, tank 2i with depth
    # h + eps e_i and tank 2i + 1 with h - eps e_i, stepped together
    from paper_2406_00991_amd import pmgw
    eps, n = 1e-6, 256
    H = np.repeat(wv["h"][None, :], 2 * n, axis=0)
    H[0::2][np.arange(n), np.arange(n)] += eps
    H[1::2][np.arange(n), np.arange(n)] -= eps
    bplan = pmgw.Plan([256] * (2 * n), [17] * (2 * n), [wv["L"]] * (2 * n), precision="fp64")
    tile2 = lambda a: torch.tensor(np.tile(np.asarray(a).ravel(), 2 * n), dtype=torch.float64,
                                   device="cuda")
    st = ag.initial_state(tile2(wv["u"]), tile2(wv["w"]), tile2(wv["eta"]))
    hb = torch.tensor(H.ravel(), dtype=torch.float64, device="cuda")
    ag.run(bplan, hb, st, wv["dt"], nsteps, rtol=1e-12, checkpoint=10)
    eta_f = st["eta"].view(2 * n, 256)[:, probe].cpu().numpy()
    fd = (eta_f[0::2] - eta_f[1::2]) / (2 * eps)
    err = np.abs(fd - g)
    print(f"256x17, 100 steps: |FD - adjoint| max {err.max():.2e}, median {np.median(err):.2e}, "
          f"max|g| {np.abs(g).max():.2e}, worst component {int(err.argmax())}", flush=True)
    # truncation eps^2 ~ 1e-12; each J carries the solves' residual noise (~1e-12 relative),
    # divided by 2 eps: a few 1e-7 relative to the gradient's scale
    assert err.max() <= 1e-5 * np.abs(g).max()

"""RK time steps captured in a HIP graph (through torch.cuda.graph on the plan's stream) replay to
the same result as eager execution.

The library's launch sequence of a stage (kernels only; no memset or copy nodes) is captured
once for one full step (five stages) of a two-class batch, whose solves fork onto the plan's side
streams and join back inside the graph. The graph is replayed three times from the same initial
state, with eager work and synchronisations between the replays; every replay must equal the
eager step bit for bit (same kernels, same launch configuration, same inputs).
"""
import numpy as np
import pytest

from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_captured_step_replays_equal_eager():
    import torch

    from paper_2406_00991_amd import pmgw
    tanks = [wl.stokes_wave(64, 17, steep=0.03), wl.stokes_wave(32, 9, steep=0.02)]
    s = torch.cuda.Stream()
    plan = pmgw.Plan([t["nx"] for t in tanks], [t["nz"] for t in tanks], [t["L"] for t in tanks],
                     precision="mixed", stream=s)
    dev = lambda key: torch.tensor(np.concatenate([np.asarray(t[key]).ravel() for t in tanks]),
                                   dtype=torch.float64, device="cuda")
    h = dev("h")
    init = dict(u=dev("u"), w=dev("w"), eta=dev("eta"))
    dt = min(t["dt"] for t in tanks)

    def fresh(st):
        for k in ("u", "w", "eta"):
            st[k].copy_(init[k])
        for k in ("Ku", "Kw", "Keta", "p"):
            st[k].zero_()

    def make():
        return dict(u=torch.empty_like(init["u"]), w=torch.empty_like(init["w"]),
                    eta=torch.empty_like(init["eta"]), Ku=torch.empty_like(init["u"]),
                    Kw=torch.empty_like(init["u"]), Keta=torch.empty_like(init["eta"]),
                    p=torch.empty_like(init["u"]))

    def step(st):
        for k in range(1, 6):
            pmgw.rk4_stage(plan, k, dt, h, st["u"], st["w"], st["eta"], st["Ku"], st["Kw"],
                           st["Keta"], st["p"], rtol=1e-10, maxit=100)

    eager = make()
    with torch.cuda.stream(s):
        fresh(eager)
        step(eager)                    # also creates the plan's side streams before capture
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in eager.items()}

    st = make()
    with torch.cuda.stream(s):
        fresh(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step(st)
    for rep in range(3):
        with torch.cuda.stream(s):
            fresh(st)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("u", "w", "eta", "Ku", "Kw", "Keta", "p"):
            assert torch.equal(st[k], ref[k]), (rep, k)
        # eager work between replays
        with torch.cuda.stream(s):
            fresh(eager)
            step(eager)
        torch.cuda.synchronize()
        for k in ("u", "eta"):
            assert torch.equal(eager[k], ref[k])

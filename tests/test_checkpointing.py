"""Host logic of the checkpointed reverse sweep (paper_2406_00991_amd.autograd), on the CPU.

The library calls are replaced by the oracle's forward stage and reverse stage on CPU tensors, so
that only the ordering of the sweep is under test: checkpoints every C steps (C dividing the step
count or not), recomputation of each segment's stage inputs, the reverse order of the stage
adjoints, and a restart of the stage-pressure record (opts.guess_steps) before every sweep that
jumps back in time. The result must equal the oracle's gradient taken without checkpoints.
"""
import types

import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from oracle import lserk
from oracle import spectral as sp
from paper_2406_00991_amd import autograd as ag
from paper_2406_00991_amd import pmgw
from paper_2406_00991_amd import workloads as wl


class FakeLib:
    def __init__(self, nx, nz, L):
        self.nx, self.nz, self.L = nx, nz, L
        self.calls = []

    def _state(self, u, w, eta, Ku, Kw, Keta, p):
        r2 = lambda t: t.numpy().reshape(self.nz, self.nx).copy()
        return lserk.State(r2(u), r2(w), eta.numpy().copy(), r2(Ku), r2(Kw), Keta.numpy().copy(),
                           r2(p))

    fail_at = None        # (kind, call index) whose solve record reports NOCONV

    def _record(self, kind, info_dev, slots):
        """Write one OK solve record per slot (iters 3, status 0) into the info slice, as the
        library does; NOCONV at the call named by fail_at."""
        if info_dev is None:
            return
        n = sum(1 for c, _ in self.calls if c == kind)
        status = 1 if self.fail_at == (kind, n) else 0
        raw = info_dev.numpy().view(np.int32).reshape(-1, 4)
        assert raw.shape[0] == slots
        raw[:, 0] = 3
        raw[:, 1] = status
        info_dev.numpy().reshape(-1, 2)[:, 1] = 1e-13

    def rk4_stage(self, plan, k, dt, h, u, w, eta, Ku, Kw, Keta, p, rtol=0, maxit=0,
                  info_dev=None):
        self._record("f", info_dev, 1)
        s = self._state(u, w, eta, Ku, Kw, Keta, p)
        lserk.stage(k, dt, h.numpy(), self.L, s, lserk.dense_solver)
        for t, a in ((u, s.u), (w, s.w), (eta, s.eta), (Ku, s.Ku), (Kw, s.Kw), (Keta, s.Keta),
                     (p, s.p)):
            t.copy_(torch.from_numpy(np.ascontiguousarray(a).ravel()))
        self.calls.append(("f", k))

    def history_reset(self, plan):
        self.calls.append(("reset", None))

    def rk4_stage_adjoint(self, plan, k, dt, h, st, bar, hbar, rtol=0, maxit=0, info_dev=None):
        self._record("r", info_dev, 2)
        s = self._state(*(st[q] for q in ("u", "w", "eta", "Ku", "Kw", "Keta", "p")))
        tp = adj.stage_tape(k, dt, h.numpy(), self.L, s)
        b = {q: (bar[q].numpy().reshape(self.nz, self.nx) if q not in ("eta", "Keta")
                 else bar[q].numpy()) for q in bar}
        out, hb = adj.stage_T(tp, b, h.numpy(), self.L)
        for q in bar:
            bar[q].copy_(torch.from_numpy(np.ascontiguousarray(out[q]).ravel()))
        hbar += torch.from_numpy(hb)
        self.calls.append(("r", k))


PLAN = types.SimpleNamespace(ntanks=1, device="cpu")


def _patch(monkeypatch, fake):
    ns = types.SimpleNamespace(
        rk4_stage=fake.rk4_stage, rk4_stage_adjoint=fake.rk4_stage_adjoint,
        history_reset=fake.history_reset,
        info_buffer=lambda n, device=None: torch.zeros(2 * n, dtype=torch.float64),
        read_info=pmgw.read_info, OK=pmgw.OK, PmgwError=pmgw.PmgwError)
    monkeypatch.setattr(ag, "pmgw", ns)


@pytest.mark.parametrize("where", [("f", 4), ("f", 17), ("r", 6)])
def test_failed_solve_inside_the_sweep_raises(monkeypatch, where):
    """A solve record with a status other than OK, in the forward run, a segment's recompute or a
    reverse stage, makes the sweep raise instead of returning a gradient."""
    nx, nz, nsteps = 16, 5, 3
    wv = wl.stokes_wave(nx, nz, steep=0.02)
    fake = FakeLib(nx, nz, wv["L"])
    fake.fail_at = where
    _patch(monkeypatch, fake)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel().copy())
    st0 = ag.initial_state(t(wv["u"]), t(wv["w"]), t(wv["eta"]))
    geta = torch.zeros(nx, dtype=torch.float64)
    geta[3] = 1.0
    with pytest.raises(pmgw.PmgwError) as ei:
        ag.gradient(PLAN, t(wv["h"]), st0, wv["dt"], nsteps, dict(eta=geta), 2)
    assert ei.value.code == pmgw.NOCONV


@pytest.mark.parametrize("checkpoint", [1, 2, 3])
def test_checkpointed_sweep_equals_plain_gradient(monkeypatch, checkpoint):
    nx, nz, nsteps, probe = 16, 5, 3, 7
    wv = dict(wl.stokes_wave(nx, nz, steep=0.02))
    wv["h"] = wv["h"] + 0.03 * np.sin(sp.x_nodes(nx, wv["L"]))
    fake = FakeLib(nx, nz, wv["L"])
    _patch(monkeypatch, fake)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel().copy())
    st0 = ag.initial_state(t(wv["u"]), t(wv["w"]), t(wv["eta"]))
    geta = torch.zeros(nx, dtype=torch.float64)
    geta[probe] = 1.0
    hbar, _ = ag.gradient(PLAN, t(wv["h"]), st0, wv["dt"], nsteps, dict(eta=geta), checkpoint)
    ref = adj.probe_gradient(wv["h"], wv["L"], dict(u=wv["u"], w=wv["w"], eta=wv["eta"]),
                             wv["dt"], nsteps, probe)
    assert np.abs(hbar.numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    rev = [k for kind, k in fake.calls if kind == "r"]
    assert rev == [5, 4, 3, 2, 1] * nsteps
    fwd = sum(1 for kind, _ in fake.calls if kind == "f")
    assert fwd == 2 * 5 * nsteps          # the checkpointed run plus one recompute per segment
    # the stage-pressure record restarts before the forward run and before every recompute
    # (the recompute jumps back in time); each reset is followed by a stage-1 forward call
    kinds = [kind for kind, _ in fake.calls]
    resets = [i for i, kind in enumerate(kinds) if kind == "reset"]
    assert len(resets) == 1 + -(-nsteps // checkpoint)
    assert all(fake.calls[i + 1] == ("f", 1) for i in resets)

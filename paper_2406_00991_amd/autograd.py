"""Gradients through the time stepping with the library's discrete adjoint.

Every stage runs in the library (rk4_stage forward, rk4_stage_adjoint reverse); this module only
orders the calls and keeps checkpoints: the state at every `checkpoint`-th step is stored during
the forward run, and the reverse sweep recomputes the stage inputs of one segment at a time from
its checkpoint (memory: n_steps/checkpoint + 5*checkpoint states instead of 5*n_steps).

Every solve's outcome goes to a device info buffer that is read once per checkpoint segment; a
solve that ends with a status other than OK (not converged, NaN) raises PmgwError.

- `gradient(...)`: adjoint sweep for given adjoints of the final (u, w, eta); returns the
  gradient w.r.t. the depth h and the adjoints of the initial (u, w, eta).
- `Rk4Steps`: the same as a torch.autograd.Function of (h, u0, w0, eta0).
"""
import torch

from . import pmgw

KEYS = ("u", "w", "eta", "Ku", "Kw", "Keta")


def _clone(st):
    return {k: v.clone() for k, v in st.items()}


def initial_state(u0, w0, eta0):
    """Stage-1 input state from a velocity field and surface: K registers at zero, p at zero."""
    z = torch.zeros_like(u0)
    return dict(u=u0.clone(), w=w0.clone(), eta=eta0.clone(), Ku=z.clone(), Kw=z.clone(),
                Keta=torch.zeros_like(eta0), p=z.clone())


class _Infos:
    """Device records of the solves of one checkpoint segment (one per stage and tank; two per
    stage and tank for reverse stages: forward recompute, then adjoint). `check` reads them once
    per segment and raises on any status other than OK, so that a NOCONV or ENAN solve inside the
    stepping does not go unnoticed."""

    def __init__(self, plan, stages, per_stage):
        self.plan, self.per = plan, per_stage
        self.buf = pmgw.info_buffer(plan.ntanks * stages * per_stage,
                                    device=getattr(plan, "device", None))
        self.n = 0

    def next(self):
        w = 2 * self.plan.ntanks * self.per
        rec = self.buf[w * self.n: w * (self.n + 1)]
        self.n += 1
        return rec

    def check(self, what):
        if self.n == 0:
            return
        used = self.buf[: 2 * self.plan.ntanks * self.per * self.n]
        for i, r in enumerate(pmgw.read_info(used)):
            if r["status"] != pmgw.OK:
                raise pmgw.PmgwError(r["status"], f"{what}: solve record {i} "
                                                  f"(stage-call {i // (self.plan.ntanks * self.per)})"
                                                  f" has status {r['status']}, relres "
                                                  f"{r['relres']:.3e}")
        self.buf.zero_()
        self.n = 0


def stage(plan, k, dt, h, st, rtol, maxit=100, info=None):
    pmgw.rk4_stage(plan, k, dt, h, st["u"], st["w"], st["eta"], st["Ku"], st["Kw"],
                   st["Keta"], st["p"], rtol=rtol, maxit=maxit,
                   info_dev=info.next() if info is not None else None)


def run(plan, h, st, dt, nsteps, rtol=1e-12, checkpoint=None):
    """Advance st (in place) by nsteps; returns the list of checkpoints taken before steps
    0, C, 2C, ... when checkpoint = C is given. Every solve's status is checked once per
    segment of C steps (or once at the end); a failed solve raises PmgwError."""
    cps = []
    seg = checkpoint or nsteps
    infos = _Infos(plan, 5 * max(1, min(seg, nsteps)), 1)
    pmgw.history_reset(plan)        # a plan with guess_steps starts its pressure record afresh
    for n in range(nsteps):
        if checkpoint and n % checkpoint == 0:
            infos.check("forward stepping")
            cps.append(_clone(st))
        for k in range(1, 6):
            stage(plan, k, dt, h, st, rtol, info=infos)
    infos.check("forward stepping")
    return cps


def gradient(plan, h, st0, dt, nsteps, bar_final, checkpoint=10, rtol=1e-12):
    """Reverse sweep. bar_final: dict with the adjoints of the final u, w, eta (K registers of
    the final state get zero adjoints). Returns (hbar, bar) where bar holds the adjoints of the
    initial state's u, w, eta, Ku, Kw, Keta. Every forward, recompute and adjoint solve is
    checked once per checkpoint segment; a failed solve raises PmgwError."""
    st = _clone(st0)
    cps = run(plan, h, st, dt, nsteps, rtol, checkpoint)
    bar = {k: torch.zeros_like(st0[k]) for k in KEYS}
    for k in ("u", "w", "eta"):
        if bar_final.get(k) is not None:
            bar[k].copy_(bar_final[k])
    hbar = torch.zeros_like(h)
    fwd = _Infos(plan, 5 * checkpoint, 1)
    rev = _Infos(plan, 5 * checkpoint, 2)
    for c in range(len(cps) - 1, -1, -1):
        first = c * checkpoint
        last = min(nsteps, first + checkpoint)
        cur = _clone(cps[c])
        inputs = []
        pmgw.history_reset(plan)    # the recompute jumps back in time: no stale pressure record
        for _ in range(first, last):
            for k in range(1, 6):
                inputs.append((k, _clone(cur)))
                stage(plan, k, dt, h, cur, rtol, info=fwd)
        for k, sin in reversed(inputs):
            pmgw.rk4_stage_adjoint(plan, k, dt, h, sin, bar, hbar, rtol=rtol,
                                   info_dev=rev.next())
        fwd.check(f"segment {c} recompute")
        rev.check(f"segment {c} reverse stages")
    return hbar, bar


class Rk4Steps(torch.autograd.Function):
    """(u, w, eta) after nsteps time steps from (u0, w0, eta0) at rest registers, as a
    differentiable function of (h, u0, w0, eta0)."""

    @staticmethod
    def forward(ctx, h, u0, w0, eta0, plan, dt, nsteps, checkpoint=10, rtol=1e-12):
        st = initial_state(u0.detach(), w0.detach(), eta0.detach())
        ctx.save_for_backward(h.detach(), u0.detach(), w0.detach(), eta0.detach())
        ctx.cfg = (plan, dt, nsteps, checkpoint, rtol)
        run(plan, h.detach(), st, dt, nsteps, rtol)
        return st["u"], st["w"], st["eta"]

    @staticmethod
    def backward(ctx, gu, gw, geta):
        h, u0, w0, eta0 = ctx.saved_tensors
        plan, dt, nsteps, checkpoint, rtol = ctx.cfg
        st0 = initial_state(u0, w0, eta0)
        z2, z1 = torch.zeros_like(u0), torch.zeros_like(eta0)
        bar_final = dict(u=gu if gu is not None else z2, w=gw if gw is not None else z2,
                         eta=geta if geta is not None else z1)
        hbar, bar = gradient(plan, h, st0, dt, nsteps, bar_final, checkpoint, rtol)
        return hbar, bar["u"], bar["w"], bar["eta"], None, None, None, None, None

"""The extrapolated initial guess of rk4_stage (opts.guess_steps) through the C ABI.

- With rtol = 1 the solve returns its starting point (the initial residual is already below
  ||b||), so the pressure after the call is the guess itself: it must equal the polynomial
  extrapolation of that stage's recorded pressures, computed here from the values read back after
  each earlier call (degree 1 after two recorded steps, 2 after three, 3 after four).
- An out-of-order stage, a changed dt and pmgw_history_reset each restart the record: the next
  call starts from p as passed.
- With opts.guess_correct the guess is that extrapolation plus the previous call's extrapolation
  error (its result minus the extrapolation it started from), computed here the same way from
  the read-back values; after a restart the first extrapolated call has no previous
  extrapolation and starts from the plain one.
- Stepping the 256 x 17 Stokes wave with the guess reaches the same states as stepping without
  it (both solve every stage to 1e-10; measured difference <= 4e-12 relative), with fewer FGMRES
  iterations per solve (measured 2.0 instead of 4.7 once four steps are recorded, 1.4 with the
  correction).
"""
import numpy as np
import pytest

from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu


class Stepper:
    def __init__(self, wv, precision="fp64", **optkw):
        import torch
        from paper_2406_00991_amd import pmgw
        self.pmgw, self.wv = pmgw, wv
        self.plan = pmgw.Plan([wv["nx"]], [wv["nz"]], [wv["L"]], precision=precision,
                              opts=pmgw.default_opts(**optkw))
        dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64,
                                     device="cuda")
        self.h, self.u, self.w, self.eta = dev(wv["h"]), dev(wv["u"]), dev(wv["w"]), dev(wv["eta"])
        self.Ku, self.Kw = torch.zeros_like(self.u), torch.zeros_like(self.u)
        self.Keta, self.p = torch.zeros_like(self.eta), torch.zeros_like(self.u)
        self.info = pmgw.info_buffer(1)
        self.iters = []

    def stage(self, k, dt=None, rtol=1e-12):
        dt = self.wv["dt"] if dt is None else dt
        self.pmgw.rk4_stage(self.plan, k, dt, self.h, self.u, self.w, self.eta, self.Ku, self.Kw,
                            self.Keta, self.p, rtol=rtol, maxit=200, info_dev=self.info)
        rec = self.pmgw.read_info(self.info)[0]
        assert rec["status"] == 0
        self.iters.append(rec["iters"])
        return self.p.cpu().numpy().copy()


def _record(S, steps):
    P = {k: [] for k in range(1, 6)}
    for _ in range(steps):
        for k in range(1, 6):
            P[k].append(S.stage(k))
    return P


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("recorded,m", [(2, 3), (3, 3), (4, 4)])
def test_guess_is_the_extrapolation_of_the_record(recorded, m):
    S = Stepper(wl.stokes_wave(32, 9), guess_steps=m)
    P = _record(S, recorded)
    got = S.stage(1, rtol=1.0)
    assert S.iters[-1] == 0
    h = P[1]
    coef = {2: (2, -1), 3: (3, -3, 1), 4: (4, -6, 4, -1)}[min(recorded, m)]
    want = sum(c * h[-1 - i] for i, c in enumerate(coef))
    assert relerr(got, want) <= 1e-13


COEF = {2: (2, -1), 3: (3, -3, 1), 4: (4, -6, 4, -1)}


def extrap(h, c):
    """Polynomial extrapolation of the last c values of h one step ahead."""
    return sum(ci * h[-1 - i] for i, ci in enumerate(COEF[c]))


@pytest.mark.parametrize("m", [3, 4])
def test_corrected_guess(m):
    S = Stepper(wl.stokes_wave(32, 9), guess_steps=m, guess_correct=1)
    P = _record(S, 4)
    # stage 1 of step 5: its record holds steps 1..4; the previous call (stage 5 of step 4)
    # started from the extrapolation of steps 1..3 of stage 5 and returned P[5][-1]
    got = S.stage(1, rtol=1.0)
    assert S.iters[-1] == 0
    want = extrap(P[1], min(4, m)) + (P[5][-1] - extrap(P[5][:-1], min(3, m)))
    assert relerr(got, want) <= 1e-13
    # and stage 2 of step 5, whose previous call is the one above (its result is its guess)
    got2 = S.stage(2, rtol=1.0)
    want2 = extrap(P[2], min(4, m)) + (got - extrap(P[1], min(4, m)))
    assert relerr(got2, want2) <= 1e-13


def test_corrected_guess_after_restart():
    S = Stepper(wl.stokes_wave(32, 9), guess_steps=3, guess_correct=1)
    _record(S, 3)
    S.pmgw.history_reset(S.plan)
    P = _record(S, 2)
    # step 3: stage 1's record holds two steps; stage 5 of step 2 had one and started from p as
    # passed, so there is no extrapolation error to add
    got = S.stage(1, rtol=1.0)
    assert relerr(got, extrap(P[1], 2)) <= 1e-13


@pytest.mark.parametrize("breaker", ["out_of_order", "dt", "reset"])
def test_record_restarts(breaker):
    S = Stepper(wl.stokes_wave(32, 9), guess_steps=3)
    _record(S, 3)
    if breaker == "out_of_order":
        S.stage(3)                       # expected k = 1
        k_next = 4
    elif breaker == "dt":
        S.stage(1, dt=0.5 * S.wv["dt"])
        k_next = 2
    else:
        S.pmgw.history_reset(S.plan)
        k_next = 1
    before = S.p.cpu().numpy().copy()
    after = S.stage(k_next, rtol=1.0)    # no record: the solve starts from p as passed
    assert S.iters[-1] == 0
    assert np.array_equal(after, before)


@pytest.mark.parametrize("correct", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_guessed_stepping_matches_plain_stepping(precision, correct):
    wv = wl.stokes_wave(256, 17)
    A = Stepper(wv, precision)
    B = Stepper(wv, precision, guess_steps=4, guess_correct=correct)
    for _ in range(10):
        for k in range(1, 6):
            A.stage(k, rtol=1e-10)
            B.stage(k, rtol=1e-10)
    for name in ("u", "w", "eta", "p"):
        a, b = getattr(A, name).cpu().numpy(), getattr(B, name).cpu().numpy()
        assert relerr(b, a) <= 1e-9, name
    assert np.mean(B.iters[25:]) < np.mean(A.iters[25:]) - 1.0, (A.iters, B.iters)

"""Pins of the oracle's low-storage Runge-Kutta stage (paper Sec. 3.1-3.3, 3.6) against the
mathematics: Runge-Kutta order conditions, rest state, the divergence constraint the projection
enforces, and linear wave theory (dispersion relation, Sec. 5.3)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import lserk
from oracle import operator as op
from oracle import spectral as sp
from paper_2406_00991_amd import workloads as wl


def test_order_conditions_exact():
    a, b, c = lserk.butcher()
    s = len(b)
    Ac = [sum(a[i][j] * c[j] for j in range(s)) for i in range(s)]
    Ac2 = [sum(a[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)]
    AAc = [sum(a[i][j] * Ac[j] for j in range(s)) for i in range(s)]
    conds = [
        (sum(b), Fraction(1)),
        (sum(b[i] * c[i] for i in range(s)), Fraction(1, 2)),
        (sum(b[i] * c[i] ** 2 for i in range(s)), Fraction(1, 3)),
        (sum(b[i] * Ac[i] for i in range(s)), Fraction(1, 6)),
        (sum(b[i] * c[i] ** 3 for i in range(s)), Fraction(1, 4)),
        (sum(b[i] * c[i] * Ac[i] for i in range(s)), Fraction(1, 8)),
        (sum(b[i] * Ac2[i] for i in range(s)), Fraction(1, 12)),
        (sum(b[i] * AAc[i] for i in range(s)), Fraction(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-15
    # Carpenter-Kennedy's published abscissae
    assert abs(float(c[1]) - 1432997174477 / 9575080441755) < 1e-15


def test_fourth_order_on_linear_ode():
    lam = -1.0 + 2.0j
    def run(n):
        y, K, dt = 1.0 + 0j, 0j, 1.0 / n
        for _ in range(n):
            for a, b in zip(lserk.ALPHA, lserk.BETA):
                K = a * K + dt * lam * y
                y = y + b * K
        return abs(y - np.exp(lam))
    e1, e2 = run(20), run(40)
    assert 14.0 < e1 / e2 < 18.5


def test_still_water_stays_at_rest():
    nx, nz, L = 16, 9, 2 * math.pi
    h = 1.0 + 0.1 * np.cos(sp.x_nodes(nx, L))
    z = np.zeros((nz, nx))
    s = lserk.State.rest_registers(z, z, np.zeros(nx))
    lserk.step(0.05, h, L, s)
    assert np.abs(s.u).max() == 0 and np.abs(s.w).max() == 0 and np.abs(s.eta).max() == 0
    assert np.abs(s.p).max() == 0


def test_projection_enforces_divergence_and_bed_flux():
    wv = wl.stokes_wave(32, 9)
    h = wv["h"] + 0.05 * np.sin(sp.x_nodes(32, wv["L"]))
    s = lserk.State.rest_registers(wv["u"], wv["w"], wv["eta"])
    for d in lserk.step(wv["dt"], h, wv["L"], s):
        assert d["div"] < 1e-9 * max(d["div_ref"], 1.0)
        assert d["bed_flux"] < 1e-9


def _airy_run(nx, nz, dt_div=1, t_frac=1.0, amp=1e-6):
    wv = wl.airy_wave(nx, nz, amp=amp)
    s = lserk.State.rest_registers(wv["u"], wv["w"], wv["eta"])
    T = t_frac * wv["period"]
    n = int(math.ceil(T / wv["dt"])) * dt_div
    dt = T / n
    mass0 = s.eta.sum()
    for _ in range(n):
        lserk.step(dt, wv["h"], wv["L"], s)
    x = sp.x_nodes(nx, wv["L"])
    exact = amp * np.cos(wv["k"] * x - wv["omega"] * T)
    return s, exact, mass0, wv


def test_linear_wave_dispersion_and_mass():
    """A small-amplitude wave travels at the linear phase speed sqrt(g tanh(kh)/k): after a
    quarter period eta = a sin(kx); total mass is conserved."""
    s, exact, mass0, wv = _airy_run(16, 9, t_frac=0.25)
    err = np.abs(s.eta - exact).max() / wv["amp"]
    assert err < 2e-3
    assert abs(s.eta.sum() - mass0) < 1e-9 * wv["amp"] * 16
    # a wrong phase speed (e.g. shallow-water sqrt(gh)) would leave a much larger error
    x = sp.x_nodes(16, wv["L"])
    wrong = wv["amp"] * np.cos(x - math.sqrt(9.81) * 0.25 * wv["period"])
    assert np.abs(s.eta - wrong).max() / wv["amp"] > 0.1


def test_time_convergence_fourth_order():
    e = []
    for m in (1, 2):
        s, exact, _, wv = _airy_run(16, 9, dt_div=m, t_frac=0.25)
        e.append(s)
    ref, exact, _, wv = _airy_run(16, 9, dt_div=8, t_frac=0.25)
    e1 = np.abs(e[0].eta - ref.eta).max()
    e2 = np.abs(e[1].eta - ref.eta).max()
    assert e1 / e2 > 10.0

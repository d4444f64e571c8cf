"""Pins of the stream-function wave (Rienecker and Fenton's Fourier approximation) that the
flume workloads use as incident wave (paper Sec. 5, harmonic generation over a submerged bar).

- the paper's printed case (H, T, h -> L, kh; tests/golden/submerged_bar_wave.txt): the
  small-amplitude wavelength is the linear-dispersion one and equals the printed L;
- small steepness: the first and second surface harmonics are Stokes' first- and second-order
  amplitudes;
- between the collocation points the surface still satisfies the free-surface conditions,
  checked in a different form than the one solved: the kinematic condition as flow tangency
  W = U eta_X (eta_X from the surface's cosine series) and Bernoulli with velocities from
  finite differences of the stream function (so a wrong term in the analytic velocities fails);
- the two wave-speed definitions differ by the depth-mean Stokes drift to leading order.
"""
import math
import os

import numpy as np
import pytest

from paper_2406_00991_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "submerged_bar_wave.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_papers_case_wavelength():
    gv = _golden()
    tiny = wl.stream_function_wave(1e-6, gv["h"], period=gv["T"])
    assert abs(tiny["L"] - gv["L"]) < 5e-4
    assert abs(tiny["k"] * gv["h"] - gv["kh"]) < 5e-3
    om = 2 * math.pi / gv["T"]
    assert abs(om * om - wl.G * tiny["k"] * math.tanh(tiny["k"] * gv["h"])) < 1e-9 * om * om
    for cur in ("euler", "mass"):
        s = wl.stream_function_wave(gv["H"], gv["h"], period=gv["T"], current=cur)
        assert s["residual"] < 1e-12
        assert abs(s["T"] - gv["T"]) < 1e-12
        assert 0.0 < s["L"] / gv["L"] - 1.0 < 3e-3     # nonlinear dispersion lengthens the wave


def test_stokes_limit():
    h, k = 1.0, 1.0
    H = 0.002
    s = wl.stream_function_wave(H, h, length=2 * math.pi / k)
    kh = k * h
    e2 = k * H * H / 16 * math.cosh(kh) * (2 + math.cosh(2 * kh)) / math.sinh(kh) ** 3
    assert abs(s["E"][1] - H / 2) < 1e-3 * H / 2
    assert abs(s["E"][2] - e2) < 1e-2 * e2
    c_lin = math.sqrt(wl.G / k * math.tanh(kh))
    assert abs(s["c"] - c_lin) < 1e-4 * c_lin


def _surface(s, X):
    k, N = s["k"], s["N"]
    q = np.arange(N + 1)
    eta = np.cos(np.outer(X, q) * k) @ s["E"]
    eta_x = -(np.sin(np.outer(X, q) * k) * (q * k)) @ s["E"]
    return eta, eta_x


def _psi(s, X, zeta):
    k, h = s["k"], s["depth"]
    j = np.arange(1, s["N"] + 1)
    return -s["ubar"] * zeta + (np.sinh(np.outer(zeta, j) * k) / np.cosh(j * k * h)
                                * np.cos(np.outer(X, j) * k)) @ s["B"]


@pytest.mark.parametrize("H", [0.02, 0.12])
def test_surface_conditions_between_collocation_points(H):
    s = wl.stream_function_wave(H, 0.4, period=2.02, N=32)
    X = np.random.default_rng(0).uniform(0, s["L"] / 2, 200)
    eta, eta_x = _surface(s, X)
    zeta = s["depth"] + eta
    # the bed and the surface are the streamlines psi = 0 and psi = -Q
    assert np.abs(_psi(s, X, 0.0 * X)).max() < 1e-15

    assert np.abs(_psi(s, X, zeta) + s["Q"]).max() < 1e-9 * s["c"] * s["depth"]
    # velocities by central differences of psi (step 1e-5 m)
    d = 1e-5
    U = (_psi(s, X, zeta + d) - _psi(s, X, zeta - d)) / (2 * d)
    W = -(_psi(s, X + d, zeta) - _psi(s, X - d, zeta)) / (2 * d)
    # flow tangent to the surface, and Bernoulli
    assert np.abs(W - U * eta_x).max() < 1e-6 * s["c"]
    bern = 0.5 * (U * U + W * W) + wl.G * eta
    assert np.abs(bern - s["R"]).max() < 1e-6 * wl.G * H


def test_wave_speed_definitions_differ_by_stokes_drift():
    H, h, T = 0.01, 0.5, 2.0
    e = wl.stream_function_wave(H, h, period=T, current="euler")
    m = wl.stream_function_wave(H, h, length=e["L"], current="mass")
    drift = wl.G * H * H / (8 * e["c"] * h)          # depth-mean Stokes drift, E / (rho c h)
    assert abs((e["c"] - m["c"]) - drift) < 0.05 * drift

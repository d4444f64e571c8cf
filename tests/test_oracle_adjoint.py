"""Pins of the oracle's discrete adjoint.

- The matrix-free transpose equals the transpose of the dense assembled operator (Kronecker
  construction, independent of the matrix-free code).
- Every reverse step of the stage is checked at once by complex-step differentiation of the
  forward stage (derivative exact to rounding, no subtractive cancellation; the forward code is
  analytic because its solves are dense LU and its FFTs complex):
  <bar_out, d out> = <bar_in, d in> + <hbar, d h> for random directions.
- The probe gradient over whole steps against complex-step derivatives of single components and
  against central finite differences.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import lserk
from oracle import operator as op
from oracle import spectral as sp
from paper_2406_00991_amd import workloads as wl

EPS_CS = 1e-30


def _sloped_wave(nx=16, nz=9, amp=0.05, steep=0.03):
    wv = wl.stokes_wave(nx, nz, steep=steep)
    wv = dict(wv)
    wv["h"] = wv["h"] + amp * np.sin(sp.x_nodes(nx, wv["L"]))
    return wv


def test_apply_transpose_equals_dense_transpose():
    rng = np.random.default_rng(3)
    nx, M, L = 16, 8, 2 * math.pi
    x = sp.x_nodes(nx, L)
    h = 1.0 + 0.1 * np.sin(x)
    go = op.Geometry(h, 0.05 * np.cos(x), L)
    gn = op.Geometry(h, 0.04 * np.cos(x + 0.3), L)
    A = op.assemble(nx, M, go, gn)
    lam = rng.standard_normal((M + 1, nx))
    got = adj.apply_T(lam, go, gn)
    want = (A.T @ lam.ravel()).reshape(lam.shape)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    c = rng.standard_normal((M + 1, nx))
    sol = adj.solve_T_dense(c, go, gn)
    assert np.abs(adj.apply_T(sol, go, gn) - c).max() <= 1e-10 * np.abs(c).max()


def _stage_cs(k, dt, h, L, s, dirs, dh, wbar):
    """Complex-step directional derivative of <wbar, stage outputs>."""
    sc = lserk.State(*(getattr(s, f) + 1j * EPS_CS * dirs.get(f, 0.0)
                       for f in ("u", "w", "eta", "Ku", "Kw", "Keta", "p")))
    hc = h + 1j * EPS_CS * dh
    lserk.stage(k, dt, hc, L, sc, lserk.dense_solver)
    J = sum(np.sum(wbar[f] * getattr(sc, f)) for f in ("u", "w", "eta", "Ku", "Kw", "Keta"))
    return J.imag / EPS_CS


@pytest.mark.parametrize("k", [1, 3])
def test_stage_adjoint_against_complex_step(k):
    rng = np.random.default_rng(10 + k)
    wv = _sloped_wave()
    h, L, dt = wv["h"], wv["L"], wv["dt"]
    nz, nx = wv["u"].shape
    s = lserk.State.rest_registers(wv["u"], wv["w"], wv["eta"])
    scale_u = np.abs(wv["u"]).max()
    s.Ku = 0.1 * scale_u * rng.standard_normal((nz, nx))
    s.Kw = 0.1 * scale_u * rng.standard_normal((nz, nx))
    s.Keta = 0.01 * rng.standard_normal(nx)
    wbar = dict(u=rng.standard_normal((nz, nx)), w=rng.standard_normal((nz, nx)),
                eta=rng.standard_normal(nx), Ku=rng.standard_normal((nz, nx)),
                Kw=rng.standard_normal((nz, nx)), Keta=rng.standard_normal(nx))
    t = adj.stage_tape(k, dt, h, L, s)
    bar_in, hbar = adj.stage_T(t, wbar, h, L)
    # one direction per input at a time, so a wrong term cannot hide behind another
    for f in ("u", "w", "eta", "Ku", "Kw", "Keta", "h"):
        shape = (nx,) if f in ("eta", "Keta", "h") else (nz, nx)
        d = rng.standard_normal(shape)
        if f == "h":
            cs = _stage_cs(k, dt, h, L, s, {}, d, wbar)
            ad = np.sum(hbar * d)
        else:
            cs = _stage_cs(k, dt, h, L, s, {f: d}, 0.0, wbar)
            ad = np.sum(bar_in[f] * d)
        assert abs(ad - cs) <= 1e-9 * max(abs(cs), 1e-12), (f, ad, cs)


def test_probe_gradient_against_complex_step_and_fd():
    wv = _sloped_wave(16, 9)
    h, L, dt = wv["h"], wv["L"], wv["dt"]
    ic = dict(u=wv["u"], w=wv["w"], eta=wv["eta"])
    nsteps, probe = 2, 12
    g = adj.probe_gradient(h, L, ic, dt, nsteps, probe)
    assert np.abs(g).max() > 0
    for i in (0, 5, 12):
        e = np.zeros(len(h))
        e[i] = 1.0
        _, s = adj.run_forward(h + 1j * EPS_CS * e, L, ic, dt, nsteps)
        cs = s.eta[probe].imag / EPS_CS
        assert abs(g[i] - cs) <= 1e-9 * np.abs(g).max(), (i, g[i], cs)
    # central differences along a random direction (truncation ~ eps^2, rounding ~ 1e-16/eps)
    rng = np.random.default_rng(4)
    d = rng.standard_normal(len(h))
    eps = 1e-5
    _, sp_ = adj.run_forward(h + eps * d, L, ic, dt, nsteps)
    _, sm_ = adj.run_forward(h - eps * d, L, ic, dt, nsteps)
    fd = (sp_.eta[probe] - sm_.eta[probe]) / (2 * eps)
    assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), np.abs(g).max())

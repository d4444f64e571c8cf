"""Pins of the oracle's discrete Poisson operator and solves against closed forms.

Paper: sigma-metrics eq. 1_Scoef, transformed gradient of Sec. 2.1, mixed-stage problem eq. poissonp
with the boundary conditions eq. bcpd and eq. bcpdneu; linear wave theory of Sec. 5.3.
"""
import math

import numpy as np
import pytest

from oracle import operator as op
from oracle import spectral as sp
from paper_2406_00991_amd import workloads as wl


def _geoms(pr):
    return (op.Geometry(pr["h"], pr["eta_old"], pr["L"]),
            op.Geometry(pr["h"], pr["eta_new"], pr["L"]))


def test_dense_equals_matrix_free_mixed_geometry():
    nx, M, L = 16, 8, 5.0
    x = sp.x_nodes(nx, L)
    h = 1.0 + 0.2 * np.sin(2 * math.pi * x / L)
    go = op.Geometry(h, 0.05 * np.cos(2 * math.pi * x / L), L)
    gn = op.Geometry(h, 0.07 * np.cos(2 * math.pi * x / L + 0.3), L)
    A = op.assemble(nx, M, go, gn)
    P = np.random.default_rng(0).standard_normal((M + 1, nx))
    ref = op.apply(P, go, gn)
    assert np.allclose(A @ P.ravel(), ref.ravel(), atol=1e-12 * np.abs(ref).max())


def test_gradient_and_divergence_against_closed_forms():
    """Grad on geometry g returns the physical gradient at g's node positions; Div likewise."""
    nx, M, L = 48, 24, 2 * math.pi
    x = sp.x_nodes(nx, L)
    s = sp.cgl_sigma(M)
    h = 1.0 - 0.15 * np.sin(x)
    g = op.Geometry(h, 0.05 * np.cos(x), L)
    z = s[:, None] * g.d[None, :] - h[None, :]
    X = x[None, :]
    p = np.cos(X) * np.cosh(z + 1.0)
    Gx, Gz = op.grad(p, g, M)
    assert np.abs(Gx + np.sin(X) * np.cosh(z + 1.0)).max() < 1e-11
    assert np.abs(Gz - np.cos(X) * np.sinh(z + 1.0)).max() < 1e-11
    Fx, Fz = np.sin(X) * z, np.cos(X) * z * z        # div = cos x z + 2 z cos x
    dv = op.div(Fx, Fz, g, M)
    assert np.abs(dv - 3.0 * np.cos(X) * z).max() < 1e-11


def test_mixed_operator_annihilates_hydrostatic_field():
    """P = beta z + gamma sampled on the OLD grid: Grad^old P = (0, beta), so interior rows vanish,
    the bed row is -beta and the surface row is P itself; a field sampled on the wrong grid fails."""
    nx, M, L = 32, 8, 2 * math.pi
    x = sp.x_nodes(nx, L)
    s = sp.cgl_sigma(M)
    h = 1.0 - 0.1 * np.sin(x)
    go = op.Geometry(h, 0.05 * np.cos(x), L)
    gn = op.Geometry(h, 0.08 * np.cos(x + 0.4), L)
    beta, gamma = 1.7, 0.3
    P = beta * (s[:, None] * go.d[None, :] - h[None, :]) + gamma
    AP = op.apply(P, go, gn)
    assert np.abs(AP[1:M]).max() < 1e-12
    assert np.allclose(AP[M], -beta, atol=1e-12)
    assert np.allclose(AP[0], P[0], atol=0)
    Pn = beta * (s[:, None] * gn.d[None, :] - h[None, :]) + gamma
    assert np.abs(op.apply(Pn, go, gn)[1:M]).max() > 1e-3


def test_manufactured_spectral_convergence():
    """Flat bed, wavy surface, harmonic exact solution: the error decays spectrally in Nz."""
    errs = {}
    for nz in (5, 7, 9, 11):
        pr = wl.manufactured(32, nz)
        go, gn = _geoms(pr)
        errs[nz] = np.abs(op.solve_dense(pr["b"], go, gn) - pr["exact"]).max()
    assert errs[5] < 3e-4 and errs[7] < 1e-6 and errs[9] < 1e-9 and errs[11] < 1e-11
    assert errs[5] > 1e2 * errs[7] > 1e4 * errs[9]


def test_manufactured_sloped_bed_convergence():
    """Sloped bed: the bed row's h_x term and the metric terms are exercised."""
    errs = []
    for nz in (5, 9, 17):
        pr = wl.manufactured_sloped(32, nz)
        go, gn = _geoms(pr)
        errs.append(np.abs(op.solve_dense(pr["b"], go, gn) - pr["exact"]).max())
    assert errs[0] > 1e3 * errs[1] and errs[2] < 1e-10


def test_airy_linear_pressure():
    """Linear theory: the dynamic pressure of the from-rest stage on a flat geometry."""
    pr = wl.airy_pressure(16, 17, depth=1.0, mode=2)
    go, gn = _geoms(pr)
    P = op.solve_dense(pr["b"], go, gn)
    assert np.abs(P - pr["exact"]).max() < 1e-10 * np.abs(pr["exact"]).max()


def test_flat_geometry_decouples_into_modes():
    """With h = d constant the operator is diagonal in x-Fourier modes: the per-mode blocks with
    cbar = 1/d^2, ebar = 1/d solve the problem exactly."""
    nx, M, L, d = 16, 8, 3.0, 0.8
    g = op.Geometry(np.full(nx, d), np.zeros(nx), L)
    cbar, ebar = op.flat_coefficients(g, g)
    assert abs(cbar - 1 / d ** 2) < 1e-15 and abs(ebar - 1 / d) < 1e-15
    blocks = op.flat_mode_blocks(nx, M, L, cbar, ebar)
    b = np.random.default_rng(3).standard_normal((M + 1, nx))
    P1 = op.flat_mode_solve(b, blocks)
    P2 = op.solve_dense(b, g, g)
    assert np.abs(P1 - P2).max() < 1e-12 * np.abs(P2).max()


def test_relres_definition():
    pr = wl.manufactured(16, 5)
    go, gn = _geoms(pr)
    P = op.solve_dense(pr["b"], go, gn)
    assert op.relres(P, pr["b"], go, gn) < 1e-13
    assert abs(op.relres(np.zeros_like(P), pr["b"], go, gn) - 1.0) < 1e-15

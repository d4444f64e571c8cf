"""Pins of the 3D oracle (x, y Fourier x sigma Chebyshev; Sec. 2.1 with the y-terms, Sec. 3.4
in y, Alg. 1): each against something other than itself.

- the matrix-free operator equals its Kronecker-product assembly;
- with data independent of y (or of x) the 3D operator is the 2D oracle's operator, slab by
  slab (a dropped or mis-signed y-term, or a transposed axis, breaks it);
- a harmonic field with a closed form on a sloped bed under a wavy surface is reproduced with
  spectral convergence;
- the column-block formula equals the assembled matrix's diagonal blocks;
- on a flat geometry the V-cycle is the exact inverse; on a sloped, moving geometry FGMRES with
  it converges to the dense solution.
"""
import math

import numpy as np
import pytest

from oracle import krylov
from oracle import operator as op
from oracle import operator3d as op3
from oracle import pmg
from oracle import pmg3d
from paper_2406_00991_amd import workloads as wl


def _geoms(nx, ny, move=True):
    Lx, Ly = 2 * math.pi, 3.0
    x = np.arange(nx) * Lx / nx
    y = np.arange(ny) * Ly / ny
    X, Y = np.meshgrid(x, y)
    h = 1.0 - 0.12 * np.sin(X) * np.cos(2 * math.pi * Y / Ly) + 0.05 * np.cos(2 * math.pi * Y / Ly)
    eo = 0.04 * np.cos(X + 0.3) * np.cos(2 * math.pi * Y / Ly)
    en = eo * 1.1 + (0.01 * np.sin(2 * math.pi * Y / Ly) if move else 0.0)
    return op3.Geometry3(h, eo, Lx, Ly), op3.Geometry3(h, en, Lx, Ly)


def test_apply_equals_assembly():
    nx, ny, M = 8, 6, 4
    go, gn = _geoms(nx, ny)
    P = np.random.default_rng(1).standard_normal((M + 1, ny, nx))
    A = op3.assemble(nx, ny, M, go, gn)
    ref = (A @ P.ravel()).reshape(P.shape)
    assert np.abs(op3.apply(P, go, gn) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_y_invariant_data_is_the_2d_operator():
    nx, ny, M = 16, 4, 8
    L = 2 * math.pi
    x = np.arange(nx) * L / nx
    h = 1.0 - 0.1 * np.sin(x)
    eo, en = 0.05 * np.cos(x), 0.06 * np.cos(x + 0.2)
    P2 = np.random.default_rng(2).standard_normal((M + 1, nx))
    go3 = op3.Geometry3(np.tile(h, (ny, 1)), np.tile(eo, (ny, 1)), L, 1.7)
    gn3 = op3.Geometry3(np.tile(h, (ny, 1)), np.tile(en, (ny, 1)), L, 1.7)
    out3 = op3.apply(np.repeat(P2[:, None, :], ny, axis=1), go3, gn3)
    out2 = op.apply(P2, op.Geometry(h, eo, L), op.Geometry(h, en, L))
    for a in range(ny):
        assert np.abs(out3[:, a, :] - out2).max() <= 1e-12 * np.abs(out2).max()


def test_x_invariant_data_is_the_2d_operator_along_y():
    nx, ny, M = 4, 16, 8
    Ly = 2.5
    y = np.arange(ny) * Ly / ny
    h = 1.0 - 0.1 * np.sin(2 * math.pi * y / Ly)
    eo, en = 0.05 * np.cos(2 * math.pi * y / Ly), 0.06 * np.cos(2 * math.pi * y / Ly + 0.2)
    P2 = np.random.default_rng(3).standard_normal((M + 1, ny))
    go3 = op3.Geometry3(np.tile(h[:, None], (1, nx)), np.tile(eo[:, None], (1, nx)), 1.3, Ly)
    gn3 = op3.Geometry3(np.tile(h[:, None], (1, nx)), np.tile(en[:, None], (1, nx)), 1.3, Ly)
    out3 = op3.apply(np.repeat(P2[:, :, None], nx, axis=2), go3, gn3)
    out2 = op.apply(P2, op.Geometry(h, eo, Ly), op.Geometry(h, en, Ly))
    for c in range(nx):
        assert np.abs(out3[:, :, c] - out2).max() <= 1e-12 * np.abs(out2).max()


def test_manufactured_harmonic_field_converges_spectrally():
    errs = []
    for nh, nz in [(8, 5), (12, 9), (16, 13)]:
        pr = wl.manufactured3d(nh, nh, nz)
        g = op3.Geometry3(pr["h"], pr["eta_old"], pr["Lx"], pr["Ly"])
        P = op3.solve_dense(pr["b"], g, g)
        errs.append(np.abs(P - pr["exact"]).max() / np.abs(pr["exact"]).max())
    assert errs[0] > 1e-5 and errs[1] < 1e-7 and errs[2] < 1e-10, errs


def test_column_blocks_formula_equals_definition():
    nx, ny, M = 8, 4, 4
    go, gn = _geoms(nx, ny)
    B = pmg3d.column_blocks(nx, ny, M, go, gn)
    A = op3.assemble(nx, ny, M, go, gn)
    nh = nx * ny
    for a in range(ny):
        for c in range(nx):
            idx = np.arange(M + 1) * nh + a * nx + c
            blk = A[np.ix_(idx, idx)]
            assert np.abs(B[a, c] - blk).max() <= 1e-11 * np.abs(blk).max()


def test_vcycle_exact_on_flat_geometry():
    nx, ny, M = 8, 6, 8
    g = op3.Geometry3(np.full((ny, nx), 0.7), np.zeros((ny, nx)), 2.0, 1.5)
    H = pmg3d.Hierarchy3(nx, ny, M, g, g, pmg.PmgOptions(omega_m=1.0))
    f = np.random.default_rng(4).standard_normal((M + 1, ny, nx))
    ref = op3.solve_dense(f, g, g)
    assert np.abs(H(f) - ref).max() <= 1e-11 * np.abs(ref).max()


def test_fgmres_with_the_3d_cycle_reaches_the_dense_solution():
    nx, ny, M = 16, 8, 8
    go, gn = _geoms(nx, ny)
    f = np.random.default_rng(5).standard_normal((M + 1, ny, nx))
    H = pmg3d.Hierarchy3(nx, ny, M, go, gn)
    x, inf = krylov.fgmres(lambda v: op3.apply(v, go, gn), f, H, rtol=1e-12)
    ref = op3.solve_dense(f, go, gn)
    assert inf["converged"] and inf["iters"] <= 12
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)

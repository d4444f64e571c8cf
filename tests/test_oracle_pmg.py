"""Pins of the oracle's p-multigrid pieces (paper Sec. 4, Alg. 1) and of its Krylov solver."""
import math

import numpy as np
import pytest

from oracle import krylov
from oracle import operator as op
from oracle import pmg
from oracle import spectral as sp
from paper_2406_00991_amd import workloads as wl


def test_levels():
    assert pmg.level_orders(32) == [32, 16, 8, 4, 2]
    assert pmg.level_orders(2) == [2]


@pytest.mark.parametrize("Mf", [4, 8, 16, 32])
def test_transfers(Mf):
    Mc = Mf // 2
    R = pmg.restriction_matrix(Mf)
    P = pmg.prolongation_matrix(Mf)
    assert np.allclose(R @ P, np.eye(Mc + 1), atol=1e-13)
    sf, sc = sp.cgl_sigma(Mf), sp.cgl_sigma(Mc)
    for p in range(Mc + 1):
        assert np.abs(P @ sc ** p - sf ** p).max() < 1e-13       # interpolation is exact
        assert np.abs(R @ sf ** p - sc ** p).max() < 1e-13       # truncation keeps degree <= Mc
    # a fine-only mode (T_Mf) restricts to zero in the interior rows
    tM = np.cos(Mf * np.arccos(sp.cgl_xi(Mf)))
    assert np.abs((R @ tM)[1:Mc]).max() < 1e-13
    # coarse nodes are the even fine nodes
    assert np.allclose(P[::2], np.eye(Mc + 1), atol=1e-14)


def _sloped_geoms(nx, L=2 * math.pi):
    x = sp.x_nodes(nx, L)
    h = 1.0 - 0.15 * np.sin(2 * math.pi * x / L)
    go = op.Geometry(h, 0.05 * np.cos(2 * math.pi * x / L), L)
    gn = op.Geometry(h, 0.06 * np.cos(2 * math.pi * x / L + 0.2), L)
    return go, gn


@pytest.mark.parametrize("M", [2, 8])
def test_column_blocks_formula_equals_definition(M):
    nx = 16
    go, gn = _sloped_geoms(nx)
    A = op.assemble(nx, M, go, gn)
    assert np.allclose(pmg.column_blocks(nx, M, go, gn), pmg.column_blocks_from_dense(A, nx, M),
                       atol=1e-10 * np.abs(A).max())


def test_dxx_diagonal():
    nx, L = 16, 3.0
    D = sp.dx_matrix(nx, L)
    assert np.allclose(np.diag(D @ D), pmg.dxx_diagonal(nx, L), rtol=1e-13)


def test_vcycle_is_exact_on_flat_geometry():
    """On a flat geometry the mode step with omega_m = 1 inverts the operator, so the V-cycle
    returns A^-1 f whatever else it does."""
    nx, M, L = 16, 8, 2.0
    g = op.Geometry(np.full(nx, 0.7), np.zeros(nx), L)
    H = pmg.Hierarchy(nx, M, g, g, pmg.PmgOptions(omega_m=1.0))
    f = np.random.default_rng(5).standard_normal((M + 1, nx))
    assert np.abs(H(f) - op.solve_dense(f, g, g)).max() < 1e-11 * np.abs(op.solve_dense(f, g, g)).max()


def test_vcycle_linear_and_contracting():
    nx, M = 16, 8
    go, gn = _sloped_geoms(nx)
    H = pmg.Hierarchy(nx, M, go, gn, pmg.PmgOptions())
    rng = np.random.default_rng(7)
    f, g = rng.standard_normal((2, M + 1, nx))
    assert np.abs(H(np.zeros_like(f))).max() == 0.0
    assert np.allclose(H(2 * f - 3 * g), 2 * H(f) - 3 * H(g), atol=1e-10 * np.abs(H(f)).max())
    # error propagation I - V A has spectral radius < 1 (dense, small grid)
    n = nx * (M + 1)
    A = op.assemble(nx, M, go, gn)
    V = np.column_stack([H(np.eye(n)[:, c].reshape(M + 1, nx)).ravel() for c in range(n)])
    rho = np.abs(np.linalg.eigvals(np.eye(n) - V @ A)).max()
    assert rho < 0.5


def test_vcycle_exact_coarse_two_levels():
    """With two levels and an exact coarse solve, the V-cycle is the textbook two-grid operator
    S (I - P A_c^-1 R A) S composed with the pre-smoother; check one application by hand."""
    nx, M = 8, 4
    go, gn = _sloped_geoms(nx)
    o = pmg.PmgOptions(coarse="exact")
    H = pmg.Hierarchy(nx, M, go, gn, o)
    f = np.random.default_rng(9).standard_normal((M + 1, nx))
    lev, levc = H.levels
    x = lev.pair(np.zeros_like(f), f, o)
    Ac = op.assemble(nx, 2, go, gn)
    ec = np.linalg.solve(Ac, (H.R[0] @ (f - op.apply(x, go, gn))).ravel()).reshape(3, nx)
    x = lev.pair(x + H.P[0] @ ec, f, o)
    assert np.allclose(H(f), x, atol=1e-12 * np.abs(x).max())


def test_fgmres_identity_preconditioner_matches_direct():
    pr = wl.manufactured_sloped(16, 5)
    go = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    x, info = krylov.fgmres(lambda v: op.apply(v, go, go), pr["b"], None, rtol=1e-12, restart=100,
                            maxit=400)
    xd = op.solve_dense(pr["b"], go, go)
    assert info["converged"] and np.abs(x - xd).max() < 1e-9 * np.abs(xd).max()


@pytest.mark.parametrize("maker", [lambda: wl.manufactured(32, 9), lambda: wl.manufactured_sloped(32, 9),
                                   lambda: wl.stokes_rest_problem(64, 17)])
def test_pmg_fgmres_converges_to_direct(maker):
    pr = maker()
    go = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    gn = op.Geometry(pr["h"], pr["eta_new"], pr["L"])
    H = pmg.Hierarchy(pr["nx"], pr["nz"] - 1, go, gn)
    x, info = krylov.fgmres(lambda v: op.apply(v, go, gn), pr["b"], H, rtol=1e-13)
    xd = op.solve_dense(pr["b"], go, gn)
    assert info["converged"] and info["iters"] <= 10
    assert np.linalg.norm(x - xd) < 1e-11 * np.linalg.norm(xd)


def test_mode_damping_rule():
    """The mode-step damping is 1 for flat and mildly varying depth, equals the closed form at a
    known depth ratio, and on a strongly varying tank it lowers the FGMRES iteration count."""
    nx, L = 32, 2 * math.pi
    x = sp.x_nodes(nx, L)
    flat = op.Geometry(np.ones(nx), np.zeros(nx), L)
    assert pmg.mode_damping(flat, flat) == 1.0
    mild = op.Geometry(np.ones(nx), 0.15 * np.cos(x), L)          # depth ratio 1.35
    assert pmg.mode_damping(mild, mild) == 1.0
    # depth from 0.5 to 1.5: c = 1/d^2 ratio 9 -> 2/(1 + 4.5^0.4)
    deep = op.Geometry(np.ones(nx), 0.5 * np.cos(x), L)
    assert abs(pmg.mode_damping(deep, deep) - 2.0 / (1.0 + 4.5 ** 0.4)) < 1e-14
    t = wl.batch(0, 512)[4]                                       # 128 x 17, depth ratio 2.6
    g = op.Geometry(t["h"], t["eta_old"], t["L"])
    its = []
    for adapt in (False, True):
        H = pmg.Hierarchy(t["nx"], t["nz"] - 1, g, g, pmg.PmgOptions(adapt_omega_m=adapt))
        _, info = krylov.fgmres(lambda v: op.apply(v, g, g), t["b"], H, rtol=1e-10, maxit=60)
        assert info["converged"]
        its.append(info["iters"])
    assert its[1] < its[0]


def test_fmg_linear_and_fewer_iterations():
    """Alg. 2 as a preconditioner: a fixed linear map, equal on one level to the V-cycle, equal
    to its correction form (on each level u + V_0(f - A u) with V_0 the cycle from zero, which is
    how the GPU evaluates it), and FGMRES preconditioned by it converges to the dense solution."""
    pr = wl.manufactured_sloped(32, 17)
    g = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    H = pmg.Hierarchy(32, 16, g, g, pmg.PmgOptions(cycle="FMG"))
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, 17, 32))
    assert np.abs(H(a + 2 * b) - H(a) - 2 * H(b)).max() <= 1e-10 * np.abs(H(a)).max()
    H1 = pmg.Hierarchy(32, 2, g, g, pmg.PmgOptions(cycle="FMG"))
    H1v = pmg.Hierarchy(32, 2, g, g, pmg.PmgOptions())
    f3 = rng.standard_normal((3, 32))
    assert np.array_equal(H1(f3), H1v(f3))
    fs = [a]
    for l in range(len(H.levels) - 1):
        fs.append(H.R[l] @ fs[-1])
    u = H.vcycle(fs[-1], len(H.levels) - 1)
    for l in range(len(H.levels) - 2, -1, -1):
        u = H.P[l] @ u
        u = u + H.vcycle(fs[l] - H.levels[l].apply(u), l)
    assert np.abs(u - H(a)).max() <= 1e-11 * np.abs(u).max()
    ref = op.solve_dense(pr["b"], g, g)
    x, info = krylov.fgmres(lambda v: op.apply(v, g, g), pr["b"], H, rtol=1e-12, maxit=60)
    assert info["converged"]
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("nx,M", [(32, 8), (64, 4)])
def test_bed_block_equals_definition(nx, M):
    """The bed-line block from its formula equals the bed row's own block of the assembled A
    (columns of the bed-row unknowns), on a sloped bed under a moving surface (the bed row uses
    the old geometry)."""
    go, gn = _sloped_geoms(nx)
    lev = pmg.Level(nx, M, go, gn)
    A = op.assemble(nx, M, go, gn)
    bed = M * nx + np.arange(nx)
    Lb = A[np.ix_(bed, bed)]
    assert np.abs(lev.bed_block() - Lb).max() <= 1e-12 * np.abs(Lb).max()


def test_bed_step_zeroes_the_bed_residual():
    """The bed-line step is an exact solve of the bed row with the other rows held: afterwards
    the bed row's residual vanishes, and the other rows of x are unchanged."""
    nx, M = 64, 4
    go, gn = _sloped_geoms(nx)
    lev = pmg.Level(nx, M, go, gn)
    rng = np.random.default_rng(3)
    x, f = rng.standard_normal((2, M + 1, nx))
    y = lev.bed_step(x, f)
    r = f - op.apply(y, go, gn)
    assert np.abs(r[M]).max() <= 1e-11 * np.abs(f).max()
    assert np.array_equal(y[:M], x[:M])


def test_bed_line_restores_contraction_on_a_steep_bed():
    """On the sloped manufactured problem at 128 x 5 (max|h_x| kappa_max / M^2 = 0.6) the cycle
    without the bed-line step amplifies the error (dense spectral radius of I - V A above 1,
    measured 8.2); with it the radius is about 0.1."""
    nx, M = 128, 4
    pr = wl.manufactured_sloped(nx, M + 1)
    g = op.Geometry(pr["h"], pr["eta_old"], pr["L"])
    A = op.assemble(nx, M, g, g)
    n = A.shape[0]
    rhos = []
    for bl in (False, True):
        H = pmg.Hierarchy(nx, M, g, g, pmg.PmgOptions(bed_line=bl))
        V = np.column_stack([H(np.eye(n)[:, c].reshape(M + 1, nx)).ravel() for c in range(n)])
        rhos.append(np.abs(np.linalg.eigvals(np.eye(n) - V @ A)).max())
    assert rhos[0] > 1.0 and rhos[1] < 0.2, rhos

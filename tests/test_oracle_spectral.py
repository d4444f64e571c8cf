"""Pins of the oracle's derivative operators against closed forms (paper Sec. 3.4-3.6)."""
import math

import numpy as np
import pytest

from oracle import spectral as sp


@pytest.mark.parametrize("nx,L", [(16, 2 * math.pi), (32, 7.3), (64, 30.0)])
def test_dx_exact_on_trig_polynomials(nx, L):
    x = sp.x_nodes(nx, L)
    k0 = 2 * math.pi / L
    kmax = nx // 2 - 1
    f = np.sin(3 * k0 * x) + 0.5 * np.cos(kmax * k0 * x) + 2.0
    df = 3 * k0 * np.cos(3 * k0 * x) - 0.5 * kmax * k0 * np.sin(kmax * k0 * x)
    assert np.allclose(sp.dx(f, L), df, rtol=0, atol=1e-12 * np.abs(df).max())


def test_dx_zeroes_nyquist():
    nx, L = 16, 2 * math.pi
    x = sp.x_nodes(nx, L)
    f = np.cos(nx // 2 * x)          # (-1)^i, the Nyquist mode
    assert np.abs(sp.dx(f, L)).max() < 1e-13


@pytest.mark.parametrize("nx,L", [(8, 2 * math.pi), (32, 3.0)])
def test_dx_matrix_equals_fft_form(nx, L):
    D = sp.dx_matrix(nx, L)
    rng = np.random.default_rng(1)
    f = rng.standard_normal(nx)
    assert np.allclose(D @ f, sp.dx(f, L), atol=1e-12 * np.abs(D @ f).max())


def test_dxx_spectral_matches_closed_form():
    nx, L = 32, 2 * math.pi
    x = sp.x_nodes(nx, L)
    f = np.cos(5 * x)
    assert np.allclose(sp.dxx_spectral(f, L), -25 * np.cos(5 * x), atol=1e-11)


@pytest.mark.parametrize("M", [2, 4, 8, 16, 32])
def test_dsig_exact_on_polynomials(M):
    s = sp.cgl_sigma(M)
    D = sp.dsig_matrix(M)
    for p in range(0, M + 1):
        f = s ** p
        df = p * s ** (p - 1) if p > 0 else np.zeros_like(s)
        assert np.abs(D @ f - df).max() <= 1e-12 * M * M * max(1.0, p)


def test_cgl_nodes_surface_to_bed():
    s = sp.cgl_sigma(8)
    assert s[0] == 1.0 and abs(s[-1]) < 1e-16
    assert np.all(np.diff(s) < 0)


@pytest.mark.parametrize("M", [4, 8, 16, 32])
def test_dsig_constant_and_recursion(M):
    D = sp.dsig_matrix(M)
    assert np.abs(D @ np.ones(M + 1)).max() < 1e-12 * M * M
    rng = np.random.default_rng(M)
    f = rng.standard_normal((M + 1, 3))
    assert np.allclose(D @ f, sp.dsig_modal(f), atol=1e-11 * M * M)


def test_cheb_transform_roundtrip_and_values():
    M = 8
    C = sp.cheb_forward_matrix(M)
    E = sp.cheb_eval_matrix(M, sp.cgl_xi(M))
    assert np.allclose(E @ C, np.eye(M + 1), atol=1e-14)
    # T_3 sampled at the nodes has coefficient vector e_3
    xi = sp.cgl_xi(M)
    t3 = 4 * xi ** 3 - 3 * xi
    a = C @ t3
    e3 = np.zeros(M + 1)
    e3[3] = 1.0
    assert np.allclose(a, e3, atol=1e-14)


def test_filters():
    # x: modes up to N_c untouched, the top mode damped by exp(-alpha (N - N_c)^2/(N + 1 - N_c)^2)
    nx, L = 32, 2 * math.pi
    x = sp.x_nodes(nx, L)
    low = np.cos(7 * x)
    assert np.allclose(sp.filter_x(low, L), low, atol=1e-14)
    top = np.cos(15 * x)
    ratio = (sp.filter_x(top, L) @ top) / (top @ top)
    N, Nc = 16, 8
    assert abs(ratio - math.exp(-36 * ((15 - Nc) / (N + 1 - Nc)) ** 2)) < 1e-12
    # sigma: a polynomial of degree <= floor(0.9 M) is unchanged, T_M is damped
    M = 16
    F = sp.filter_sigma_matrix(M)
    s = sp.cgl_sigma(M)
    assert np.allclose(F @ s ** 5, s ** 5, atol=1e-13)
    tM = np.cos(M * np.arccos(sp.cgl_xi(M)))
    assert np.linalg.norm(F @ tM) < 0.1 * np.linalg.norm(tM)

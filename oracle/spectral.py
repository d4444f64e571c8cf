"""Grids and derivative operators of the hybrid Fourier x Chebyshev discretisation.

Oracle (test infrastructure only).

Paper Sec. 3.4 (spatial discretisation) and Sec. 3.5 (computation of derivatives):

- x: equispaced periodic nodes, derivatives by FFT with the multipliers i*k (first) and -k^2
  (second). The build uses Nx nodes, Nx even, x_i = i L / Nx, and zeroes the Nyquist
  coefficient in the first derivative (the reading of the node formula and of the Nyquist mode is
  documented with the design).
- sigma: Chebyshev-Gauss-Lobatto nodes. The paper's node formula cos(m pi/(M+1)) omits an end
  point and lives on [-1, 1]; the oracle takes the Lobatto nodes xi_j = cos(j pi / M), j = 0..M,
  and maps them to sigma = (1 + xi) / 2, so sigma_0 = 1 is the free surface and sigma_M = 0 the bed.
  Then d/dsigma = 2 d/dxi.
- The paper evaluates sigma-derivatives through Chebyshev coefficients and a backward recursion
  (eq. chebDeriv and the recursion below it). The oracle provides that recursion and the nodal
  differentiation matrix; both give the same result up to rounding.
"""
import numpy as np


# ----------------------------------------------------------------------------- Fourier (x)

def x_nodes(nx, L):
    """Periodic nodes x_i = i L / nx, i = 0..nx-1 (Sec. 3.4)."""
    return np.arange(nx, dtype=np.float64) * (L / nx)


def wavenumbers(nx, L, zero_nyquist=True):
    """kappa_k = 2 pi k / L in FFT order; the Nyquist entry is set to 0 when asked (Sec. 3.5)."""
    k = np.fft.fftfreq(nx, d=1.0 / nx)
    kap = 2.0 * np.pi * k / L
    if zero_nyquist and nx % 2 == 0:
        kap[nx // 2] = 0.0
    return kap


def dx(f, L):
    """First x-derivative along the last axis: F^-1(i kappa F(f)), Nyquist zeroed (Sec. 3.5).

    The multiplier is odd in k, so the operator is real: real input gives real output, and a
    complex input is differentiated part by part (real and imaginary separately), so that the
    rounding of one part never leaks into the other (complex-step derivatives rely on that).
    """
    f = np.asarray(f)
    if np.iscomplexobj(f):
        return dx(f.real, L) + 1j * dx(f.imag, L)
    nx = f.shape[-1]
    return np.fft.ifft(1j * wavenumbers(nx, L) * np.fft.fft(f, axis=-1), axis=-1).real


def dxx_spectral(f, L):
    """Second x-derivative with the multiplier -k^2 of Sec. 3.5 (Nyquist kept: it is -(nx/2)^2 k0^2).

    Used only by the pins; the operator itself composes two first derivatives.
    """
    f = np.asarray(f)
    nx = f.shape[-1]
    kap = wavenumbers(nx, L, zero_nyquist=False)
    out = np.fft.ifft(-(kap ** 2) * np.fft.fft(f, axis=-1), axis=-1)
    return out.real if np.isrealobj(f) else out


def dx_matrix(nx, L):
    """Dense periodic differentiation matrix, (pi/L)(-1)^(i-l) cot((i-l) pi / nx), zero diagonal.

    This is the matrix of the FFT derivative with the Nyquist mode zeroed, written in closed form.
    """
    i = np.arange(nx)
    diff = i[:, None] - i[None, :]
    D = np.zeros((nx, nx))
    off = diff != 0
    D[off] = (np.pi / L) * ((-1.0) ** diff[off]) / np.tan(diff[off] * np.pi / nx)
    return D


def filter_x(f, L, frac=0.5, alpha=36.0, s=2.0):
    """Exponential cut-off filter in x (Sec. 3.6), applied along the last axis.

    Mode index i = |k|, N = nx/2, N_c = floor(frac * N): factor 1 for i <= N_c and
    exp(-alpha ((i - N_c)/(N + 1 - N_c))^s) above. (The exponent's sign is printed positive; a
    filter must damp, so the oracle uses the negative sign.) Complex input is filtered part by
    part, as in ``dx``.
    """
    f = np.asarray(f)
    if np.iscomplexobj(f):
        return filter_x(f.real, L, frac, alpha, s) + 1j * filter_x(f.imag, L, frac, alpha, s)
    nx = f.shape[-1]
    i = np.abs(np.fft.fftfreq(nx, d=1.0 / nx))
    sig = filter_factors(nx // 2, int(np.floor(frac * (nx // 2))), alpha, s, i)
    return np.fft.ifft(sig * np.fft.fft(f, axis=-1), axis=-1).real


def filter_factors(N, Nc, alpha, s, i):
    """F_S(i, N_c, alpha, s) of Sec. 3.6 with the damping sign."""
    i = np.asarray(i, dtype=np.float64)
    out = np.ones_like(i)
    hi = i > Nc
    out[hi] = np.exp(-alpha * ((i[hi] - Nc) / (N + 1.0 - Nc)) ** s)
    return out


# ----------------------------------------------------------------------------- Chebyshev (sigma)

def cgl_xi(M):
    """Chebyshev-Gauss-Lobatto nodes xi_j = cos(j pi / M), j = 0..M (xi_0 = 1)."""
    return np.cos(np.pi * np.arange(M + 1) / M)


def cgl_sigma(M):
    """sigma_j = (1 + xi_j)/2: row 0 is the free surface (sigma = 1), row M the bed (sigma = 0)."""
    return 0.5 * (1.0 + cgl_xi(M))


def dxi_matrix(M):
    """Chebyshev collocation derivative on the CGL nodes (closed form, negative-sum diagonal).

    D_jl = (c_j / c_l)(-1)^(j+l) / (xi_j - xi_l) for j != l with c_0 = c_M = 2, else 1; the node
    differences are evaluated as 2 sin((j+l) pi/2M) sin((l-j) pi/2M) to avoid cancellation, and
    the diagonal is minus the row sum so that D * 1 = 0 exactly.
    """
    n = M + 1
    j = np.arange(n)
    c = np.ones(n)
    c[0] = c[M] = 2.0
    J, Lm = np.meshgrid(j, j, indexing="ij")
    dxi = 2.0 * np.sin((J + Lm) * np.pi / (2 * M)) * np.sin((Lm - J) * np.pi / (2 * M))
    D = np.zeros((n, n))
    off = J != Lm
    D[off] = (c[J[off]] / c[Lm[off]]) * ((-1.0) ** (J[off] + Lm[off])) / dxi[off]
    D[j, j] = -D.sum(axis=1)
    return D


def dsig_matrix(M):
    """d/dsigma on the CGL nodes: 2 * D_xi (sigma = (1 + xi)/2)."""
    return 2.0 * dxi_matrix(M)


def cheb_forward_matrix(M):
    """Nodal values on the CGL nodes -> Chebyshev coefficients a_0..a_M (discrete DCT-I).

    a_m = 2/(M cbar_m) sum_j f_j T_m(xi_j) / cbar_j with cbar_0 = cbar_M = 2, else 1, so that
    f_j = sum_m a_m T_m(xi_j) exactly.
    """
    n = M + 1
    cb = np.ones(n)
    cb[0] = cb[M] = 2.0
    m = np.arange(n)
    T = np.cos(np.pi * np.outer(m, m) / M)          # T_m(xi_j), symmetric in (m, j)
    return (2.0 / M) * T / cb[:, None] / cb[None, :]


def cheb_eval_matrix(M, xi):
    """E[j, m] = T_m(xi_j) for m = 0..M at arbitrary points xi in [-1, 1]."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.cos(np.outer(np.arccos(np.clip(xi, -1.0, 1.0)), np.arange(M + 1)))


def cheb_derivative_coeffs(a):
    """Coefficients of d/dxi of sum_m a_m T_m by the backward recursion of Sec. 3.5.

    b_{q-1} = (b_{q+1} + 2 q a_q) / c_{q-1} for q = M, ..., 1, with b_M = b_{M+1} = 0, c_0 = 2 and
    c_q = 1 otherwise. (The printed start index is off by one; this is the standard recursion.)
    Works along axis 0.
    """
    a = np.asarray(a)
    M = a.shape[0] - 1
    b = np.zeros((M + 2,) + a.shape[1:], dtype=a.dtype)
    for q in range(M, 0, -1):
        cq = 2.0 if q - 1 == 0 else 1.0
        b[q - 1] = (b[q + 1] + 2.0 * q * a[q]) / cq
    return b[: M + 1]


def dsig_modal(f):
    """d/dsigma of nodal CGL values along axis 0 via coefficients + recursion (Sec. 3.5)."""
    f = np.asarray(f)
    M = f.shape[0] - 1
    a = np.tensordot(cheb_forward_matrix(M), f, axes=(1, 0))
    b = cheb_derivative_coeffs(a)
    E = cheb_eval_matrix(M, cgl_xi(M))
    return 2.0 * np.tensordot(E, b, axes=(1, 0))


def filter_sigma_matrix(M, frac=0.9, alpha=36.0, s=2.0):
    """Nodal filter along sigma: Chebyshev coefficients scaled by F_S(m, floor(frac M)) (Sec. 3.6)."""
    C = cheb_forward_matrix(M)
    E = cheb_eval_matrix(M, cgl_xi(M))
    fac = filter_factors(M, int(np.floor(frac * M)), alpha, s, np.arange(M + 1))
    return E @ (fac[:, None] * C)

"""The discrete mixed-stage pressure Poisson operator and its direct solution.

Oracle (test infrastructure only).

Fields are arrays P[j, i] with j = 0..M the sigma row (row 0 = free surface, row M = bed) and
i = 0..Nx-1 the x column.

- sigma-metrics, eq. 1_Scoef: d = h + eta, sigma_x = (h_x - sigma d_x)/d, sigma_z = 1/d, with h_x
  and d_x spectral x-derivatives.
- Transformed gradient of Sec. 2.1: Grad P = (D_x P + sigma_x D_s P, D_s P / d).
- The mixed-stage problem eq. poissonp puts the stage-k divergence on the stage-(k-1) gradient:
  interior rows are Div^new(Grad^old P). Row 0 carries the surface Dirichlet condition eq. bcpd
  (P = 0 data on z = eta); row M carries the bed condition eq. bcpdneu, n . Grad^old P with the
  un-normalised outward normal n = -(h_x, 1) (any normalisation cancels against the right-hand
  side).
- ``assemble`` writes the same operator as a dense matrix with Kronecker products
  (vec index j*Nx + i): D_x acts as I (x) D_x, D_s as D_s (x) I.
"""
import numpy as np
import scipy.linalg as sla

from . import spectral as sp


class Geometry:
    """sigma-metrics of one geometry (h, eta) on an Nx-periodic domain of length L (eq. 1_Scoef)."""

    def __init__(self, h, eta, L):
        self.h = np.asarray(h)
        self.eta = np.asarray(eta)
        self.L = float(L)
        self.d = self.h + self.eta
        self.hx = sp.dx(self.h, L)
        self.dxd = sp.dx(self.d, L)
        self.inv_d = 1.0 / self.d

    def sigma_x(self, sigma):
        """sigma_x[j, i] = (h_x,i - sigma_j d_x,i) / d_i."""
        return (self.hx[None, :] - np.asarray(sigma)[:, None] * self.dxd[None, :]) * self.inv_d[None, :]


def grad(P, g, M):
    """Transformed gradient (G_x, G_z) of the nodal field P on geometry g (Sec. 2.1)."""
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    Ps = Ds @ P
    Gx = sp.dx(P, g.L) + g.sigma_x(sig) * Ps
    Gz = Ps * g.inv_d[None, :]
    return Gx, Gz


def div(Fx, Fz, g, M):
    """Transformed divergence D_x F_x + sigma_x D_s F_x + D_s F_z / d on geometry g (Sec. 2.1)."""
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    return sp.dx(Fx, g.L) + g.sigma_x(sig) * (Ds @ Fx) + (Ds @ Fz) * g.inv_d[None, :]


def apply(P, g_old, g_new):
    """A P: interior Div^new Grad^old P, row 0 = P (Dirichlet), row M = -(h_x G_x + G_z) (bed)."""
    P = np.asarray(P)
    M = P.shape[0] - 1
    Gx, Gz = grad(P, g_old, M)
    out = div(Gx, Gz, g_new, M)
    out[0] = P[0]
    out[M] = -(g_old.hx * Gx[M] + Gz[M])
    return out


def assemble(nx, M, g_old, g_new):
    """Dense (Nz*Nx)^2 matrix of ``apply`` built from Kronecker products (vec index j*Nx + i)."""
    nz = M + 1
    Dx = sp.dx_matrix(nx, g_old.L)
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    DX = np.kron(np.eye(nz), Dx)
    DS = np.kron(Ds, np.eye(nx))
    Sxo = np.diag(g_old.sigma_x(sig).ravel())
    Sxn = np.diag(g_new.sigma_x(sig).ravel())
    Io = np.diag(np.tile(g_old.inv_d, nz))
    In = np.diag(np.tile(g_new.inv_d, nz))
    GX = DX + Sxo @ DS
    GZ = Io @ DS
    A = DX @ GX + Sxn @ DS @ GX + In @ DS @ GZ
    top = slice(0, nx)
    bed = slice(M * nx, nz * nx)
    A[top] = 0.0
    A[top, top] = np.eye(nx)
    A[bed] = -(np.diag(g_old.hx) @ GX[bed] + GZ[bed])
    return A


def solve_dense(b, g_old, g_new):
    """Definition-mode solve: P = A^-1 b by LU with partial pivoting on the dense matrix."""
    b = np.asarray(b)
    M = b.shape[0] - 1
    nx = b.shape[1]
    A = assemble(nx, M, g_old, g_new)
    return sla.lu_solve(sla.lu_factor(A), b.ravel()).reshape(b.shape)


def relres(P, b, g_old, g_new):
    """||b - A P||_2 / ||b||_2 over all entries, boundary rows included, no row scaling."""
    r = np.asarray(b) - apply(P, g_old, g_new)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


# ----------------------------------------------------------------------------- flat-mode solver

def flat_mode_blocks(nx, M, L, cbar, ebar):
    """Per-Fourier-mode matrices of the flat (x-averaged) operator.

    For mode k with kappa_k (Nyquist -> 0, because D_x annihilates it): row 0 = e_0, interior rows
    -kappa^2 e_j + cbar (D_s^2)_j, bed row -ebar (D_s)_M. On a flat geometry with depth d this is
    exactly the operator restricted to mode k when cbar = 1/d^2 and ebar = 1/d.
    Returns an array [nx, Nz, Nz].
    """
    nz = M + 1
    Ds = sp.dsig_matrix(M)
    Q = Ds @ Ds
    kap = sp.wavenumbers(nx, L)
    out = np.empty((nx, nz, nz))
    for k in range(nx):
        B = cbar * Q - kap[k] ** 2 * np.eye(nz)
        B[0] = 0.0
        B[0, 0] = 1.0
        B[M] = -ebar * Ds[M]
        out[k] = B
    return out


def flat_coefficients(g_old, g_new):
    """x-averages used by the flat-mode operator: cbar = <1/(d_o d_n)>, ebar = <(1 + h_x^2)/d_o>."""
    cbar = float(np.mean(g_old.inv_d * g_new.inv_d))
    ebar = float(np.mean((1.0 + g_old.hx ** 2) * g_old.inv_d))
    return cbar, ebar


def flat_mode_solve(r, blocks):
    """Apply the inverse of the flat operator: FFT rows, solve each mode's Nz x Nz system, iFFT."""
    R = np.fft.fft(r, axis=1)
    S = np.empty_like(R)
    for k in range(r.shape[1]):
        S[:, k] = np.linalg.solve(blocks[k], R[:, k])
    out = np.fft.ifft(S, axis=1)
    return out.real if np.isrealobj(r) else out

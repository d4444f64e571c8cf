"""The discrete mixed-stage pressure Poisson operator of a 3D tank: x and y periodic Fourier,
sigma Chebyshev.

Oracle (test infrastructure only).

Fields are arrays P[j, iy, ix] with j = 0..M the sigma row (row 0 = free surface, row M = bed),
iy = 0..Ny-1 and ix = 0..Nx-1 the horizontal nodes of the Ly x Lx periodic domain.

The 3D form carries the y-terms that the paper keeps throughout its sigma-transform (Sec. 2.1,
eq. 1_chain and eq. 1_Scoef with the horizontal gradient (d/dx, d/dy)), and Sec. 3.4's Fourier
derivatives apply in y as in x:
- metrics: d = h + eta, sigma_x = (h_x - sigma d_x)/d, sigma_y = (h_y - sigma d_y)/d,
  sigma_z = 1/d, all horizontal derivatives spectral;
- Grad P = (D_x P + sigma_x D_s P, D_y P + sigma_y D_s P, D_s P / d);
- Div F = D_x F_x + sigma_x D_s F_x + D_y F_y + sigma_y D_s F_y + D_s F_z / d;
- rows: 0 = P (Dirichlet surface), 1..M-1 = Div^new Grad^old P, M = the bed condition
  -(h_x G_x + h_y G_y + G_z) with the un-normalised outward normal -(h_x, h_y, 1) on the old
  geometry (eq. poissonp, eq. bcpd, eq. bcpdneu).
"""
import numpy as np
import scipy.linalg as sla

from . import spectral as sp


def dy(f, L):
    """First y-derivative along the second-last axis (same multiplier as ``spectral.dx``)."""
    return np.swapaxes(sp.dx(np.swapaxes(np.asarray(f), -1, -2), L), -1, -2)


class Geometry3:
    """sigma-metrics of one geometry h(y, x), eta(y, x) on an Ly x Lx periodic domain."""

    def __init__(self, h, eta, Lx, Ly):
        self.h = np.asarray(h, dtype=float)
        self.eta = np.asarray(eta, dtype=float)
        self.Lx, self.Ly = float(Lx), float(Ly)
        self.d = self.h + self.eta
        self.hx = sp.dx(self.h, Lx)
        self.hy = dy(self.h, Ly)
        self.dxd = sp.dx(self.d, Lx)
        self.dyd = dy(self.d, Ly)
        self.inv_d = 1.0 / self.d

    def sigma_x(self, sigma):
        s = np.asarray(sigma)[:, None, None]
        return (self.hx[None] - s * self.dxd[None]) * self.inv_d[None]

    def sigma_y(self, sigma):
        s = np.asarray(sigma)[:, None, None]
        return (self.hy[None] - s * self.dyd[None]) * self.inv_d[None]


def _ds(P):
    M = P.shape[0] - 1
    return np.tensordot(sp.dsig_matrix(M), P, axes=(1, 0))


def grad(P, g):
    """Transformed gradient (G_x, G_y, G_z) of the nodal field P on geometry g."""
    M = P.shape[0] - 1
    sig = sp.cgl_sigma(M)
    Ps = _ds(P)
    Gx = sp.dx(P, g.Lx) + g.sigma_x(sig) * Ps
    Gy = dy(P, g.Ly) + g.sigma_y(sig) * Ps
    Gz = Ps * g.inv_d[None]
    return Gx, Gy, Gz


def div(Fx, Fy, Fz, g):
    """Transformed divergence on geometry g."""
    M = Fx.shape[0] - 1
    sig = sp.cgl_sigma(M)
    return (sp.dx(Fx, g.Lx) + g.sigma_x(sig) * _ds(Fx) + dy(Fy, g.Ly) + g.sigma_y(sig) * _ds(Fy)
            + _ds(Fz) * g.inv_d[None])


def apply(P, g_old, g_new):
    """A P: interior Div^new Grad^old P, row 0 = P, row M = -(h_x G_x + h_y G_y + G_z)."""
    P = np.asarray(P)
    M = P.shape[0] - 1
    Gx, Gy, Gz = grad(P, g_old)
    out = div(Gx, Gy, Gz, g_new)
    out[0] = P[0]
    out[M] = -(g_old.hx * Gx[M] + g_old.hy * Gy[M] + Gz[M])
    return out


def assemble(nx, ny, M, g_old, g_new):
    """Dense matrix of ``apply`` from Kronecker products, vec index (j Ny + iy) Nx + ix."""
    nz = M + 1
    Dx = sp.dx_matrix(nx, g_old.Lx)
    Dy = sp.dx_matrix(ny, g_old.Ly)
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    Ih, Iz = np.eye(nx * ny), np.eye(nz)
    DX = np.kron(Iz, np.kron(np.eye(ny), Dx))
    DY = np.kron(Iz, np.kron(Dy, np.eye(nx)))
    DS = np.kron(Ds, Ih)
    Sxo = np.diag(g_old.sigma_x(sig).ravel())
    Syo = np.diag(g_old.sigma_y(sig).ravel())
    Sxn = np.diag(g_new.sigma_x(sig).ravel())
    Syn = np.diag(g_new.sigma_y(sig).ravel())
    Io = np.diag(np.tile(g_old.inv_d.ravel(), nz))
    In = np.diag(np.tile(g_new.inv_d.ravel(), nz))
    GX = DX + Sxo @ DS
    GY = DY + Syo @ DS
    GZ = Io @ DS
    A = DX @ GX + Sxn @ DS @ GX + DY @ GY + Syn @ DS @ GY + In @ DS @ GZ
    nh = nx * ny
    top = slice(0, nh)
    bed = slice(M * nh, nz * nh)
    A[top] = 0.0
    A[top, top] = np.eye(nh)
    A[bed] = -(np.diag(g_old.hx.ravel()) @ GX[bed] + np.diag(g_old.hy.ravel()) @ GY[bed]
               + GZ[bed])
    return A


def solve_dense(b, g_old, g_new):
    """Definition-mode solve P = A^-1 b (dense LU)."""
    b = np.asarray(b)
    M = b.shape[0] - 1
    ny, nx = b.shape[1], b.shape[2]
    A = assemble(nx, ny, M, g_old, g_new)
    return sla.lu_solve(sla.lu_factor(A), b.ravel()).reshape(b.shape)


def relres(P, b, g_old, g_new):
    r = np.asarray(b) - apply(P, g_old, g_new)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def flat_coefficients(g_old, g_new):
    """Horizontal averages of the flat-mode operator: cbar = <1/(d_o d_n)>,
    ebar = <(1 + h_x^2 + h_y^2)/d_o>."""
    cbar = float(np.mean(g_old.inv_d * g_new.inv_d))
    ebar = float(np.mean((1.0 + g_old.hx ** 2 + g_old.hy ** 2) * g_old.inv_d))
    return cbar, ebar


def flat_mode_blocks(nx, ny, M, Lx, Ly, cbar, ebar):
    """Per-mode (ky, kx) matrices of the flat operator: row 0 = e_0, interior
    -(kappa_x^2 + kappa_y^2) e_j + cbar (D_s^2)_j, bed row -ebar (D_s)_M. Array [ny, nx, Nz, Nz]."""
    nz = M + 1
    Ds = sp.dsig_matrix(M)
    Q = Ds @ Ds
    kx = sp.wavenumbers(nx, Lx)
    ky = sp.wavenumbers(ny, Ly)
    out = np.empty((ny, nx, nz, nz))
    for a in range(ny):
        for c in range(nx):
            B = cbar * Q - (kx[c] ** 2 + ky[a] ** 2) * np.eye(nz)
            B[0] = 0.0
            B[0, 0] = 1.0
            B[M] = -ebar * Ds[M]
            out[a, c] = B
    return out


def flat_mode_solve(r, blocks):
    """Inverse of the flat operator: 2D FFT of every row, one Nz x Nz solve per mode, inverse."""
    R = np.fft.fft2(r, axes=(-2, -1))
    S = np.empty_like(R)
    ny, nx = r.shape[1], r.shape[2]
    for a in range(ny):
        for c in range(nx):
            S[:, a, c] = np.linalg.solve(blocks[a, c], R[:, a, c])
    out = np.fft.ifft2(S, axes=(-2, -1))
    return out.real if np.isrealobj(r) else out

"""p-multigrid V-cycle on the Chebyshev order for the 3D tank (Alg. 1), dense steps.

Oracle (test infrastructure only).

The same cycle as ``pmg`` with the 3D operator of ``operator3d``: levels M_l = M / 2^l down to 2
with Nx, Ny and the horizontal metrics unchanged; restriction and prolongation act on every
(y, x) column; the smoothing pair is
- the column step: block Jacobi with the exact inverse of each column's horizontal-diagonal
  block of A (D_x and D_y have zero diagonals, so the block is (c_xx + c_yy) I +
  diag(sx_n) D_s diag(sx_o) D_s + diag(sy_n) D_s diag(sy_o) D_s + D_s^2/(d_n d_o), surface row e_0,
  bed row -(h_x sx_o[M] + h_y sy_o[M] + 1/d_o) (D_s)_M), damping omega_c;
- the mode step: the exact inverse of the horizontally averaged flat operator per Fourier mode
  (kx, ky), damping omega_m scaled by ``pmg.mode_damping``.
The coarsest level runs ``coarse_pairs`` pairs from zero, or a dense LU with coarse='exact'.
"""
from dataclasses import replace

import numpy as np
import scipy.linalg as sla

from . import operator3d as op3
from . import pmg
from . import spectral as sp


def column_blocks(nx, ny, M, g_old, g_new):
    """B at every column (iy, ix), array [ny, nx, Nz, Nz], from the formula."""
    nz = M + 1
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    sxo, syo = g_old.sigma_x(sig), g_old.sigma_y(sig)
    sxn, syn = g_new.sigma_x(sig), g_new.sigma_y(sig)
    cxx = pmg.dxx_diagonal(nx, g_old.Lx)
    cyy = pmg.dxx_diagonal(ny, g_old.Ly) if ny > 1 else 0.0
    out = np.empty((ny, nx, nz, nz))
    for a in range(ny):
        for c in range(nx):
            B = ((cxx + cyy) * np.eye(nz)
                 + np.diag(sxn[:, a, c]) @ Ds @ np.diag(sxo[:, a, c]) @ Ds
                 + np.diag(syn[:, a, c]) @ Ds @ np.diag(syo[:, a, c]) @ Ds
                 + g_new.inv_d[a, c] * g_old.inv_d[a, c] * (Ds @ Ds))
            B[0] = 0.0
            B[0, 0] = 1.0
            B[M] = -(g_old.hx[a, c] * sxo[M, a, c] + g_old.hy[a, c] * syo[M, a, c]
                     + g_old.inv_d[a, c]) * Ds[M]
            out[a, c] = B
    return out


class Level3:
    def __init__(self, nx, ny, M, g_old, g_new):
        self.nx, self.ny, self.M = nx, ny, M
        self.g_old, self.g_new = g_old, g_new
        self.col = column_blocks(nx, ny, M, g_old, g_new)
        cbar, ebar = op3.flat_coefficients(g_old, g_new)
        self.mode = op3.flat_mode_blocks(nx, ny, M, g_old.Lx, g_old.Ly, cbar, ebar)
        self._lu = None

    def apply(self, x):
        return op3.apply(x, self.g_old, self.g_new)

    def column_step(self, x, f, omega):
        r = f - self.apply(x)
        corr = np.empty_like(r)
        for a in range(self.ny):
            for c in range(self.nx):
                corr[:, a, c] = np.linalg.solve(self.col[a, c], r[:, a, c])
        return x + omega * corr

    def mode_step(self, x, f, omega):
        return x + omega * op3.flat_mode_solve(f - self.apply(x), self.mode)

    def pair(self, x, f, o):
        x = self.column_step(x, f, o.omega_c)
        return self.mode_step(x, f, o.omega_m)

    def exact(self, f):
        if self._lu is None:
            self._lu = sla.lu_factor(op3.assemble(self.nx, self.ny, self.M, self.g_old,
                                                  self.g_new))
        return sla.lu_solve(self._lu, f.ravel()).reshape(f.shape)


class Hierarchy3:
    """V-cycle (Alg. 1, correction scheme from a zero guess) for the 3D operator."""

    def __init__(self, nx, ny, M, g_old, g_new, opts=None):
        opts = opts or pmg.PmgOptions()
        if opts.adapt_omega_m:
            opts = replace(opts, omega_m=opts.omega_m * pmg.mode_damping(g_old, g_new),
                           adapt_omega_m=False)
        self.opts = opts
        self.orders = pmg.level_orders(M)
        self.levels = [Level3(nx, ny, m, g_old, g_new) for m in self.orders]
        self.R = [pmg.restriction_matrix(m) for m in self.orders[:-1]]
        self.P = [pmg.prolongation_matrix(m) for m in self.orders[:-1]]

    @staticmethod
    def _rows(T, v):
        return np.tensordot(T, v, axes=(1, 0))

    def vcycle(self, f, l=0):
        o = self.opts
        lev = self.levels[l]
        x = np.zeros_like(f)
        if l == len(self.levels) - 1:
            if o.coarse == "exact":
                return lev.exact(f)
            for _ in range(o.coarse_pairs):
                x = lev.pair(x, f, o)
            return x
        for _ in range(o.nu1):
            x = lev.pair(x, f, o)
        ec = self.vcycle(self._rows(self.R[l], f - lev.apply(x)), l + 1)
        x = x + self._rows(self.P[l], ec)
        for _ in range(o.nu2):
            x = lev.pair(x, f, o)
        return x

    def __call__(self, f):
        return self.vcycle(np.asarray(f))

"""p-multigrid V-cycle on the Chebyshev order (Alg. 1), as a plain composition of dense steps.

Oracle (test infrastructure only).

- Coarsening (Sec. 4.1): the rule doubles, level by level towards the fine grid, whichever of the
  two orders is smaller (the printed conditions "= and <" are read as "<="). Going coarse it
  therefore halves the smaller order. Every grid used here has Nx >= 2M, so only the Chebyshev
  order is coarsened: M_l = M / 2^l down to M_L = 2, with Nx and the x-metrics unchanged.
- Coarse operators are the same discrete operator re-discretised at order M_l.
- Transfers (Sec. 4.2): restriction takes Chebyshev coefficients, drops the modes above the coarse
  order and evaluates at the coarse nodes; prolongation is the zero-padded expansion evaluated at
  the fine nodes (polynomial interpolation). The residual's boundary rows are injected: the
  coarse surface and bed rows take the fine surface and bed rows, which sit at the same sigma.
- Smoother (Sec. 4.3): the paper smooths with Gauss-Seidel over column blocks A_rr (one block per
  x column, Nz x Nz). The oracle keeps that block: the x-diagonal block of A at column i. Its
  relaxation is parallel (block Jacobi, damping omega_c), and it is paired with a second line
  relaxation along x: the exact inverse of the x-averaged flat operator, mode by mode (damping
  omega_m, scaled per geometry by ``mode_damping``). One "pair" is a column step followed by a mode
  step, each from the current residual.
- Optional third step of a pair (``bed_line``): the bed row's boundary condition couples the
  columns through h_x D_x, which neither the column blocks (D_x has a zero diagonal) nor the
  x-averaged mode blocks (h_x averages to zero) contain. The bed-line step solves the bed row's
  own Nx x Nx block of A exactly, with the other rows held: x_M += L_b^-1 (f - A x)_M, where
  L_b = -(diag(h_x) D_x + diag((h_x sigma_x[M] + 1/d) (D_sigma)_MM)) on the old geometry. It is
  a line relaxation along x, the Sec. 4.3 smoother's block idea applied to the bed row.
- Coarsest level (Alg. 1, p = 1): the paper uses a direct solver. Here the coarsest level still
  couples all Nx columns densely, so the oracle runs ``coarse_pairs`` smoothing pairs from a zero
  guess there (a fixed linear map); ``coarse='exact'`` uses a dense LU instead, for comparison.
- V-cycle (Alg. 1) as the correction scheme: on level l, smooth A_l x = f from the initial guess
  (nu1 pairs), form the residual r = f - A_l x, restrict it, solve the coarse residual equation
  A_{l+1} e = R r approximately by the same cycle from a zero guess, add the prolongated correction
  P e, and smooth again (nu2 pairs). The value of the recursive call is the coarse correction e.
- Full multigrid (Alg. 2) as nested iteration: the right-hand side is restricted to every level;
  each level's V-cycle starts from the prolongated result of the next coarser level (from zero on
  the coarsest level), ending with the finest level's V-cycle.
"""
from dataclasses import dataclass, replace

import numpy as np
import scipy.linalg as sla

from . import operator as op
from . import spectral as sp


@dataclass
class PmgOptions:
    nu1: int = 1
    nu2: int = 1
    omega_c: float = 1.0
    omega_m: float = 1.0
    coarse_pairs: int = 1
    coarse: str = "smooth"        # "smooth" (fixed pairs) or "exact" (dense LU)
    adapt_omega_m: bool = True    # scale omega_m by mode_damping(geometry)
    cycle: str = "V"              # preconditioner: "V" (Alg. 1) or "FMG" (Alg. 2)
    bed_line: bool = False        # add the bed-line step to every smoothing pair


def mode_damping(g_old, g_new):
    """Damping factor of the flat-mode step for one geometry pair (the paper gives no damping).

    The mode step inverts the x-averaged operator, whose sigma-sigma coefficient is the mean of
    c = 1/(d_old d_new); where c varies along x the step over- and under-corrects locally. With
    r = max c / min c the factor is min(1, 2 / (1 + (r/2)^0.4)): exactly 1 on flat and mildly
    varying geometries (r <= 2, depth ratios up to ~1.4, such as the 256 x 17 Stokes wave),
    ~0.75 at depth ratio 2.7 and ~0.56 for the trapezoidal bar (ratio 4.6). The form and its two
    constants were chosen from FGMRES iteration counts measured with this oracle on those
    workloads; it is a tuning rule, not a result of the paper.
    """
    c = np.asarray(g_old.inv_d * g_new.inv_d)
    r = float(np.max(np.abs(c)) / np.min(np.abs(c)))
    return min(1.0, 2.0 / (1.0 + (r / 2.0) ** 0.4))


def level_orders(M):
    """M, M/2, ..., 2 (M must be a power of two >= 2)."""
    out = [M]
    while out[-1] > 2:
        out.append(out[-1] // 2)
    return out


def restriction_matrix(Mf):
    """(Mc+1) x (Mf+1): coefficients, truncate to Mc = Mf/2, evaluate at coarse nodes; inject rows 0, M."""
    Mc = Mf // 2
    C = sp.cheb_forward_matrix(Mf)[: Mc + 1]
    E = sp.cheb_eval_matrix(Mc, sp.cgl_xi(Mc))
    R = E @ C
    R[0] = 0.0
    R[0, 0] = 1.0
    R[Mc] = 0.0
    R[Mc, Mf] = 1.0
    return R


def prolongation_matrix(Mf):
    """(Mf+1) x (Mc+1): interpolate the coarse-degree polynomial at the fine nodes."""
    Mc = Mf // 2
    C = sp.cheb_forward_matrix(Mc)
    E = sp.cheb_eval_matrix(Mc, sp.cgl_xi(Mf))
    return E @ C


def dxx_diagonal(nx, L):
    """Diagonal entry of D_x D_x: -(1/nx) sum_k kappa_k^2 with the Nyquist mode zeroed."""
    return -float(np.sum(sp.wavenumbers(nx, L) ** 2)) / nx


def column_blocks(nx, M, g_old, g_new):
    """B_i = x-diagonal block of A at column i (formula), array [nx, Nz, Nz].

    Interior rows: diag(D_xx) I + diag(sx_n) D_s diag(sx_o) D_s + D_s^2 / (d_n d_o); row 0 = e_0;
    row M = -(h_x sx_o[M] + 1/d_o) (D_s)_M. (D_x has a zero diagonal, so the mixed x-sigma terms
    contribute nothing to the block.)
    """
    nz = M + 1
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    sxo = g_old.sigma_x(sig)
    sxn = g_new.sigma_x(sig)
    cxx = dxx_diagonal(nx, g_old.L)
    out = np.empty((nx, nz, nz))
    for i in range(nx):
        B = cxx * np.eye(nz) + np.diag(sxn[:, i]) @ Ds @ np.diag(sxo[:, i]) @ Ds \
            + g_new.inv_d[i] * g_old.inv_d[i] * (Ds @ Ds)
        B[0] = 0.0
        B[0, 0] = 1.0
        B[M] = -(g_old.hx[i] * sxo[M, i] + g_old.inv_d[i]) * Ds[M]
        out[i] = B
    return out


def column_blocks_from_dense(A, nx, M):
    """The same blocks read off an assembled matrix (the definition); used by the pins."""
    nz = M + 1
    out = np.empty((nx, nz, nz))
    for i in range(nx):
        idx = np.arange(nz) * nx + i
        out[i] = A[np.ix_(idx, idx)]
    return out


class Level:
    def __init__(self, nx, M, g_old, g_new):
        self.nx, self.M = nx, M
        self.g_old, self.g_new = g_old, g_new
        self.col = column_blocks(nx, M, g_old, g_new)
        cbar, ebar = op.flat_coefficients(g_old, g_new)
        self.mode = op.flat_mode_blocks(nx, M, g_old.L, cbar, ebar)
        self._coarse_lu = None

    def apply(self, x):
        return op.apply(x, self.g_old, self.g_new)

    def column_step(self, x, f, omega):
        r = f - self.apply(x)
        corr = np.empty_like(r)
        for i in range(self.nx):
            corr[:, i] = np.linalg.solve(self.col[i], r[:, i])
        return x + omega * corr

    def mode_step(self, x, f, omega):
        r = f - self.apply(x)
        return x + omega * op.flat_mode_solve(r, self.mode)

    def bed_block(self):
        """L_b: the bed row's coupling to the bed-row unknowns (Nx x Nx), from the formula."""
        g = self.g_old
        M = self.M
        dsmm = sp.dsig_matrix(M)[M, M]
        sxm = g.sigma_x(sp.cgl_sigma(M))[M]
        c = (g.hx * sxm + g.inv_d) * dsmm
        return -(g.hx[:, None] * sp.dx_matrix(self.nx, g.L) + np.diag(c))

    def bed_step(self, x, f):
        """Exact line solve of the bed row: x_M += L_b^-1 (f - A x)_M."""
        if getattr(self, "_bed_lu", None) is None:
            self._bed_lu = sla.lu_factor(self.bed_block())
        r = f - self.apply(x)
        x = np.array(x, dtype=np.result_type(x, r))
        x[self.M] = x[self.M] + sla.lu_solve(self._bed_lu, r[self.M])
        return x

    def pair(self, x, f, o):
        x = self.column_step(x, f, o.omega_c)
        x = self.mode_step(x, f, o.omega_m)
        if o.bed_line:
            x = self.bed_step(x, f)
        return x

    def exact(self, f):
        if self._coarse_lu is None:
            A = op.assemble(self.nx, self.M, self.g_old, self.g_new)
            self._coarse_lu = sla.lu_factor(A)
        return sla.lu_solve(self._coarse_lu, f.ravel()).reshape(f.shape)


class Hierarchy:
    """Levels M_l = M/2^l (fine to coarse) with transfers; ``vcycle`` is Alg. 1 from a zero guess."""

    def __init__(self, nx, M, g_old, g_new, opts=None):
        opts = opts or PmgOptions()
        if opts.adapt_omega_m:
            opts = replace(opts, omega_m=opts.omega_m * mode_damping(g_old, g_new),
                           adapt_omega_m=False)
        self.opts = opts
        self.orders = level_orders(M)
        self.levels = [Level(nx, m, g_old, g_new) for m in self.orders]
        self.R = [restriction_matrix(m) for m in self.orders[:-1]]
        self.P = [prolongation_matrix(m) for m in self.orders[:-1]]

    def vcycle(self, f, l=0, x0=None):
        """V-cycle (Alg. 1) for A_l x = f on level l from the initial guess x0 (zero when None):
        the correction scheme described in the module docstring."""
        o = self.opts
        lev = self.levels[l]
        x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.result_type(f, x0))
        if l == len(self.levels) - 1:
            if o.coarse == "exact":
                return lev.exact(f)
            for _ in range(o.coarse_pairs):
                x = lev.pair(x, f, o)
            return x
        for _ in range(o.nu1):
            x = lev.pair(x, f, o)
        r = f - lev.apply(x)
        ec = self.vcycle(self.R[l] @ r, l + 1)
        x = x + self.P[l] @ ec
        for _ in range(o.nu2):
            x = lev.pair(x, f, o)
        return x

    def fmg(self, f):
        """Full multigrid (Alg. 2) as nested iteration: right-hand sides f_l = R f_{l-1} on every
        level (the paper does not say how the coarser right-hand sides are formed; restriction is
        the reading taken), then from the coarsest level up a V-cycle for A_l u = f_l started from
        the prolongated approximation of the level below (from zero on the coarsest level)."""
        fs = [np.asarray(f)]
        for l in range(len(self.levels) - 1):
            fs.append(self.R[l] @ fs[-1])
        u = None
        for l in range(len(self.levels) - 1, 0, -1):
            u = self.vcycle(fs[l], l, x0=u)
            u = self.P[l - 1] @ u
        return self.vcycle(fs[0], 0, x0=u)

    def __call__(self, f):
        if self.opts.cycle == "FMG":
            return self.fmg(np.asarray(f))
        return self.vcycle(np.asarray(f))

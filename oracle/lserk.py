"""Low-storage explicit Runge-Kutta stepping with the per-stage pressure projection.

Oracle (test infrastructure only).

- The 2N-storage form of eq. LSERK: K^k = alpha_k K^(k-1) + dt f(y^(k-1)), y^(k) = y^(k-1) +
  beta_k K^k. The paper gives no coefficients; the oracle uses the five-stage fourth-order set of
  Carpenter and Kennedy (1994). ``butcher`` rewrites them as a Butcher tableau for the order pins.
- One stage (Sec. 3.2, 3.3, 3.6), from the state (u, w, eta, K_u, K_w, K_eta) of stage k-1:
  1. surface: K_eta <- alpha K_eta + dt eta_t with eta_t = -u~ D_x eta + w~ (kinematic condition,
     u~, w~ the surface row); eta <- eta + beta K_eta; x-filter of eta (new surface).
  2. sigma-metrics of the old surface (stage k-1) and of the new one.
  3. forcing at the old stage: F_u = -u D_x u - w_s D_s u - g D_x eta + nu Div Grad u and
     F_w = -u D_x w - w_s D_s w + nu Div Grad w, with w_s = sigma_t + u sigma_x + w / d and
     sigma_t = -sigma eta_t / d (eq. 1_Scoef with d_t = eta_t); the hydrostatic pressure leaves
     -g D_x eta in the horizontal equation and cancels gravity in the vertical one.
  4. provisional velocity u* = u + beta (alpha K_u + dt F_u), likewise w*.
  5. pressure: A p = b with A the mixed-stage operator (old gradient, new divergence), interior
     b = rho/(beta dt) Div^new(u*, w*), surface b = 0, bed b = -rho/(beta dt)(h_x u* + w*)
     (eq. poissonp with eq. bcpd and eq. bcpdneu; from div u^(k) = 0 and n . u^(k) = 0 on the bed).
  6. K_u <- alpha K_u + dt (F_u - G_x / rho), K_w likewise with G_z, (G_x, G_z) = Grad^old p;
     u <- u + beta K_u, w <- w + beta K_w. Here Div^new(u, w) vanishes inside (to the solver
     tolerance) and n . u = 0 on the bed.
  7. filter u and w in x and sigma (Sec. 3.6); K is not filtered.

Two model options (``Physics``), for the oscillatory boundary-layer case (Sec. 5, oscillatory wave
boundary layer):
- ``linear``: the linearised equations (eq. NSElin with eq. linFS): no advection terms in F_u, F_w
  (the sigma_t mesh-velocity term, second order in the amplitude, goes with them),
  eta_t = w~, and the sigma-map held on the still-water domain (d = h, metrics of eta = 0 for
  both the old and the new geometry), so the boundary conditions sit at z = 0.
- ``no_slip``: u = 0 on the bed (the paper's no-slip condition) for both velocity components.
  The bed row of the pressure problem keeps its form: with the bed rows of u and K zero at the
  stage start, the provisional bed velocity is beta dt (F_u, F_w), so the Neumann datum is the
  normal component of the momentum forcing, viscous stress included. After the update and the
  filter the bed rows of u, w, K_u and K_w are set to zero (the projection cannot remove the
  tangential slip by itself).
"""
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from . import operator as op
from . import spectral as sp

# Carpenter-Kennedy (5,4) 2N-storage coefficients.
CK_ALPHA = [Fraction(0), Fraction(-567301805773, 1357537059087),
            Fraction(-2404267990393, 2016746695238), Fraction(-3550918686646, 2091501179385),
            Fraction(-1275806237668, 842570457699)]
CK_BETA = [Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
           Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
           Fraction(2277821191437, 14882151754819)]
ALPHA = [float(a) for a in CK_ALPHA]
BETA = [float(b) for b in CK_BETA]


def butcher(alpha=CK_ALPHA, beta=CK_BETA):
    """Butcher tableau (a, b, c) of the 2N scheme (exact rationals).

    With f_j = f(y^(j-1)), y^(k) = y^n + dt sum_j C[k][j] f_j where
    C[k][j] = sum_{m=j..k} beta_m prod_{i=j+1..m} alpha_i; stage i evaluates f at y^(i-1), so
    a[i][j] = C[i-1][j] and b[j] = C[s][j].
    """
    s = len(alpha)
    C = [[Fraction(0)] * (s + 1) for _ in range(s + 1)]
    for k in range(1, s + 1):
        for j in range(1, k + 1):
            tot = Fraction(0)
            for m in range(j, k + 1):
                prod = Fraction(1)
                for i in range(j + 1, m + 1):
                    prod *= alpha[i - 1]
                tot += beta[m - 1] * prod
            C[k][j] = tot
    a = [[C[i - 1][j] if j < i else Fraction(0) for j in range(1, s + 1)] for i in range(1, s + 1)]
    b = [C[s][j] for j in range(1, s + 1)]
    c = [sum(row) for row in a]
    return a, b, c


@dataclass
class Physics:
    rho: float = 1000.0
    g: float = 9.81
    nu: float = 1e-6
    filt_alpha: float = 36.0
    filt_s: float = 2.0
    filt_fx: float = 0.5
    filt_fz: float = 0.9
    linear: bool = False
    no_slip: bool = False


@dataclass
class State:
    u: np.ndarray
    w: np.ndarray
    eta: np.ndarray
    Ku: np.ndarray
    Kw: np.ndarray
    Keta: np.ndarray
    p: np.ndarray

    @staticmethod
    def rest_registers(u, w, eta):
        z = np.zeros_like(u)
        return State(u.copy(), w.copy(), eta.copy(), z.copy(), z.copy(), np.zeros_like(eta), z.copy())


def filter_field(F, L, ph):
    M = F.shape[0] - 1
    Fs = sp.filter_sigma_matrix(M, ph.filt_fz, ph.filt_alpha, ph.filt_s)
    return Fs @ sp.filter_x(F, L, ph.filt_fx, ph.filt_alpha, ph.filt_s)


def forcing(u, w, eta, eta_t, g_old, ph):
    """(F_u, F_w) at the old stage (step 3 above)."""
    M = u.shape[0] - 1
    L = g_old.L
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    sx = g_old.sigma_x(sig)
    st = -sig[:, None] * (eta_t * g_old.inv_d)[None, :]
    ws = st + u * sx + w * g_old.inv_d[None, :]
    def visc(f):
        v = ph.nu * op.div(*op.grad(f, g_old, M), g_old, M)
        if ph.no_slip:
            v[0] = 0.0
        return v
    if ph.linear:
        return -ph.g * sp.dx(eta, L)[None, :] + visc(u), visc(w)
    Fu = -u * sp.dx(u, L) - ws * (Ds @ u) - ph.g * sp.dx(eta, L)[None, :] + visc(u)
    Fw = -u * sp.dx(w, L) - ws * (Ds @ w) + visc(w)
    return Fu, Fw


def rhs(us, ws_, g_new, hx, scale):
    """Right-hand side of the stage's pressure problem (step 5 above)."""
    M = us.shape[0] - 1
    b = scale * op.div(us, ws_, g_new, M)
    b[0] = 0.0
    b[M] = -scale * (hx * us[M] + ws_[M])
    return b


def stage(k, dt, h, L, s, solve, ph=None):
    """Advance State s through stage k (1..5) in place. solve(b, g_old, g_new, p0) -> p.

    Returns diagnostics: max |interior Div^new u^(k)| before the filter, and its reference scale
    max |interior Div^new u*|.
    """
    ph = ph or Physics()
    a, bcoef = ALPHA[k - 1], BETA[k - 1]
    M = s.u.shape[0] - 1
    eta_old = s.eta.copy()
    if ph.linear:
        eta_t = s.w[0].copy()
    else:
        eta_t = -s.u[0] * sp.dx(eta_old, L) + s.w[0]
    s.Keta = a * s.Keta + dt * eta_t
    eta_new = sp.filter_x(eta_old + bcoef * s.Keta, L, ph.filt_fx, ph.filt_alpha, ph.filt_s)
    if ph.linear:
        g_old = op.Geometry(h, np.zeros_like(eta_old), L)
        g_new = g_old
    else:
        g_old = op.Geometry(h, eta_old, L)
        g_new = op.Geometry(h, eta_new, L)
    Fu, Fw = forcing(s.u, s.w, eta_old, eta_t, g_old, ph)
    us = s.u + bcoef * (a * s.Ku + dt * Fu)
    ws_ = s.w + bcoef * (a * s.Kw + dt * Fw)
    scale = ph.rho / (bcoef * dt)
    b = rhs(us, ws_, g_new, g_old.hx, scale)
    p = solve(b, g_old, g_new, s.p)
    Gx, Gz = op.grad(p, g_old, M)
    s.Ku = a * s.Ku + dt * (Fu - Gx / ph.rho)
    s.Kw = a * s.Kw + dt * (Fw - Gz / ph.rho)
    u = s.u + bcoef * s.Ku
    w = s.w + bcoef * s.Kw
    div_after = np.abs(op.div(u, w, g_new, M)[1:M]).max()
    div_ref = np.abs(op.div(us, ws_, g_new, M)[1:M]).max()
    s.u = filter_field(u, L, ph)
    s.w = filter_field(w, L, ph)
    if ph.no_slip:
        for f in (s.u, s.w, s.Ku, s.Kw):
            f[M] = 0.0
    s.eta = eta_new
    s.p = p
    return dict(div=div_after, div_ref=div_ref, bed_flux=np.abs(g_old.hx * u[M] + w[M]).max())


def dense_solver(b, g_old, g_new, p0):
    return op.solve_dense(b, g_old, g_new)


def step(dt, h, L, s, solve=dense_solver, ph=None):
    """One full time step: the five stages."""
    diags = []
    for k in range(1, 6):
        diags.append(stage(k, dt, h, L, s, solve, ph))
    return diags

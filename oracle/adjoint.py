"""Discrete adjoint of the pressure solve and of the time-stepping stage, w.r.t. the state and
the still-water depth h(x).

Oracle (test infrastructure only). The paper has no adjoint; this module is the reference for
the GPU adjoint. It is the transpose, step by step, of the forward computation of
``operator.apply`` and ``lserk.stage``, written out by hand (reverse mode). The pins are the
dense transpose of the assembled operator and complex-step derivatives of the forward code.

Notation: a geometry is (a, b, i) per x with sigma_x = a + b sigma, a = h_x / d, b = -d_x / d,
i = 1/d, d = h + eta (eq. 1_Scoef). ``GeoBar`` collects the adjoints of a, b, i of one geometry;
``geometry_T`` maps them (plus a direct adjoint of h_x) back to h and eta.

- D_x is real and antisymmetric (odd multiplier, Nyquist zeroed), so D_x^T = -D_x.
- The x-filter has an even real multiplier, so it is symmetric.
- D_sigma and the sigma-filter are plain matrices; their transposes are explicit.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import lserk
from . import operator as op
from . import spectral as sp


@dataclass
class GeoBar:
    """Adjoints of the metric rows (a, b, i) of one geometry, each [Nx]."""
    a: np.ndarray
    b: np.ndarray
    i: np.ndarray

    @staticmethod
    def zeros(nx, dtype=float):
        return GeoBar(np.zeros(nx, dtype), np.zeros(nx, dtype), np.zeros(nx, dtype))


def _ab(g):
    """(a, b) of sigma_x = a + b sigma for an ``operator.Geometry``."""
    return g.hx * g.inv_d, -g.dxd * g.inv_d


def dxT(f, L):
    return -sp.dx(f, L)


def sigx_T(S, gb, sig):
    """Accumulate the adjoint S of sigma_x[j, i] = a_i + b_i sigma_j into gb."""
    gb.a += S.sum(axis=0)
    gb.b += (sig[:, None] * S).sum(axis=0)


def grad_T(Gbx, Gbz, P, g, gb, M):
    """Adjoint of (G_x, G_z) = Grad^g P: returns Pbar; accumulates the metric adjoints of g.

    G_x = D_x P + sigma_x D_s P, G_z = i D_s P.
    """
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    Ps = Ds @ P
    sigx_T(Gbx * Ps, gb, sig)
    gb.i += (Gbz * Ps).sum(axis=0)
    return dxT(Gbx, g.L) + Ds.T @ (g.sigma_x(sig) * Gbx + g.inv_d[None, :] * Gbz)


def div_T(Db, Fx, Fz, g, gb, M):
    """Adjoint of D = Div^g(F_x, F_z) = D_x F_x + sigma_x D_s F_x + i D_s F_z: returns
    (Fxbar, Fzbar); accumulates the metric adjoints of g."""
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    sigx_T(Db * (Ds @ Fx), gb, sig)
    gb.i += (Db * (Ds @ Fz)).sum(axis=0)
    Fxb = dxT(Db, g.L) + Ds.T @ (g.sigma_x(sig) * Db)
    Fzb = Ds.T @ (g.inv_d[None, :] * Db)
    return Fxb, Fzb


def _bed_rows_T(lam, Gx, hx, M):
    """Adjoint of the bed row -(h_x G_x[M] + G_z[M]) for the weight lam[M]: (Gxbar, Gzbar, hxbar)
    contributions."""
    Gbx = np.zeros_like(lam)
    Gbz = np.zeros_like(lam)
    Gbx[M] = -hx * lam[M]
    Gbz[M] = -lam[M]
    return Gbx, Gbz, -lam[M] * Gx[M]


def apply_T(lam, g_old, g_new):
    """A^T lam for the operator of ``operator.apply`` (matrix-free transpose)."""
    lam = np.asarray(lam)
    M = lam.shape[0] - 1
    nx = lam.shape[1]
    gbo, gbn = GeoBar.zeros(nx, lam.dtype), GeoBar.zeros(nx, lam.dtype)
    zero = np.zeros_like(lam)
    Li = lam.copy()
    Li[0] = 0.0
    Li[M] = 0.0
    Gbx, Gbz = div_T(Li, zero, zero, g_new, gbn, M)
    bx, bz, _ = _bed_rows_T(lam, zero, g_old.hx, M)
    out = grad_T(Gbx + bx, Gbz + bz, zero, g_old, gbo, M)
    out[0] += lam[0]
    return out


def solve_T_dense(c, g_old, g_new):
    """lam = A^-T c by LU of the dense assembled matrix."""
    c = np.asarray(c)
    M = c.shape[0] - 1
    A = op.assemble(c.shape[1], M, g_old, g_new)
    return sla.lu_solve(sla.lu_factor(A), c.ravel(), trans=1).reshape(c.shape)


def operator_metric_T(lam, P, g_old, g_new, gbo, gbn):
    """Accumulate the adjoint of the metrics in lam^T A(metrics) P into gbo, gbn; returns the
    adjoint of h_x from the bed row."""
    M = P.shape[0] - 1
    Gx, Gz = op.grad(P, g_old, M)
    Li = lam.copy()
    Li[0] = 0.0
    Li[M] = 0.0
    Gbx, Gbz = div_T(Li, Gx, Gz, g_new, gbn, M)
    bx, bz, hxb = _bed_rows_T(lam, Gx, g_old.hx, M)
    grad_T(Gbx + bx, Gbz + bz, P, g_old, gbo, M)
    return hxb


def geometry_T(gb, hxb, g):
    """(hbar, etabar) from the metric adjoints gb of g = Geometry(h, eta) and a direct adjoint
    hxb of h_x."""
    d, hx, dxd, i = g.d, g.hx, g.dxd, g.inv_d
    hxt = gb.a * i + hxb
    dxdb = -gb.b * i
    db = -(gb.a * hx) * i * i + (gb.b * dxd) * i * i - gb.i * i * i + dxT(dxdb, g.L)
    hb = db + dxT(hxt, g.L)
    return hb, db


# ----------------------------------------------------------------------------- the stage
@dataclass
class Tape:
    """Forward intermediates of one stage, recomputed from the stage's input state."""
    k: int
    a: float
    beta: float
    dt: float
    u: np.ndarray
    w: np.ndarray
    eta: np.ndarray
    Ku: np.ndarray
    Kw: np.ndarray
    eta_t: np.ndarray
    g_old: object
    g_new: object
    us: np.ndarray
    ws: np.ndarray
    p: np.ndarray
    extra: dict = field(default_factory=dict)


def stage_tape(k, dt, h, L, s, ph=None):
    """Run the forward stage on a copy of s with dense solves and record what the adjoint needs."""
    ph = ph or lserk.Physics()
    a, beta = lserk.ALPHA[k - 1], lserk.BETA[k - 1]
    g_old = op.Geometry(h, s.eta, L)
    eta_t = -s.u[0] * sp.dx(s.eta, L) + s.w[0]
    Keta = a * s.Keta + dt * eta_t
    eta_new = sp.filter_x(s.eta + beta * Keta, L, ph.filt_fx, ph.filt_alpha, ph.filt_s)
    g_new = op.Geometry(h, eta_new, L)
    Fu, Fw = lserk.forcing(s.u, s.w, s.eta, eta_t, g_old, ph)
    us = s.u + beta * (a * s.Ku + dt * Fu)
    ws = s.w + beta * (a * s.Kw + dt * Fw)
    b = lserk.rhs(us, ws, g_new, g_old.hx, ph.rho / (beta * dt))
    p = op.solve_dense(b, g_old, g_new)
    return Tape(k, a, beta, dt, s.u, s.w, s.eta, s.Ku, s.Kw, eta_t, g_old, g_new, us, ws, p)


def forcing_T(Fub, Fwb, t, gbo, ph):
    """Adjoint of lserk.forcing at the tape's old stage: returns (ubar, wbar, etabar, eta_t bar);
    accumulates the old-geometry metric adjoints."""
    u, w, g = t.u, t.w, t.g_old
    M = u.shape[0] - 1
    L = g.L
    Ds = sp.dsig_matrix(M)
    sig = sp.cgl_sigma(M)
    sx = g.sigma_x(sig)
    idd = g.inv_d[None, :]
    st = -sig[:, None] * (t.eta_t * g.inv_d)[None, :]
    wsig = st + u * sx + w * idd
    ux, wx, us_, ws_ = sp.dx(u, L), sp.dx(w, L), Ds @ u, Ds @ w
    # -u D_x u, -u D_x w
    ub = -Fub * ux + sp.dx(u * Fub, L) - Fwb * wx
    wb = sp.dx(u * Fwb, L)
    # -w_sigma D_s u, -w_sigma D_s w
    wsb = -Fub * us_ - Fwb * ws_
    ub = ub + Ds.T @ (-wsig * Fub)
    wb = wb + Ds.T @ (-wsig * Fwb)
    # -g D_x eta (broadcast over rows)
    etab = ph.g * sp.dx(Fub.sum(axis=0), L)
    # nu Div Grad f on the old geometry, for f = u and f = w
    for f, Fb, acc in ((u, Fub, "u"), (w, Fwb, "w")):
        Gx, Gz = op.grad(f, g, M)
        Gbx, Gbz = div_T(ph.nu * Fb, Gx, Gz, g, gbo, M)
        fb = grad_T(Gbx, Gbz, f, g, gbo, M)
        if acc == "u":
            ub = ub + fb
        else:
            wb = wb + fb
    # w_sigma = sigma_t + u sigma_x + w / d, sigma_t = -sigma eta_t / d
    ub = ub + wsb * sx
    sigx_T(wsb * u, gbo, sig)
    wb = wb + wsb * idd
    gbo.i += (wsb * w).sum(axis=0)
    etatb = (-sig[:, None] * g.inv_d[None, :] * wsb).sum(axis=0)
    gbo.i += (-sig[:, None] * t.eta_t[None, :] * wsb).sum(axis=0)
    return ub, wb, etab, etatb


def stage_T(t, bar, h, L, ph=None):
    """Reverse one stage.

    bar: dict of adjoints of the stage outputs u, w, eta, Ku, Kw, Keta (p is not an output that
    later stages use). Returns (adjoints of the stage inputs as a dict, hbar contribution).
    """
    ph = ph or lserk.Physics()
    a, beta, dt = t.a, t.beta, t.dt
    M = t.u.shape[0] - 1
    nx = t.u.shape[1]
    Fs = sp.filter_sigma_matrix(M, ph.filt_fz, ph.filt_alpha, ph.filt_s)
    fx = lambda f: sp.filter_x(f, L, ph.filt_fx, ph.filt_alpha, ph.filt_s)
    g_old, g_new = t.g_old, t.g_new
    gbo, gbn = GeoBar.zeros(nx, t.u.dtype), GeoBar.zeros(nx, t.u.dtype)
    hxb = np.zeros(nx, dtype=t.u.dtype)
    scale = ph.rho / (beta * dt)
    # filters of u and w: u_out = Fs Fx (u + beta Ku_new)
    uh = fx(Fs.T @ bar["u"])
    wh = fx(Fs.T @ bar["w"])
    ub, wb = uh.copy(), wh.copy()
    Kun_b = bar["Ku"] + beta * uh
    Kwn_b = bar["Kw"] + beta * wh
    # Ku_new = a Ku + dt (Fu - Gx / rho)
    Kub = a * Kun_b
    Kwb = a * Kwn_b
    Fub = dt * Kun_b
    Fwb = dt * Kwn_b
    Gbx = -(dt / ph.rho) * Kun_b
    Gbz = -(dt / ph.rho) * Kwn_b
    # (Gx, Gz) = Grad^old p
    pb = grad_T(Gbx, Gbz, t.p, g_old, gbo, M)
    # p = A^-1 b: lam = A^-T pbar; b gets lam; the metrics get -lam^T dA p
    lam = solve_T_dense(pb, g_old, g_new)
    gbo_m, gbn_m = GeoBar.zeros(nx, t.u.dtype), GeoBar.zeros(nx, t.u.dtype)
    hxb_m = operator_metric_T(lam, t.p, g_old, g_new, gbo_m, gbn_m)
    for gb, gm in ((gbo, gbo_m), (gbn, gbn_m)):
        gb.a -= gm.a
        gb.b -= gm.b
        gb.i -= gm.i
    hxb -= hxb_m
    # b = scale Div^new(u*, w*) inside, 0 at the surface, -scale (h_x u*_M + w*_M) at the bed
    Li = scale * lam
    Li[0] = 0.0
    Li[M] = 0.0
    usb, wsb = div_T(Li, t.us, t.ws, g_new, gbn, M)
    usb[M] += -scale * g_old.hx * lam[M]
    wsb[M] += -scale * lam[M]
    hxb += -scale * t.us[M] * lam[M]
    # u* = u + beta (a Ku + dt Fu)
    ub += usb
    wb += wsb
    Kub += beta * a * usb
    Kwb += beta * a * wsb
    Fub += beta * dt * usb
    Fwb += beta * dt * wsb
    # forcing on the old stage
    fu, fw, etab, etatb = forcing_T(Fub, Fwb, t, gbo, ph)
    ub += fu
    wb += fw
    # eta_new = Fx(eta + beta Keta_new): bar["eta"] is the adjoint of eta_new, plus the new
    # geometry's metrics
    hb_n, eta_new_b = geometry_T(gbn, np.zeros(nx, dtype=t.u.dtype), g_new)
    e1b = fx(bar["eta"] + eta_new_b)
    etab = etab + e1b
    Ketan_b = bar["Keta"] + beta * e1b
    # Keta_new = a Keta + dt eta_t
    Ketab = a * Ketan_b
    etatb = etatb + dt * Ketan_b
    # eta_t = -u[0] D_x eta + w[0]
    ub[0] += -sp.dx(t.eta, L) * etatb
    wb[0] += etatb
    etab = etab + dxT(-t.u[0] * etatb, L)
    # old geometry (h, eta)
    hb_o, eta_old_b = geometry_T(gbo, hxb, g_old)
    etab = etab + eta_old_b
    return dict(u=ub, w=wb, eta=etab, Ku=Kub, Kw=Kwb, Keta=Ketab), hb_o + hb_n


def run_forward(h, L, ic, dt, nsteps, ph=None, solve=lserk.dense_solver):
    """States at the input of every stage (list of lserk.State) and the final state."""
    s = lserk.State.rest_registers(ic["u"], ic["w"], ic["eta"])
    s = lserk.State(*(np.asarray(x, dtype=np.result_type(x, h)) for x in
                      (s.u, s.w, s.eta, s.Ku, s.Kw, s.Keta, s.p)))
    states = []
    for _ in range(nsteps):
        for k in range(1, 6):
            states.append(lserk.State(s.u.copy(), s.w.copy(), s.eta.copy(), s.Ku.copy(),
                                      s.Kw.copy(), s.Keta.copy(), s.p.copy()))
            lserk.stage(k, dt, h, L, s, solve, ph)
    return states, s


def probe_gradient(h, L, ic, dt, nsteps, probe, ph=None):
    """dJ/dh for J = eta[probe] after nsteps steps from the initial state ic (independent of h)."""
    states, _ = run_forward(h, L, ic, dt, nsteps, ph)
    nx = len(h)
    z2 = np.zeros_like(ic["u"], dtype=float)
    bar = dict(u=z2.copy(), w=z2.copy(), eta=np.zeros(nx), Ku=z2.copy(), Kw=z2.copy(),
               Keta=np.zeros(nx))
    bar["eta"][probe] = 1.0
    hb = np.zeros(nx)
    for idx in range(len(states) - 1, -1, -1):
        k = idx % 5 + 1
        t = stage_tape(k, dt, h, L, states[idx], ph)
        bar, hbs = stage_T(t, bar, h, L, ph)
        hb += hbs
    return hb

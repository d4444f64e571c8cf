"""Relaxation zones of the wave flume: the target fields of an incident stream-function wave on
the sigma grid, and the blend toward them (paper Sec. 5, harmonic generation over a submerged
bar: waves generated and absorbed by relaxation zones).

Oracle (test infrastructure only).

- ``stream_target``: the wave of coefficients [k, c, ubar, h0, x0, E_0..E_N, B_1..B_N] (the
  Fourier approximation of a steady wave, crest at x = x0 + c t) at time t: with X = x - x0 - c t,
  eta = a S(x) sum_q E_q cos(q k X); on the target's own sigma grid zeta_j = sigma_j (h0 + eta),
  u = a S ((c - ubar) + sum_q q k B_q cosh(q k zeta) / cosh(q k h0) cos(q k X)),
  w = a S sum_q q k B_q sinh(q k zeta) / cosh(q k h0) sin(q k X)
  (the stream function's velocities in the earth frame); a is a scalar ramp, S a window per
  column. The hyperbolic ratios are taken as exp(q k (zeta - h0)) (1 +- exp(-2 q k zeta)) /
  (1 + exp(-2 q k h0)) so that high modes do not overflow.
- ``relax``: q <- q + r (q_target - q) per column, on u and w (every row) and eta, once per time
  step after the five stages (the 2N registers K are multiplied by zero at the next step's first
  stage, so they need no blend).
"""
import numpy as np


def stream_target(coef, nmodes, x, sigma, t, a=1.0, S=None):
    k, c, ubar, h0, x0 = coef[:5]
    E = np.asarray(coef[5:6 + nmodes])
    B = np.asarray(coef[6 + nmodes:6 + 2 * nmodes])
    x = np.asarray(x, dtype=np.float64)
    S = np.ones_like(x) if S is None else np.asarray(S)
    X = x - x0 - c * t
    q = np.arange(nmodes + 1)
    eta = a * S * (np.cos(np.outer(X, q) * k) @ E)
    zeta = np.asarray(sigma)[:, None] * (h0 + eta)[None, :]        # [nz][nx]
    j = np.arange(1, nmodes + 1)
    kj = k * j
    up = np.exp(kj[None, None, :] * (zeta[..., None] - h0))
    em = np.exp(-2.0 * kj[None, None, :] * zeta[..., None])
    den = 1.0 + np.exp(-2.0 * kj * h0)
    ch = up * (1.0 + em) / den
    sh = up * (1.0 - em) / den
    cosX = np.cos(np.outer(X, kj))[None]
    sinX = np.sin(np.outer(X, kj))[None]
    u = a * S[None, :] * ((c - ubar) + np.sum(kj * B * ch * cosX, axis=-1))
    w = a * S[None, :] * np.sum(kj * B * sh * sinX, axis=-1)
    return u, w, eta


def relax(q, qt, r):
    """q + r (qt - q), r per column (broadcast over rows for 2D fields)."""
    return q + np.asarray(r) * (np.asarray(qt) - np.asarray(q))

"""Seeded synthetic workloads for the pressure Poisson solve and the RK time stepping.

This module generates inputs only: bathymetry h(x), surface elevation eta(x), right-hand sides and
initial fields, all from closed-form expressions evaluated at the grid nodes. It holds none of the
method's arithmetic (no derivative operators, no metrics, no solves), so the GPU path and the CPU
checker can both draw their inputs from it.

Fields are float64 arrays laid out [Nz][Nx]: row j sits at sigma_j = (1 + cos(j pi / M)) / 2
(row 0 = free surface, row M = bed), column i at x_i = i L / Nx.

The paper's own workloads (stream-function waves, the Beji-Battjes flume record) are not
available; the recipes below stand in for them with the same shapes, depths, wave steepnesses and
bathymetry types.
"""
import math

import numpy as np

G = 9.81
RHO = 1000.0


def nodes(nx, nz, L):
    """x_i and sigma_j of the grid on which every input below is sampled."""
    M = nz - 1
    x = np.arange(nx, dtype=np.float64) * (L / nx)
    sigma = 0.5 * (1.0 + np.cos(np.pi * np.arange(nz) / M))
    return x, sigma


def _phi(u):
    return np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def _Phi(u):
    from scipy.special import ndtr
    return ndtr(u)


def rest_rhs(h, hx, eta_x, eta_xx, nz):
    """Right-hand side of the first RK stage started from rest, from closed-form derivatives.

    From rest (u = w = K = 0) the provisional velocity is u* = -beta dt g eta_x, uniform in sigma,
    w* = 0, so the scaled divergence is -rho g eta_xx in the interior, 0 on the surface row and the
    bed-normal flux rho g h_x eta_x on the bed row.
    """
    nx = h.shape[0]
    b = np.empty((nz, nx))
    b[:] = -RHO * G * eta_xx[None, :]
    b[0] = 0.0
    b[nz - 1] = RHO * G * hx * eta_x
    return b


# ----------------------------------------------------------------------------- single problems

def manufactured(nx=32, nz=9, amp=0.05):
    """Flat bed h = 1, eta = amp cos x on L = 2 pi; exact p = cos x cosh(z + h) / cosh h.

    p is harmonic in (x, z) and has zero normal derivative on the flat bed, so the discrete problem
    has b = p on the surface row and 0 elsewhere.
    """
    L = 2.0 * math.pi
    x, sigma = nodes(nx, nz, L)
    h = np.ones(nx)
    eta = amp * np.cos(x)
    d = h + eta
    exact = np.cos(x)[None, :] * np.cosh(sigma[:, None] * d[None, :]) / math.cosh(1.0)
    b = np.zeros((nz, nx))
    b[0] = exact[0]
    return dict(name="manufactured", nx=nx, nz=nz, L=L, h=h, eta_old=eta, eta_new=eta.copy(),
                b=b, exact=exact)


def manufactured_sloped(nx=32, nz=9, amp=0.05, bed=0.15, kwave=1.0):
    """Sloped bed and wavy surface with a harmonic exact solution p = cos(k x) cosh(k (z + 1)).

    h = 1 - bed sin x, eta = amp cos x, L = 2 pi. Surface row: p at z = eta; interior rows: 0;
    bed row: the outward normal flux -(h_x p_x + p_z) at z = -h.
    """
    L = 2.0 * math.pi
    x, sigma = nodes(nx, nz, L)
    k = kwave
    h = 1.0 - bed * np.sin(x)
    hx = -bed * np.cos(x)
    eta = amp * np.cos(x)
    d = h + eta
    z = sigma[:, None] * d[None, :] - h[None, :]
    exact = np.cos(k * x)[None, :] * np.cosh(k * (z + 1.0))
    zb = -h
    px = -k * np.sin(k * x) * np.cosh(k * (zb + 1.0))
    pz = k * np.cos(k * x) * np.sinh(k * (zb + 1.0))
    b = np.zeros((nz, nx))
    b[0] = exact[0]
    b[nz - 1] = -(hx * px + pz)
    return dict(name="manufactured_sloped", nx=nx, nz=nz, L=L, h=h, eta_old=eta,
                eta_new=eta.copy(), b=b, exact=exact)


def manufactured3d(nx=16, ny=16, nz=9, amp=0.05, bed=0.15, kx=1.0, ky=1.0):
    """3D tank (x, y periodic on 2 pi x 2 pi) with a sloped bed and a wavy surface, and the
    harmonic exact solution p = cos(kx x) cos(ky y) cosh(k (z + 1)), k = sqrt(kx^2 + ky^2).

    h = 1 - bed sin x cos y, eta = amp cos x cos y. Surface row: p at z = eta; interior rows: 0;
    bed row: the outward normal flux -(h_x p_x + h_y p_y + p_z) at z = -h. Fields [nz][ny][nx].
    """
    L = 2.0 * math.pi
    x = np.arange(nx) * L / nx
    y = np.arange(ny) * L / ny
    X, Y = np.meshgrid(x, y)
    sigma = 0.5 * (1.0 + np.cos(np.arange(nz) * math.pi / (nz - 1)))
    k = math.hypot(kx, ky)
    h = 1.0 - bed * np.sin(X) * np.cos(Y)
    hx = -bed * np.cos(X) * np.cos(Y)
    hy = bed * np.sin(X) * np.sin(Y)
    eta = amp * np.cos(X) * np.cos(Y)
    d = h + eta
    z = sigma[:, None, None] * d[None] - h[None]
    exact = np.cos(kx * X)[None] * np.cos(ky * Y)[None] * np.cosh(k * (z + 1.0))
    zb = -h
    px = -kx * np.sin(kx * X) * np.cos(ky * Y) * np.cosh(k * (zb + 1.0))
    py = -ky * np.cos(kx * X) * np.sin(ky * Y) * np.cosh(k * (zb + 1.0))
    pz = k * np.cos(kx * X) * np.cos(ky * Y) * np.sinh(k * (zb + 1.0))
    b = np.zeros((nz, ny, nx))
    b[0] = exact[0]
    b[nz - 1] = -(hx * px + hy * py + pz)
    return dict(name="manufactured3d", nx=nx, ny=ny, nz=nz, Lx=L, Ly=L, h=h, eta_old=eta,
                eta_new=eta.copy(), b=b, exact=exact)


def airy_pressure(nx=16, nz=17, depth=1.0, amp=1e-3, mode=2):
    """Linear (Airy) pressure problem on a flat geometry (surface held at z = 0).

    The right-hand side comes from a surface eta = amp cos(k x) through the from-rest stage:
    b = -rho g eta_xx inside, 0 on both boundary rows; the exact dynamic pressure is
    rho g amp cos(k x) [cosh(k (z + h)) / cosh(k h) - 1].
    """
    L = 2.0 * math.pi
    x, sigma = nodes(nx, nz, L)
    k = float(mode)
    h = np.full(nx, depth)
    eta_geom = np.zeros(nx)
    eta = amp * np.cos(k * x)
    b = rest_rhs(h, np.zeros(nx), -amp * k * np.sin(k * x), -amp * k * k * np.cos(k * x), nz)
    z = sigma[:, None] * depth - depth
    exact = RHO * G * amp * np.cos(k * x)[None, :] * (np.cosh(k * (z + depth)) / math.cosh(k * depth) - 1.0)
    return dict(name="airy_pressure", nx=nx, nz=nz, L=L, h=h, eta_old=eta_geom,
                eta_new=eta_geom.copy(), b=b, exact=exact, eta_wave=eta)


def bar(seed=0, nx=1024, nz=33):
    """Trapezoidal submerged bar, first RK stage from rest (single geometry).

    Depth 0.4; from x0 = L/4 a 1:20 up-slope to 0.1 over 6 m, a 2 m crest, a 1:10 down-slope over
    3 m, then flat. The corners are mollified with a Gaussian of width 0.1 m in closed form
    (h = h0 + sum_i dm_i s G((x - x_i)/s), G(u) = u Phi(u) + phi(u)), which keeps h smooth and
    periodic. The seed draws kh in [0.5, 2] (w.r.t. h0), L = lambda ceil(30/lambda), a phase, and a
    band-limited noise field (modes up to nx/4) of 1 % of the amplitude; H = 0.05 h0.
    """
    rng = np.random.default_rng(seed)
    h0, sg = 0.4, 0.1
    kh = rng.uniform(0.5, 2.0)
    k = kh / h0
    lam = 2.0 * math.pi / k
    L = lam * math.ceil(30.0 / lam)
    ph = rng.uniform(0.0, 2.0 * math.pi)
    H = 0.05 * h0
    x, _ = nodes(nx, nz, L)
    x0 = L / 4.0
    br = np.array([x0, x0 + 6.0, x0 + 8.0, x0 + 11.0])
    dm = np.array([-0.05, 0.05, 0.1, -0.1])
    u = (x[None, :] - br[:, None]) / sg
    h = h0 + np.sum(dm[:, None] * sg * (u * _Phi(u) + _phi(u)), axis=0)
    hx = np.sum(dm[:, None] * _Phi(u), axis=0)
    eta = (H / 2.0) * np.cos(k * x + ph)
    eta_x = -(H / 2.0) * k * np.sin(k * x + ph)
    eta_xx = -(H / 2.0) * k * k * np.cos(k * x + ph)
    nmodes = nx // 4
    m = np.arange(1, nmodes + 1)
    km = 2.0 * math.pi * m / L
    std = 0.01 * H / 2.0
    ca = rng.standard_normal(nmodes) * std / math.sqrt(nmodes)
    cb = rng.standard_normal(nmodes) * std / math.sqrt(nmodes)
    arg = np.outer(km, x)
    eta = eta + ca @ np.cos(arg) + cb @ np.sin(arg)
    eta_x = eta_x + (-ca * km) @ np.sin(arg) + (cb * km) @ np.cos(arg)
    eta_xx = eta_xx - (ca * km * km) @ np.cos(arg) - (cb * km * km) @ np.sin(arg)
    b = rest_rhs(h, hx, eta_x, eta_xx, nz)
    return dict(name=f"bar_s{seed}", nx=nx, nz=nz, L=L, h=h, eta_old=eta, eta_new=eta.copy(), b=b,
                kh=kh)


def tank(rng, nx, nz):
    """One random tank of the batched workload (first stage from rest, single geometry)."""
    hbar = rng.uniform(0.5, 2.0)
    L = 8.0 * math.pi * hbar
    x, _ = nodes(nx, nz, L)
    K = 2.0 * math.pi / L
    if rng.uniform() < 0.5:
        h = np.full(nx, hbar)
        hx = np.zeros(nx)
    else:
        Ah = rng.uniform(0.5, 1.0) * min(0.1 * L / (2.0 * math.pi), hbar - 0.5, 2.0 - hbar)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        h = hbar + Ah * np.cos(K * x + ph)
        hx = -Ah * K * np.sin(K * x + ph)
    m = int(rng.integers(2, 9))
    a = rng.uniform(0.01, 0.08) * hbar
    phe = rng.uniform(0.0, 2.0 * math.pi)
    km = m * K
    eta = a * np.cos(km * x + phe)
    eta_x = -a * km * np.sin(km * x + phe)
    eta_xx = -a * km * km * np.cos(km * x + phe)
    b = rest_rhs(h, hx, eta_x, eta_xx, nz)
    return dict(nx=nx, nz=nz, L=L, h=h, eta_old=eta, eta_new=eta.copy(), b=b)


def batch(seed=0, ntanks=512, nx_choices=(64, 128, 256, 512), nz_choices=(9, 17, 33)):
    """Many independent tanks of uneven (Nx, Nz): depth in [0.5, 2], L = 8 pi hbar, flat or cosine
    beds (slope <= 1:10), surface amplitude in [0.01, 0.08] hbar with kh = m/4 in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    tanks = []
    for _ in range(ntanks):
        nx = int(rng.choice(nx_choices))
        nz = int(rng.choice(nz_choices))
        tanks.append(tank(rng, nx, nz))
    return tanks


# ----------------------------------------------------------------------------- time stepping

def stokes_wave(nx=256, nz=17, depth=1.0, k=1.0, steep=0.05, cfl=0.5):
    """Second-order Stokes wave initial state on a flat bed (periodic, one wavelength per L).

    eta = (H/2) cos(kx) + (k H^2/16) cosh(kh)(2 + cosh 2kh)/sinh^3(kh) cos(2kx);
    phi = (g H / 2w) cosh(k(z+h))/cosh(kh) sin(kx) + (3 H^2 w / 32) cosh(2k(z+h))/sinh^4(kh) sin(2kx),
    u = phi_x, w = phi_z at the nodes z_ij = sigma_j d_i - h; w^2 = g k tanh(kh), H = steep * L,
    dt = cfl * dx / c with c = w / k.
    """
    L = 2.0 * math.pi / k
    H = steep * L
    x, sigma = nodes(nx, nz, L)
    kh = k * depth
    om = math.sqrt(G * k * math.tanh(kh))
    h = np.full(nx, depth)
    eta = (H / 2.0) * np.cos(k * x) + (k * H * H / 16.0) * math.cosh(kh) * (2.0 + math.cosh(2 * kh)) \
        / math.sinh(kh) ** 3 * np.cos(2 * k * x)
    d = h + eta
    z = sigma[:, None] * d[None, :] - h[None, :]
    zp = z + depth
    a1 = G * H / (2.0 * om) / math.cosh(kh)
    a2 = 3.0 * H * H * om / 32.0 / math.sinh(kh) ** 4
    X = x[None, :]
    u = a1 * k * np.cosh(k * zp) * np.cos(k * X) + a2 * 2 * k * np.cosh(2 * k * zp) * np.cos(2 * k * X)
    w = a1 * k * np.sinh(k * zp) * np.sin(k * X) + a2 * 2 * k * np.sinh(2 * k * zp) * np.sin(2 * k * X)
    c = om / k
    dt = cfl * (L / nx) / c
    return dict(name="stokes", nx=nx, nz=nz, L=L, h=h, eta=eta, u=u, w=w, dt=dt, omega=om, H=H)


def stokes_rest_problem(nx=256, nz=17):
    """A single Poisson problem at the Stokes-wave geometry, first stage from rest."""
    s = stokes_wave(nx, nz)
    L, H, k = s["L"], s["H"], 2.0 * math.pi / s["L"]
    x, _ = nodes(nx, nz, L)
    kh = k
    a2 = (k * H * H / 16.0) * math.cosh(kh) * (2.0 + math.cosh(2 * kh)) / math.sinh(kh) ** 3
    eta_x = -(H / 2.0) * k * np.sin(k * x) - a2 * 2 * k * np.sin(2 * k * x)
    eta_xx = -(H / 2.0) * k * k * np.cos(k * x) - a2 * 4 * k * k * np.cos(2 * k * x)
    b = rest_rhs(s["h"], np.zeros(nx), eta_x, eta_xx, nz)
    return dict(name="stokes_rest", nx=nx, nz=nz, L=L, h=s["h"], eta_old=s["eta"],
                eta_new=s["eta"].copy(), b=b)


def airy_wave(nx=16, nz=9, depth=1.0, k=1.0, amp=1e-6, cfl=0.5):
    """Small-amplitude (linear) progressive wave eta = a cos(kx), u = a w cosh(k(z+h))/sinh(kh)
    cos(kx), w = a w sinh(k(z+h))/sinh(kh) sin(kx) at t = 0 with w^2 = g k tanh(kh); periodic
    L = 2 pi / k, flat bed. Also returns the period and dt = cfl dx / c."""
    L = 2.0 * math.pi / k
    x, sigma = nodes(nx, nz, L)
    om = math.sqrt(G * k * math.tanh(k * depth))
    h = np.full(nx, depth)
    eta = amp * np.cos(k * x)
    d = h + eta
    z = sigma[:, None] * d[None, :] - h[None, :]
    zp = z + depth
    u = amp * om * np.cosh(k * zp) / math.sinh(k * depth) * np.cos(k * x)[None, :]
    w = amp * om * np.sinh(k * zp) / math.sinh(k * depth) * np.sin(k * x)[None, :]
    c = om / k
    return dict(name="airy", nx=nx, nz=nz, L=L, h=h, eta=eta, u=u, w=w, omega=om,
                period=2.0 * math.pi / om, dt=cfl * (L / nx) / c, amp=amp, k=k)


def stokes_layer(nx=64, nz=33, depth=0.1, H=0.02, kh=0.6725, nu=1e-6, steps_per_period=40):
    """Oscillatory wave boundary layer over a no-slip flat bed (linear wave, periodic domain).

    One wavelength per domain, k h = 0.6725 and H = 0.02 m as in the paper's boundary-layer case;
    the depth (not stated there) is 0.1 m so that at 33 sigma rows two nodes lie inside the layer
    thickness 3 pi delta_1 / 4. The wave is a single Fourier mode; Nx = 64 (the paper uses 20)
    meets the solver's Nx >= 2 (Nz - 1). With theta = omega t - k x, zeta = z + h the height above the bed,
    delta_1 = (2 nu / omega)^(1/2) and U_0m = pi H / (T sinh kh) the outer velocity amplitude at
    the bed, ``exact(t)`` gives the linear potential wave with the Stokes-layer correction
    (``exact(t, layer=False)`` the potential wave alone)
        u = (pi H / T) cosh(k zeta) / sinh(kh) cos(theta) - U_0m exp(-zeta/delta_1) cos(theta - zeta/delta_1),
        w = -(pi H / T) sinh(k zeta) / sinh(kh) sin(theta),  eta = (H/2) cos(k x - omega t)
    (the boundary-layer solution of small-amplitude wave theory; the bed amplitude of the printed
    U_0m is used). The initial state is exact(0) with u = w = 0 on the bed row; dt = T /
    steps_per_period.
    """
    k = kh / depth
    L = 2.0 * math.pi / k
    om = math.sqrt(G * k * math.tanh(kh))
    T = 2.0 * math.pi / om
    d1 = math.sqrt(2.0 * nu / om)
    U0m = math.pi * H / (T * math.sinh(kh))
    x, sigma = nodes(nx, nz, L)
    zeta = sigma[:, None] * depth * np.ones((1, nx))

    def exact(t, layer=True):
        th = om * t - k * x[None, :]
        u = (math.pi * H / T) * np.cosh(k * zeta) / math.sinh(kh) * np.cos(th)
        if layer:
            u = u - U0m * np.exp(-zeta / d1) * np.cos(th - zeta / d1)
        w = -(math.pi * H / T) * np.sinh(k * zeta) / math.sinh(kh) * np.sin(th)
        return u, w, (H / 2.0) * np.cos(k * x - om * t)

    u, w, eta = exact(0.0)
    u[-1] = 0.0
    w[-1] = 0.0
    return dict(name="stokes_layer", nx=nx, nz=nz, L=L, h=np.full(nx, depth), u=u, w=w, eta=eta,
                dt=T / steps_per_period, T=T, omega=om, k=k, delta1=d1, U0m=U0m, nu=nu,
                zeta=zeta, exact=exact)


def stream_function_wave(H, depth, period=None, length=None, N=24, current="euler", iters=40,
                         tol=1e-13):
    """Steady nonlinear wave of height H on depth h by the Fourier approximation method of
    Rienecker and Fenton (1981), from either the period or the wavelength. current: "euler" =
    Stokes' first definition of the wave speed (zero mean Eulerian current, c = ubar), "mass" =
    the second (zero mean mass transport, c = Q / h, as in a closed flume).

    In the frame moving with the wave (X = x - c t, zeta = z + h) the stream function is
        psi = -ubar zeta + sum_{j=1..N} B_j sinh(j k zeta) / cosh(j k h) cos(j k X),
    so the bed is the streamline psi = 0 and the relative velocities are U = psi_zeta,
    W = -psi_X; at the N + 1 collocation points X_m = m L / (2N) on half a wavelength the surface
    zeta = h + eta_m is the streamline psi = -Q and satisfies Bernoulli,
    (U^2 + W^2) / 2 + g eta_m = R; the mean of eta is zero, eta_0 - eta_N = H, and k c T = 2 pi
    (period given) or k = 2 pi / L (wavelength given). Newton's method on these 2N + 5 equations
    from the linear wave. Earth-frame velocities: u = c + U, w = W. Returns k, c, ubar, Q, R,
    B (j = 1..N), the surface cosine coefficients E (j = 0..N) and the collocation surface eta_m,
    plus the largest residual.
    """
    g = G
    h = float(depth)
    if length is not None:
        k0 = 2.0 * math.pi / length
    else:
        om = 2.0 * math.pi / period
        k0 = om * om / g
        for _ in range(200):                       # linear dispersion relation
            k0 = k0 - (g * k0 * math.tanh(k0 * h) - om * om) / (
                g * math.tanh(k0 * h) + g * k0 * h / math.cosh(k0 * h) ** 2)
    c0 = math.sqrt(g / k0 * math.tanh(k0 * h))
    m = np.arange(N + 1)
    j = np.arange(1, N + 1)
    # unknowns: [k, ubar, Q, R, B_1..B_N, eta_0..eta_N]
    x = np.zeros(2 * N + 5)
    x[0], x[1], x[2], x[3] = k0, c0, c0 * h, 0.5 * c0 * c0
    x[4] = c0 * (H / 2.0) / math.tanh(k0 * h)
    x[4 + N:] = (H / 2.0) * np.cos(math.pi * m / N)

    def residual(x):
        k, ub, Q, R = x[0], x[1], x[2], x[3]
        B, eta = x[4:4 + N], x[4 + N:]
        kX = np.outer(math.pi * m / N, j)          # j k X_m with X_m = m L / (2N)
        zeta = h + eta
        jkz = np.outer(zeta, j) * k
        ch = np.cosh(j * k * h)
        S = np.sinh(jkz) / ch
        C = np.cosh(jkz) / ch
        psi = -ub * zeta + (S * np.cos(kX)) @ B
        U = -ub + (C * np.cos(kX)) @ (j * k * B)
        W = (S * np.sin(kX)) @ (j * k * B)
        f = np.empty_like(x)
        f[:N + 1] = psi + Q
        f[N + 1:2 * N + 2] = 0.5 * (U * U + W * W) + g * eta - R
        wts = np.ones(N + 1)
        wts[0] = wts[-1] = 0.5
        f[2 * N + 2] = (wts @ eta) / N
        f[2 * N + 3] = eta[0] - eta[-1] - H
        cw = ub if current == "euler" else Q / h
        f[2 * N + 4] = (k * cw * period - 2.0 * math.pi) if length is None else (k - k0)
        return f

    res = np.inf
    for _ in range(iters):
        f = residual(x)
        res = float(np.abs(f).max())
        if res < tol:
            break
        J = np.empty((x.size, x.size))
        for q in range(x.size):
            d = 1e-7 * max(1.0, abs(x[q]))
            xp = x.copy()
            xp[q] += d
            xm = x.copy()
            xm[q] -= d
            J[:, q] = (residual(xp) - residual(xm)) / (2.0 * d)
        x = x - np.linalg.solve(J, f)
    k, ub, Q, R = x[0], x[1], x[2], x[3]
    c = ub if current == "euler" else Q / h
    B, eta = x[4:4 + N].copy(), x[4 + N:].copy()
    # cosine coefficients of the surface through the N + 1 points (trapezoidal DCT-I)
    wts = np.ones(N + 1)
    wts[0] = wts[-1] = 0.5
    E = np.array([(2.0 / N) * np.sum(wts * eta * np.cos(math.pi * q * m / N))
                  for q in range(N + 1)])
    E[0] *= 0.5
    E[N] *= 0.5
    return dict(k=float(k), c=float(c), ubar=float(ub), Q=float(Q), R=float(R), B=B, E=E,
                eta_m=eta, H=H, depth=h, L=2.0 * math.pi / float(k),
                T=2.0 * math.pi / (float(k) * float(c)), residual=res, N=N)


def smooth_ramp(chi):
    """0 at chi <= 0, 1 at chi >= 1, chi^3 (10 - 15 chi + 6 chi^2) between (zero slope and
    curvature at both ends)."""
    c = np.clip(chi, 0.0, 1.0)
    return c * c * c * (10.0 - 15.0 * c + 6.0 * c * c)


def flume_zones(x, length, zone, ext=None):
    """Relaxation strength r(x) and target window S(x) of a periodic flume (paper Sec. 5,
    harmonic generation over a submerged bar: generation and absorption zones of one wavelength,
    the generation zone carried on past the right end so that the periodic domain stays smooth).

    - generation zone [0, zone): S = 1, r falls from 1 at x = 0 to 0 at x = zone;
    - absorption zone [length - ext - zone, length - ext): S = 0 (still water), r rises 0 -> 1;
    - extension [length - ext, length): r = 1, S rises 0 -> 1, meeting the generation zone's
      fully relaxed end at the periodic seam (ext = zone / 2 unless given).
    """
    ext = 0.5 * zone if ext is None else ext
    x = np.asarray(x, dtype=np.float64)
    r = np.zeros_like(x)
    S = np.zeros_like(x)
    g = x < zone
    r[g] = 1.0 - smooth_ramp(x[g] / zone)
    S[g] = 1.0
    a0 = length - ext - zone
    a = (x >= a0) & (x < length - ext)
    r[a] = smooth_ramp((x[a] - a0) / zone)
    e = x >= length - ext
    r[e] = 1.0
    S[e] = smooth_ramp((x[e] - (length - ext)) / ext)
    return r, S


def stream_coef(sf, x0=0.0):
    """Packed coefficients of a stream-function wave for the target evaluation:
    [k, c, ubar, h0, x0, E_0..E_N, B_1..B_N] (crest at x = x0 + c t)."""
    return np.concatenate([[sf["k"], sf["c"], sf["ubar"], sf["depth"], x0], sf["E"], sf["B"]])


def flat_flume(nx=128, nz=17, waves=4, H=0.02, depth=0.4, period=2.02, steps_per_period=40):
    """Periodic flat flume of `waves` wavelengths with zones of one wavelength (flume_zones),
    still water at t = 0, incident stream-function wave (zero mass transport) ramped in over two
    periods. Returns the tank dict of the stepping tests plus r, S, coef, T and dt."""
    sf = stream_function_wave(H, depth, period=period, current="mass")
    L = waves * sf["L"]
    x, _ = nodes(nx, nz, L)
    r, S = flume_zones(x, L, sf["L"])
    z = np.zeros((nz, nx))
    return dict(name="flat_flume", nx=nx, nz=nz, L=L, h=np.full(nx, depth), u=z, w=z.copy(),
                eta=np.zeros(nx), r=r, S=S, coef=stream_coef(sf), nmodes=sf["N"], sf=sf,
                T=period, dt=period / steps_per_period)


def bar_flume(nx=1024, nz=33, H=0.02, period=2.02, steps_per_period=200):
    """The submerged-bar flume (paper Sec. 5, harmonic generation over a submerged bar): depth
    0.4 m, a 1:20 slope up to 0.1 m over 6 m, a 2 m crest, a 1:10 slope down over 3 m (corners
    mollified as in ``bar``), in a periodic domain of ten incident wavelengths with the
    generation zone at the left (the bar starts 6 m past it) and the absorption zone before the
    right end (flume_zones); still water at t = 0 and the stream-function wave (H = 0.02 m,
    T = 2.02 s, zero mass transport) ramped in over two periods."""
    h0, sg = 0.4, 0.1
    sf = stream_function_wave(H, h0, period=period, current="mass")
    L = 10.0 * sf["L"]
    x, _ = nodes(nx, nz, L)
    x0 = sf["L"] + 6.0
    br = np.array([x0, x0 + 6.0, x0 + 8.0, x0 + 11.0])
    dm = np.array([-0.05, 0.05, 0.1, -0.1])
    u = (x[None, :] - br[:, None]) / sg
    h = h0 + np.sum(dm[:, None] * sg * (u * _Phi(u) + _phi(u)), axis=0)
    r, S = flume_zones(x, L, sf["L"])
    z = np.zeros((nz, nx))
    return dict(name="bar_flume", nx=nx, nz=nz, L=L, h=h, u=z, w=z.copy(), eta=np.zeros(nx),
                r=r, S=S, coef=stream_coef(sf), nmodes=sf["N"], sf=sf, T=period,
                dt=period / steps_per_period)


def ramp_in(t, T):
    """Amplitude factor of the incident wave: smooth_ramp over the first two periods."""
    return float(smooth_ramp(np.array(t / (2.0 * T))))

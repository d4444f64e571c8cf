"""GPU parity of the stage's model options, the linearised equations (eq. NSElin, eq. linFS) and
the no-slip bed (paper Sec. 5, oscillatory wave boundary layer), through rk4_stage in the C ABI,
against the oracle; and the oscillatory boundary layer on the GPU against its closed form.

Parity tolerances are those of the default stage (relative to each field's max norm): eta 1e-12;
u, w, K_u, K_w, K_eta 1e-9; p 1e-8 (both sides solve to 1e-12 and below), raised where the
discrete problem's own rounding floor is above them: at 64 x 33 the pressure solve stalls at a
relative residual of ~4e-13 (any solver, either precision of the cycle), which the operator's
conditioning turns into ~5e-9 in p and, through G_x, G_z and the stages, up to ~2e-7 in K. The
floor is measured on the CPU as the disagreement of the oracle's two solvers (dense LU and
p-multigrid FGMRES at 1e-12) on the same stage, and the bound per field is
max(default tolerance, 10 x floor). The closed-form bound is the oracle's own pin: 3 % of the
outer bed velocity amplitude U_0m on the nodes within 6 delta_1 of the bed (the oracle reaches
0.8 % after half a period, 1.3 % after one).
"""
import copy

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import krylov
from oracle import lserk
from oracle import operator as op
from oracle import pmg
from oracle import spectral as sp
from paper_2406_00991_amd import workloads as wl

pytestmark = pytest.mark.gpu


class Tank:
    def __init__(self, t, precision, **optkw):
        import torch
        from paper_2406_00991_amd import pmgw
        self.pmgw, self.t = pmgw, t
        self.plan = pmgw.Plan([t["nx"]], [t["nz"]], [t["L"]], precision=precision,
                              opts=pmgw.default_opts(**optkw))
        dev = lambda a: torch.tensor(np.asarray(a).ravel(), dtype=torch.float64, device="cuda")
        self.h, self.u, self.w, self.eta = dev(t["h"]), dev(t["u"]), dev(t["w"]), dev(t["eta"])
        self.Ku, self.Kw = torch.zeros_like(self.u), torch.zeros_like(self.u)
        self.Keta, self.p = torch.zeros_like(self.eta), torch.zeros_like(self.u)
        self.info = pmgw.info_buffer(1)

    def stage(self, k, dt, rtol=1e-12):
        self.pmgw.rk4_stage(self.plan, k, dt, self.h, self.u, self.w, self.eta, self.Ku, self.Kw,
                            self.Keta, self.p, rtol=rtol, maxit=300, info_dev=self.info)
        assert self.pmgw.read_info(self.info)[0]["status"] == 0

    def fields(self):
        shp = (self.t["nz"], self.t["nx"])
        two = {k: getattr(self, k).cpu().numpy().reshape(shp) for k in ("u", "w", "Ku", "Kw", "p")}
        one = {k: getattr(self, k).cpu().numpy() for k in ("eta", "Keta")}
        return {**two, **one}


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


TOL = dict(eta=1e-12, u=1e-9, w=1e-9, Ku=1e-9, Kw=1e-9, Keta=1e-9, p=1e-8)


def compare(got, s, floor=None):
    for key, tol in TOL.items():
        bound = max(tol, 10.0 * floor[key]) if floor else tol
        err = relerr(got[key], getattr(s, key))
        assert err <= bound, (key, err, bound)


def fgmres_solver(rtol):
    def solve(b, g_old, g_new, p0):
        H = pmg.Hierarchy(b.shape[1], b.shape[0] - 1, g_old, g_new, pmg.PmgOptions())
        x, info = krylov.fgmres(lambda v: op.apply(v, g_old, g_new), b, H, x0=p0, rtol=rtol,
                                restart=30, maxit=300)
        return x
    return solve


def fixed_solver(t):
    M = t["nz"] - 1
    g = op.Geometry(t["h"], np.zeros(t["nx"]), t["L"])
    lu = sla.lu_factor(op.assemble(t["nx"], M, g, g))
    return lambda b, go, gn, p0: sla.lu_solve(lu, b.ravel()).reshape(b.shape)


def layer_case():
    return wl.stokes_layer(64, 33), dict(nu_visc=1e-6, filt_fx=1.0, filt_fz=1.0, linear=1,
                                         no_slip=1)


def sloped_case(no_slip, linear, nu):
    t = dict(wl.stokes_wave(32, 17, steep=0.03))
    t["h"] = t["h"] + 0.05 * np.sin(sp.x_nodes(32, t["L"]))
    if no_slip:
        t["u"], t["w"] = t["u"].copy(), t["w"].copy()
        t["u"][-1] = 0.0
        t["w"][-1] = 0.0
    return t, dict(nu_visc=nu, linear=linear, no_slip=no_slip)


def physics(opts):
    return lserk.Physics(nu=opts["nu_visc"], filt_fx=opts.get("filt_fx", 0.5),
                         filt_fz=opts.get("filt_fz", 0.9), linear=bool(opts["linear"]),
                         no_slip=bool(opts["no_slip"]))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_linear_no_slip_layer_stage_parity(precision):
    """Two steps of the 64 x 33 boundary-layer workload; every stage is compared."""
    t, o = layer_case()
    G = Tank(t, precision, **o)
    s = lserk.State.rest_registers(t["u"], t["w"], t["eta"])
    s2 = copy.deepcopy(s)
    ph, solve, solve2 = physics(o), fixed_solver(t), fgmres_solver(1e-12)
    for _ in range(2):
        for k in range(1, 6):
            G.stage(k, t["dt"])
            lserk.stage(k, t["dt"], t["h"], t["L"], s, solve, ph)
            lserk.stage(k, t["dt"], t["h"], t["L"], s2, solve2, ph)
            floor = {key: relerr(getattr(s2, key), getattr(s, key)) for key in TOL}
            compare(G.fields(), s, floor)


@pytest.mark.parametrize("no_slip,linear", [(1, 0), (0, 1), (1, 1)])
def test_model_options_on_a_sloped_bed(no_slip, linear):
    """One step of a 32 x 17 wave over a sloped bed with the default filters and a viscosity of
    1e-3 (large enough that the surface-row and bed-row treatments change the result)."""
    t, o = sloped_case(no_slip, linear, 1e-3)
    G = Tank(t, "fp64", **o)
    s = lserk.State.rest_registers(t["u"], t["w"], t["eta"])
    ph = physics(o)
    solve = fixed_solver(t) if linear else lserk.dense_solver
    for k in range(1, 6):
        G.stage(k, t["dt"])
        lserk.stage(k, t["dt"], t["h"], t["L"], s, solve, ph)
    got = G.fields()
    compare(got, s)
    if no_slip:
        for key in ("u", "w", "Ku", "Kw"):
            assert np.all(got[key][-1] == 0.0), key


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stokes_layer_matches_closed_form(precision):
    """One wave period (40 steps, solves to 1e-10 as in the stepping benchmark) on the GPU: the
    near-bed velocity profile against the closed-form oscillatory boundary layer."""
    t, o = layer_case()
    G = Tank(t, precision, **o)
    n = int(round(t["T"] / t["dt"]))
    for _ in range(n):
        for k in range(1, 6):
            G.stage(k, t["dt"], rtol=1e-10)
    got = G.fields()
    ue, _, _ = t["exact"](n * t["dt"])
    near = t["zeta"][:, 0] < 6 * t["delta1"]
    assert near.sum() >= 4
    err = np.abs(got["u"][near] - ue[near]).max() / t["U0m"]
    assert err <= 0.03, err
    assert np.all(got["u"][-1] == 0.0) and np.all(got["w"][-1] == 0.0)


def test_adjoint_stage_refuses_model_options():
    import torch
    from paper_2406_00991_amd import pmgw
    t, o = layer_case()
    G = Tank(t, "fp64", **o)
    state = dict(u=G.u, w=G.w, eta=G.eta, Ku=G.Ku, Kw=G.Kw, Keta=G.Keta)
    bar = {k: torch.zeros_like(v) for k, v in state.items()}
    with pytest.raises(pmgw.PmgwError):
        pmgw.rk4_stage_adjoint(G.plan, 1, t["dt"], G.h, state, bar, torch.zeros_like(G.h))

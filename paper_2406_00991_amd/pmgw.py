"""Python binding of the HIP library libpmgw.so (argument marshalling only).

Every computation runs in the library's kernels; PyTorch provides device memory and the stream.
The functions keep the C names: ``laplacian_apply``, ``pmg_vcycle``, ``poisson_solve``,
``rk4_stage``, ``pmgw_adjoint_solve``; ``Plan`` wraps plan creation, workspace binding and
geometry. There is no CPU fallback: a missing library raises ``PmgwError``.
"""
import ctypes
import os
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmgw.so")

OK, NOCONV, EINVAL, EGEOM, ENAN, EWORKSPACE, EDEVICE = 0, 1, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOCONV", -1: "EINVAL", -2: "EGEOM", -3: "ENAN", -4: "EWORKSPACE",
                -5: "EDEVICE"}


class PmgwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("coarse_pairs", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("omega_c", ctypes.c_double), ("omega_m", ctypes.c_double),
                ("rho", ctypes.c_double), ("g", ctypes.c_double), ("nu_visc", ctypes.c_double),
                ("filt_alpha", ctypes.c_double), ("filt_s", ctypes.c_double),
                ("filt_fx", ctypes.c_double), ("filt_fz", ctypes.c_double),
                ("threads", ctypes.c_int32), ("adapt_omega_m", ctypes.c_int32),
                ("cycle", ctypes.c_int32), ("coarse_exact", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("class_threads", ctypes.c_int32 * 5),
                ("class_resident", ctypes.c_int32 * 5), ("bed_line", ctypes.c_int32),
                ("linear", ctypes.c_int32), ("no_slip", ctypes.c_int32),
                ("guess_steps", ctypes.c_int32), ("guess_correct", ctypes.c_int32)]

# finest-level row counts of the per-class options (class_threads, class_resident)
CLASS_ROWS = (3, 5, 9, 17, 33)


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def lib():
    """Load libpmgw.so from the package directory (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PmgwError(EINVAL, f"{LIB_PATH} not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.pmgw_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.pmgw_default_opts.restype = None
        L.pmgw_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), _dp, ctypes.c_int32,
                                       ctypes.POINTER(Opts), _vp]
        L.pmgw_workspace_bytes.argtypes = [_vp]
        L.pmgw_workspace_bytes.restype = ctypes.c_size_t
        L.pmgw_bind_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.pmgw_field_offsets.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]
        L.pmgw_set_geometry.argtypes = [_vp, _vp, _vp, _vp]
        L.laplacian_apply.argtypes = [_vp, _vp, _vp]
        L.pmg_vcycle.argtypes = [_vp, _vp, _vp]
        L.pmgw_fmg.argtypes = [_vp, _vp, _vp]
        L.poisson_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(Info), _vp]
        L.rk4_stage.argtypes = [_vp, ctypes.c_int32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, _vp]
        L.pmgw_adjoint_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                         ctypes.POINTER(Info), _vp]
        L.pmgw_adjoint_apply.argtypes = [_vp, _vp, _vp]
        L.rk4_stage_adjoint.argtypes = ([_vp, ctypes.c_int32, ctypes.c_double] + [_vp] * 14 +
                                        [ctypes.c_double, ctypes.c_int32, _vp])
        L.pmgw_adjoint_vcycle.argtypes = [_vp, _vp, _vp]
        L.pmgw_history_reset.argtypes = [_vp]
        L.pmgw_stream_target.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, _vp, _vp, _vp, _vp]
        L.pmgw_relax.argtypes = [_vp] + [_vp] * 7
        L.pmgw_plan_destroy.argtypes = [_vp]
        L.pmgw_plan_destroy.restype = None
        L.pmgw_last_error.restype = ctypes.c_char_p
        L.poisson_solve_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double,
                                            ctypes.c_int32, ctypes.POINTER(Info), _vp]
        L.pmgw3_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32] + \
            [ctypes.POINTER(ctypes.c_int32)] * 3 + [_dp, _dp, ctypes.c_int32,
                                                   ctypes.POINTER(Opts), _vp]
        L.pmgw3_workspace_bytes.argtypes = [_vp]
        L.pmgw3_workspace_bytes.restype = ctypes.c_size_t
        L.pmgw3_bind_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.pmgw3_field_offsets.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]
        L.pmgw3_set_geometry.argtypes = [_vp, _vp, _vp, _vp]
        L.pmgw3_laplacian_apply.argtypes = [_vp, _vp, _vp]
        L.pmgw3_vcycle.argtypes = [_vp, _vp, _vp]
        L.pmgw3_poisson_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                          ctypes.POINTER(Info), _vp]
        L.pmgw3_plan_destroy.argtypes = [_vp]
        L.pmgw3_plan_destroy.restype = None
        L.pmgw_profile.argtypes = [_vp, ctypes.c_int32]
        L.pmgw_profile_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), _dp, _dp]
        _lib = L
    return _lib


_DEBUG_SYNC = os.environ.get("PMGW_DEBUG_SYNC") == "1"


def _trace(name):
    """With PMGW_DEBUG_SYNC=1, wait for the GPU after each library call and print its name."""
    if _DEBUG_SYNC:
        import torch
        torch.cuda.synchronize()
        print(f"[pmgw] {name} done", flush=True)


def _check(rc, soft_ok=False):
    if rc < 0 or (rc > 0 and not soft_ok):
        raise PmgwError(rc, lib().pmgw_last_error().decode())
    return rc


def default_opts(**kw):
    o = Opts()
    lib().pmgw_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k in ("class_threads", "class_resident"):
            # a list of 5 values, or a dict {rows: value} for some classes
            arr = getattr(o, k)
            items = v.items() if isinstance(v, dict) else zip(CLASS_ROWS, v)
            for rows, val in items:
                arr[CLASS_ROWS.index(int(rows))] = int(val)
        else:
            setattr(o, k, v)
    return o


def _ptr(t, dtype=None, numel=None, device=None):
    """Device address of a tensor after checking what the C ABI cannot: dtype, element count
    (the library takes no lengths, so a short field would be read or written past its end),
    contiguity and device. Raises PmgwError(EINVAL) before any library call."""
    return _ptrs([(t, dtype, numel)], device)[0]


def _ptrs(items, device=None):
    """_ptr for several tensors: every shape check of every tensor runs before the device checks,
    so a wrong length is reported as such whatever the order of the arguments."""
    for t, dtype, numel in items:
        if t is None:
            continue
        if dtype is not None and t.dtype != dtype:
            raise PmgwError(EINVAL, f"tensor must be {dtype}, got {t.dtype}")
        if numel is not None and t.numel() != numel:
            raise PmgwError(EINVAL, f"tensor must have {numel} elements, got {t.numel()}")
        if not t.is_contiguous():
            raise PmgwError(EINVAL, "tensor must be contiguous")
    out = []
    for t, _, _ in items:
        if t is None:
            out.append(None)
            continue
        if not t.is_cuda:
            raise PmgwError(EINVAL, "tensor must be on the GPU")
        if device is not None and t.device.index != device:
            raise PmgwError(EINVAL, f"tensor must be on cuda:{device}, got {t.device}")
        out.append(ctypes.c_void_p(t.data_ptr()))
    return out


def _fields(plan, *spec):
    """Pointers for (tensor, kind) pairs of one call: kind 2 = packed 2D field (off2d[-1]
    float64), 1 = packed 1D field (off1d[-1] float64), 'i1' / 'i2' = an info buffer of one or two
    records per tank (or None)."""
    import torch
    size = {2: plan.n2d, 1: plan.n1d, "i1": 2 * plan.ntanks, "i2": 4 * plan.ntanks}
    return _ptrs([(t, torch.float64, size[k]) for t, k in spec], plan.device_index)


class Plan:
    """A solver plan for one or more tanks (sizes nx[t], nz[t], lengths L[t]).

    precision: "fp64" or "mixed". The workspace is a torch uint8 tensor owned by the plan.
    """

    def __init__(self, nx, nz, L, precision="fp64", opts=None, device=None, stream=None,
                 allocate=True):
        import torch
        nx = [int(v) for v in (nx if hasattr(nx, "__len__") else [nx])]
        nz = [int(v) for v in (nz if hasattr(nz, "__len__") else [nz])]
        L = [float(v) for v in (L if hasattr(L, "__len__") else [L])]
        if not (len(nx) == len(nz) == len(L)):
            raise PmgwError(EINVAL, "nx, nz and L must have the same length")
        self.ntanks = len(nx)
        self.nx, self.nz, self.L = nx, nz, L
        self.precision = precision
        prec = {"fp64": FP64, "mixed": MIXED}.get(precision)
        if prec is None:
            raise PmgwError(EINVAL, "precision must be 'fp64' or 'mixed'")
        self.opts = opts if opts is not None else default_opts()
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self.stream = stream
        sh = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        h = ctypes.c_void_p()
        a_nx = (ctypes.c_int32 * self.ntanks)(*nx)
        a_nz = (ctypes.c_int32 * self.ntanks)(*nz)
        a_L = (ctypes.c_double * self.ntanks)(*L)
        _check(lib().pmgw_plan_create(ctypes.byref(h), self.ntanks, a_nx, a_nz, a_L, prec,
                                      ctypes.byref(self.opts), sh))
        self._h = h
        o2 = (ctypes.c_int64 * (self.ntanks + 1))()
        o1 = (ctypes.c_int64 * (self.ntanks + 1))()
        _check(lib().pmgw_field_offsets(h, o2, o1))
        self.off2d = list(o2)
        self.off1d = list(o1)
        self.n2d = self.off2d[-1]
        self.n1d = self.off1d[-1]
        self.workspace_bytes = int(lib().pmgw_workspace_bytes(h))
        self.device = device if device is not None else "cuda"
        self.device_index = None
        if torch.cuda.is_available():
            dv = torch.device(self.device)
            self.device_index = dv.index if dv.index is not None else torch.cuda.current_device()
        self.ws = None
        if allocate:
            self.bind(torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device))
        self.info_dev = None

    def bind(self, ws):
        self.ws = ws
        _check(lib().pmgw_bind_workspace(self._h, _ptr(ws, device=self.device_index), ws.numel()))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                lib().pmgw_plan_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass

    # -- helpers
    def field(self, fill=0.0):
        import torch
        return torch.full((self.n2d,), fill, dtype=torch.float64, device=self.device)

    def split2d(self, flat):
        return [flat[self.off2d[t]:self.off2d[t + 1]].view(self.nz[t], self.nx[t])
                for t in range(self.ntanks)]

    def split1d(self, flat):
        return [flat[self.off1d[t]:self.off1d[t + 1]] for t in range(self.ntanks)]

    def set_geometry(self, h, eta_old, eta_new=None):
        import torch
        eta_new = eta_old if eta_new is None else eta_new
        self._geo = (h, eta_old, eta_new)
        _check(lib().pmgw_set_geometry(self._h, *_fields(self, (h, 1), (eta_old, 1),
                                                         (eta_new, 1))))
        _trace("set_geometry")

    def apply(self, p, out=None):
        out = self.field() if out is None else out
        laplacian_apply(self, p, out)
        return out

    def vcycle(self, r, out=None):
        out = self.field() if out is None else out
        pmg_vcycle(self, r, out)
        return out

    def solve(self, b, p=None, rtol=1e-10, maxit=100, sync=True):
        p = self.field() if p is None else p
        info = poisson_solve(self, b, p, rtol, maxit, sync=sync)
        return p, info


def laplacian_apply(plan, p, Ap):
    import torch
    _check(lib().laplacian_apply(plan._h, *_fields(plan, (p, 2), (Ap, 2))))
    _trace("laplacian_apply")


def pmg_vcycle(plan, r, z):
    import torch
    _check(lib().pmg_vcycle(plan._h, *_fields(plan, (r, 2), (z, 2))))
    _trace("pmg_vcycle")


def fmg(plan, r, z):
    import torch
    _check(lib().pmgw_fmg(plan._h, *_fields(plan, (r, 2), (z, 2))))
    _trace("pmgw_fmg")


def poisson_solve(plan, b, p, rtol=1e-10, maxit=100, sync=True, info_dev=None):
    """Returns a list of (iters, status, relres) per tank when sync, else None."""
    return _solve("poisson_solve", plan, b, p, rtol, maxit, sync, info_dev)


def adjoint_solve(plan, g, lam, rtol=1e-10, maxit=100, sync=True, info_dev=None):
    """lam = A^-T g (lam holds the initial guess). Returns per-tank info like poisson_solve."""
    return _solve("pmgw_adjoint_solve", plan, g, lam, rtol, maxit, sync, info_dev)


def adjoint_apply(plan, lam, out):
    import torch
    _check(lib().pmgw_adjoint_apply(plan._h, *_fields(plan, (lam, 2), (out, 2))))
    _trace("pmgw_adjoint_apply")


def adjoint_vcycle(plan, r, z):
    import torch
    _check(lib().pmgw_adjoint_vcycle(plan._h, *_fields(plan, (r, 2), (z, 2))))
    _trace("pmgw_adjoint_vcycle")


def _solve(name, plan, b, p, rtol, maxit, sync, info_dev):
    import torch
    bp, pp, dptr = _fields(plan, (b, 2), (p, 2), (info_dev, "i1"))
    infos = (Info * plan.ntanks)() if sync else None
    rc = getattr(lib(), name)(plan._h, bp, pp, float(rtol), int(maxit), infos, dptr)
    _trace(name)
    if rc < 0:
        msg = lib().pmgw_last_error().decode()
        out = [(i.iters, i.status, i.relres) for i in infos] if infos is not None else None
        err = PmgwError(rc, msg)
        err.info = out
        raise err
    if not sync:
        return None
    out = [(i.iters, i.status, i.relres) for i in infos]
    if rc == NOCONV:
        warnings.warn(name + ": a tank did not converge: " +
                      lib().pmgw_last_error().decode())
    return out


def poisson_solve_noalloc(plan, h, eta_old, eta_new, b, p, rtol=1e-10, maxit=100, sync=True,
                          info_dev=None):
    """Geometry and solve in the library's static scratch array (no workspace, no device
    allocation). Returns per-tank info like poisson_solve."""
    *geo, bp, pp, dptr = _fields(plan, (h, 1), (eta_old, 1), (eta_new, 1), (b, 2), (p, 2),
                                 (info_dev, "i1"))
    infos = (Info * plan.ntanks)() if sync else None
    rc = lib().poisson_solve_noalloc(plan._h, *geo, bp, pp, float(rtol), int(maxit), infos, dptr)
    _trace("poisson_solve_noalloc")
    if rc < 0:
        err = PmgwError(rc, lib().pmgw_last_error().decode())
        err.info = [(i.iters, i.status, i.relres) for i in infos] if infos is not None else None
        raise err
    if not sync:
        return None
    out = [(i.iters, i.status, i.relres) for i in infos]
    if rc == NOCONV:
        warnings.warn("poisson_solve_noalloc: a tank did not converge: " +
                      lib().pmgw_last_error().decode())
    return out


def rk4_stage(plan, k, dt, h, u, w, eta, Ku, Kw, Keta, p, rtol=1e-10, maxit=100, info_dev=None):
    """One stage k (1..5) of the low-storage RK scheme with the pressure projection, in place."""
    *args, dptr = _fields(plan, (h, 1), (u, 2), (w, 2), (eta, 1), (Ku, 2), (Kw, 2), (Keta, 1),
                          (p, 2), (info_dev, "i1"))
    _check(lib().rk4_stage(plan._h, int(k), float(dt), *args, float(rtol), int(maxit), dptr))
    _trace("rk4_stage")


def rk4_stage_adjoint(plan, k, dt, h, state, bar, hbar, rtol=1e-12, maxit=200, info_dev=None):
    """Reverse of stage k. state: dict u, w, eta, Ku, Kw, Keta of the stage's INPUT state (left
    unchanged). bar: dict of the same keys holding the adjoints of the stage's outputs, replaced
    in place by the adjoints of its inputs. hbar is accumulated. info_dev (optional, 2 x ntanks
    records): the forward recompute solve's record per tank, then the adjoint solve's."""
    keys = ("u", "w", "eta", "Ku", "Kw", "Keta")
    kind = lambda q: 1 if q in ("eta", "Keta") else 2
    *args, dptr = _fields(plan, (h, 1), *[(state[q], kind(q)) for q in keys],
                          *[(bar[q], kind(q)) for q in keys], (hbar, 1), (info_dev, "i2"))
    _check(lib().rk4_stage_adjoint(plan._h, int(k), float(dt), *args, float(rtol), int(maxit),
                                   dptr))
    _trace("rk4_stage_adjoint")


def rk4_step(plan, dt, h, u, w, eta, Ku, Kw, Keta, p, rtol=1e-10, maxit=100, info_dev=None):
    """One full time step: stages 1..5 (stage 1 multiplies the registers K by zero)."""
    for k in range(1, 6):
        rk4_stage(plan, k, dt, h, u, w, eta, Ku, Kw, Keta, p, rtol, maxit, info_dev)


def stream_target(plan, coef, nmodes, t, a, window, u_t, w_t, eta_t):
    """Relaxation targets at time t: the stream-function wave of coefficients coef (device
    float64, ntanks x (2 nmodes + 6)) times a * window, into u_t, w_t (2D) and eta_t (1D)."""
    import torch
    (cp,) = _ptrs([(coef, torch.float64, plan.ntanks * (2 * int(nmodes) + 6))],
                  plan.device_index)
    args = _fields(plan, (window, 1), (u_t, 2), (w_t, 2), (eta_t, 1))
    _check(lib().pmgw_stream_target(plan._h, cp, int(nmodes), float(t), float(a), *args))
    _trace("stream_target")


def relax(plan, r, u_t, w_t, eta_t, u, w, eta):
    """q <- q + r (q_t - q) for u, w and eta (r per column)."""
    _check(lib().pmgw_relax(plan._h, *_fields(plan, (r, 1), (u_t, 2), (w_t, 2), (eta_t, 1),
                                              (u, 2), (w, 2), (eta, 1))))
    _trace("relax")


def history_reset(plan):
    """Forget the stage pressures recorded for opts.guess_steps (and the last extrapolation of
    opts.guess_correct)."""
    _check(lib().pmgw_history_reset(plan._h))


def profile_start(plan, capacity):
    """Record event-pair timings of the next `capacity` solve-kernel launches of the plan."""
    _check(lib().pmgw_profile(plan._h, int(capacity)))


def profile_read(plan):
    """(launches, total_ms, max_ms) of the recorded solve launches (synchronises)."""
    n = ctypes.c_int32()
    tot = ctypes.c_double()
    mx = ctypes.c_double()
    _check(lib().pmgw_profile_read(plan._h, ctypes.byref(n), ctypes.byref(tot), ctypes.byref(mx)))
    return n.value, tot.value, mx.value


def info_buffer(ntanks, device=None):
    """Device array of ntanks pmgw_info records (16 bytes each) for the info_dev arguments
    (2 float64 slots per record; a record slice is buf[2 r: 2 (r + n)])."""
    import torch
    return torch.zeros(ntanks * 2, dtype=torch.float64, device=device or "cuda")


def read_info(buf):
    """Synchronously read an info_buffer: list of dicts (iters, status, relres) per tank."""
    host = buf.cpu().numpy()
    raw = host.view(np.int32).reshape(-1, 4)
    rel = host.reshape(-1, 2)[:, 1]
    return [dict(iters=int(r[0]), status=int(r[1]), relres=float(x)) for r, x in zip(raw, rel)]


class Plan3:
    """A plan for 3D tanks (x, y periodic Fourier, sigma Chebyshev; float64): sizes nx[t], ny[t],
    nz[t], periods Lx[t], Ly[t]. Fields are [Nz][Ny][Nx] per tank, packed at off3d; h and eta are
    [Ny][Nx] at off2d. The workspace is a torch uint8 tensor owned by the plan."""

    def __init__(self, nx, ny, nz, Lx, Ly, opts=None, device=None, stream=None):
        import torch
        seq = lambda v, f: [f(a) for a in (v if hasattr(v, "__len__") else [v])]
        nx, ny, nz = seq(nx, int), seq(ny, int), seq(nz, int)
        Lx, Ly = seq(Lx, float), seq(Ly, float)
        if not (len(nx) == len(ny) == len(nz) == len(Lx) == len(Ly)):
            raise PmgwError(EINVAL, "nx, ny, nz, Lx and Ly must have the same length")
        self.ntanks = len(nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.opts = opts if opts is not None else default_opts()
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self.stream = stream
        sh = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        h = ctypes.c_void_p()
        arr = lambda t, v: (t * self.ntanks)(*v)
        _check(lib().pmgw3_plan_create(ctypes.byref(h), self.ntanks, arr(ctypes.c_int32, nx),
                                       arr(ctypes.c_int32, ny), arr(ctypes.c_int32, nz),
                                       arr(ctypes.c_double, Lx), arr(ctypes.c_double, Ly), FP64,
                                       ctypes.byref(self.opts), sh))
        self._h = h
        o3 = (ctypes.c_int64 * (self.ntanks + 1))()
        o2 = (ctypes.c_int64 * (self.ntanks + 1))()
        _check(lib().pmgw3_field_offsets(h, o3, o2))
        self.off3d, self.off2d = list(o3), list(o2)
        self.n3d, self.n2d = self.off3d[-1], self.off2d[-1]
        self.device = device if device is not None else "cuda"
        self.device_index = None
        if torch.cuda.is_available():
            dv = torch.device(self.device)
            self.device_index = dv.index if dv.index is not None else torch.cuda.current_device()
        self.ws = torch.empty(int(lib().pmgw3_workspace_bytes(h)), dtype=torch.uint8,
                              device=self.device)
        _check(lib().pmgw3_bind_workspace(h, _ptr(self.ws, device=self.device_index),
                                          self.ws.numel()))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                lib().pmgw3_plan_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass

    def field(self, fill=0.0):
        import torch
        return torch.full((self.n3d,), fill, dtype=torch.float64, device=self.device)

    def split3d(self, flat):
        return [flat[self.off3d[t]:self.off3d[t + 1]].view(self.nz[t], self.ny[t], self.nx[t])
                for t in range(self.ntanks)]

    def _f(self, *items):
        return _ptrs([(t, _torch_f64(), n) for t, n in items], self.device_index)

    def set_geometry(self, h, eta_old, eta_new=None):
        eta_new = eta_old if eta_new is None else eta_new
        self._geo = (h, eta_old, eta_new)
        _check(lib().pmgw3_set_geometry(self._h, *self._f((h, self.n2d), (eta_old, self.n2d),
                                                          (eta_new, self.n2d))))

    def apply(self, p, out=None):
        out = self.field() if out is None else out
        _check(lib().pmgw3_laplacian_apply(self._h, *self._f((p, self.n3d), (out, self.n3d))))
        return out

    def vcycle(self, r, out=None):
        out = self.field() if out is None else out
        _check(lib().pmgw3_vcycle(self._h, *self._f((r, self.n3d), (out, self.n3d))))
        return out

    def solve(self, b, p=None, rtol=1e-10, maxit=100):
        """FGMRES from the initial guess p (zero when None); returns (p, [(iters, status, relres)])."""
        p = self.field() if p is None else p
        infos = (Info * self.ntanks)()
        rc = lib().pmgw3_poisson_solve(self._h, *self._f((b, self.n3d), (p, self.n3d)),
                                       ctypes.c_double(rtol), int(maxit), infos, None)
        _check(rc, soft_ok=True)
        return p, [(i.iters, i.status, i.relres) for i in infos]


def _torch_f64():
    import torch
    return torch.float64

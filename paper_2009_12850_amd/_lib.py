"""Thin ctypes binding of libmoncadv.so.

Argument marshalling only: every step of the advection path runs in the
library's HIP kernels.  torch supplies device memory (``tensor.data_ptr()``)
and the stream (``torch.cuda.current_stream().cuda_stream``).  If the library
has not been built, loading raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoncadv.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "monc_adv.h")

MONC_OK, MONC_EINVAL, MONC_EHIP, MONC_ECFL, MONC_ENONFINITE, MONC_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5
MONC_F64, MONC_F32, MONC_BF16 = 0, 1, 2
MONC_MAX_SCALARS = 8
MONC_MAX_NZ = 128
MONC_MAX_WORK = 64
B_CU, B_CV, B_CW, B_PU, B_QU, B_PV, B_QV, B_PW, B_QW, B_COURANT, B_NONFINITE = range(11)
B_SCALAR0 = 11
MONC_NBUDGET = B_SCALAR0 + 3 * MONC_MAX_SCALARS


class MoncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None

vp = C.c_void_p
ip = C.c_int
dp = C.c_double
PP = C.POINTER(C.c_void_p)
DPTR = C.POINTER(C.c_double)

_SIGS = {
    "monc_halo_fill": ([ip, PP, ip, ip, ip, vp], ip),
    "monc_halo_fill_f32": ([ip, PP, ip, ip, ip, vp], ip),
    "monc_halo_fill_bf16": ([ip, PP, ip, ip, ip, vp], ip),
    "monc_advect_pw": ([vp, vp, vp, vp, vp, vp, ip, ip, ip, dp, dp, vp, vp, vp, vp], ip),
    "monc_advect_pw_scaled": ([ip, vp, vp, vp, vp, vp, vp, ip, ip, ip, dp, dp, vp, vp, vp, ip, vp],
                              ip),
    "monc_advect_tvd": ([vp, vp, vp, ip, PP, PP, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp], ip),
    "monc_advect": ([ip, PP, PP, ip, DPTR, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp], ip),
    "monc_advect_pw_f32": ([vp, vp, vp, vp, vp, vp, ip, ip, ip, dp, dp, vp, vp, vp, vp], ip),
    "monc_advect_pw_bf16": ([vp, vp, vp, vp, vp, vp, ip, ip, ip, dp, dp, vp, vp, vp, vp], ip),
    "monc_advect_tvd_f32": ([vp, vp, vp, ip, PP, PP, DPTR, ip, ip, ip, dp, dp, vp, vp, vp, dp,
                             vp], ip),
    "monc_advect_tvd_bf16": ([vp, vp, vp, ip, PP, PP, DPTR, ip, ip, ip, dp, dp, vp, vp, vp, dp,
                              vp], ip),
    "monc_step_workspace_bytes": ([ip, ip, ip, ip], C.c_size_t),
    "monc_step": ([PP, PP, ip, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp, vp, vp], ip),
    "monc_step_static": ([PP, PP, ip, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp, vp], ip),
    "monc_step_mixed": ([PP, PP, ip, DPTR, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp, vp, vp],
                        ip),
    "monc_cast_working": ([ip, ip, PP, PP, DPTR, ip, ip, ip, vp], ip),
    "monc_dyn_tend": ([vp, vp, vp, vp, vp, vp, ip, ip, ip, vp, vp], ip),
    "monc_combine_step": ([ip, PP, PP, PP, PP, ip, ip, ip, dp, vp], ip),
    "monc_hybrid_step": ([PP, PP, PP, PP, ip, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp, vp, vp],
                         ip),
    "monc_step_dyn": ([PP, PP, ip, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp, vp], ip),
    "monc_step_pw_scalars": ([PP, PP, ip, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp], ip),
    "monc_advect_tvd_momentum": ([vp, vp, vp, vp, vp, vp, ip, ip, ip, dp, dp, vp, vp, vp, dp,
                                  vp, vp], ip),
    "monc_step_tvd_momentum": ([PP, PP, ip, ip, ip, ip, dp, dp, vp, vp, vp, dp, vp, vp], ip),
    "monc_ceiling_sink_bytes": ([ip], C.c_size_t),
    "monc_stream_ceiling": ([ip, vp, vp, C.c_size_t, ip, vp], ip),
    "monc_budgets_check": ([DPTR], ip),
    "monc_restrict4": ([ip, PP, PP, ip, ip, ip, vp, vp, vp, vp, vp, vp, vp], ip),
    "monc_mlp_features": ([PP, ip, ip, ip, DPTR, ip, vp, ip, vp, vp], ip),
    "monc_mlp_pack": ([vp, vp, vp], ip),
    "monc_mlp_infer": ([PP, ip, ip, ip, DPTR, ip, vp, vp, vp, vp], ip),
    "monc_mlp_forward": ([vp, ip, vp, vp, vp, vp, vp, vp, vp, vp], ip),
    "monc_mlp_backward_workspace_bytes": ([ip], C.c_size_t),
    "monc_mlp_backward": ([vp, vp, vp, vp, vp, vp, ip, vp, vp, vp, vp], ip),
    "monc_mlp_loss_workspace_bytes": ([ip], C.c_size_t),
    "monc_mlp_loss": ([vp, ip, vp, PP, PP, PP, ip, ip, ip, dp, DPTR, vp, vp, dp, vp, vp, vp,
                       vp], ip),
    "monc_mlp_adam": ([vp, vp, vp, vp, ip, dp, dp, dp, dp, vp, vp], ip),
    "monc_mlp_train_workspace_bytes": ([ip], C.c_size_t),
    "monc_mlp_train_step": ([PP, PP, PP, ip, ip, ip, DPTR, vp, ip, dp, DPTR, vp, vp, dp, vp, vp,
                             vp, ip, dp, dp, dp, dp, vp, vp, vp, vp, vp], ip),
    "monc_correct_step_workspace_bytes": ([ip, ip, ip], C.c_size_t),
    "monc_correct_step": ([PP, PP, vp, vp, PP, ip, ip, ip, dp, dp, DPTR, vp, vp, vp, dp, dp,
                           vp, vp, vp], ip),
    "monc_ensemble_create": ([vp, ip, ip, C.c_char_p, ip, C.POINTER(vp)], ip),
    "monc_ensemble_run": ([vp, ip, vp], ip),
    "monc_ensemble_set_budgets": ([vp, vp, ip], ip),
    "monc_ensemble_step": ([vp, vp], ip),
    "monc_ensemble_parity": ([vp], ip),
    "monc_ensemble_info": ([vp, C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)], ip),
    "monc_ensemble_destroy": ([vp], ip),
    "monc_strerror": ([ip], C.c_char_p),
    "monc_last_error": ([], C.c_char_p),
}


def lib():
    """Load libmoncadv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch must be loaded first: it carries its own copy of the HIP
        # runtime (same soname), and the library must bind to that copy so that
        # torch's device pointers and streams are valid in both.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2009_12850_amd.build` (there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def header_symbols():
    """Names of every function declared in include/monc_adv.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(monc_[a-z0-9_]+)\s*\(", text)))


def _check(rc: int, what: str):
    if rc != MONC_OK:
        msg = lib().monc_last_error().decode()
        raise MoncError(rc, f"{what}: {msg}")


# ---------------------------------------------------------------------------
# torch glue
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t, dtype=None, shape=None, what="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on a HIP device (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype} (got {t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _ptrs(ts, dtype, shape, what):
    arr = (C.c_void_p * max(len(ts), 1))()
    for n, t in enumerate(ts):
        arr[n] = _ptr(t, dtype, shape, f"{what}[{n}]").value
    return arr


def _grid(t):
    nx4, ny4, nz = t.shape
    return nx4 - 4, ny4 - 4, nz


def _prof(prof):
    torch = _torch()
    rdz, rho, rhon = prof
    nz = rdz.shape[0]
    return [_ptr(p, torch.float64, (nz,), n) for p, n in zip((rdz, rho, rhon),
                                                             ("rdz", "rho", "rhon"))]


_DT = {}


def _dtypes():
    torch = _torch()
    if not _DT:
        _DT.update({MONC_F64: torch.float64, MONC_F32: torch.float32,
                    MONC_BF16: torch.int16})
    return _DT


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def monc_halo_fill(fields, stream=None):
    torch = _torch()
    dt = fields[0].dtype
    nx, ny, nz = _grid(fields[0])
    shape = tuple(fields[0].shape)
    fn = {torch.float64: "monc_halo_fill", torch.float32: "monc_halo_fill_f32",
          torch.int16: "monc_halo_fill_bf16", torch.bfloat16: "monc_halo_fill_bf16"}[dt]
    arr = _ptrs(fields, dt, shape, "fields")
    _check(getattr(lib(), fn)(len(fields), arr, nx, ny, nz, _stream(stream)), fn)


def monc_advect_pw(u, v, w, su, sv, sw, dx, dy, prof, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(u)
    sh = tuple(u.shape)
    ps = [_ptr(t, torch.float64, sh, n) for t, n in
          zip((u, v, w, su, sv, sw), ("u", "v", "w", "su", "sv", "sw"))]
    _check(lib().monc_advect_pw(*ps, nx, ny, nz, float(dx), float(dy), *_prof(prof),
                                _stream(stream)), "monc_advect_pw")


def monc_advect_pw_scaled(dtype, u, v, w, su, sv, sw, dx, dy, prof, work, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(u)
    tdt = torch.float64 if dtype == MONC_F64 else torch.float32
    sh = tuple(u.shape)
    p = [_ptr(x, tdt, sh, n) for x, n in ((u, "u"), (v, "v"), (w, "w"), (su, "su"), (sv, "sv"),
                                            (sw, "sw"))]
    _check(lib().monc_advect_pw_scaled(int(dtype), *p, nx, ny, nz, float(dx), float(dy),
                                       *_prof(prof), int(work), _stream(stream)),
           "monc_advect_pw_scaled")


def monc_advect_tvd(u, v, w, q, sq, dx, dy, prof, dt, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(u)
    sh = tuple(u.shape)
    ps = [_ptr(t, torch.float64, sh, n) for t, n in zip((u, v, w), ("u", "v", "w"))]
    qa = _ptrs(q, torch.float64, sh, "q")
    sa = _ptrs(sq, torch.float64, sh, "sq")
    _check(lib().monc_advect_tvd(*ps, len(q), qa, sa, nx, ny, nz, float(dx), float(dy),
                                 *_prof(prof), float(dt), _stream(stream)),
           "monc_advect_tvd")


def monc_advect(dtype, inputs, outputs, dx, dy, prof, dt, phi0=None, stream=None):
    """Fused PW + TVD source terms.  inputs = [u, v, w, scalars...] in the
    storage dtype (float64, float32, or int16 holding bfloat16 bits); outputs
    float64 for MONC_F64, float32 otherwise."""
    torch = _torch()
    nx, ny, nz = _grid(inputs[0])
    sh = tuple(inputs[0].shape)
    nscal = len(inputs) - 3
    ia = _ptrs(inputs, _dtypes()[dtype], sh, "in")
    odt = torch.float64 if dtype == MONC_F64 else torch.float32
    oa = _ptrs(outputs, odt, sh, "out")
    p0 = None
    if phi0 is not None:
        p0 = (C.c_double * max(nscal, 1))(*[float(x) for x in phi0])
    _check(lib().monc_advect(dtype, ia, oa, nscal, p0, nx, ny, nz, float(dx), float(dy),
                             *_prof(prof), float(dt), _stream(stream)), "monc_advect")


def monc_advect_pw_narrow(dtype, u, v, w, su, sv, sw, dx, dy, prof, stream=None):
    """monc_advect_pw_f32 (dtype MONC_F32: float32 velocities) or
    monc_advect_pw_bf16 (MONC_BF16: int16 tensors holding bfloat16 bits);
    float32 source terms."""
    torch = _torch()
    fn = {MONC_F32: "monc_advect_pw_f32", MONC_BF16: "monc_advect_pw_bf16"}[dtype]
    nx, ny, nz = _grid(u)
    sh = tuple(u.shape)
    vel = [_ptr(x, _dtypes()[dtype], sh, n) for x, n in ((u, "u"), (v, "v"), (w, "w"))]
    out = [_ptr(x, torch.float32, sh, n) for x, n in ((su, "su"), (sv, "sv"), (sw, "sw"))]
    _check(getattr(lib(), fn)(*vel, *out, nx, ny, nz, float(dx), float(dy), *_prof(prof),
                              _stream(stream)), fn)


def monc_advect_tvd_narrow(dtype, u, v, w, q, sq, dx, dy, prof, dt, phi0=None, stream=None):
    """monc_advect_tvd_f32 / _bf16: TVD source terms of the narrow scalar
    copies q (list), float32 results into sq (list)."""
    torch = _torch()
    fn = {MONC_F32: "monc_advect_tvd_f32", MONC_BF16: "monc_advect_tvd_bf16"}[dtype]
    nx, ny, nz = _grid(u)
    sh = tuple(u.shape)
    vel = [_ptr(x, _dtypes()[dtype], sh, n) for x, n in ((u, "u"), (v, "v"), (w, "w"))]
    qa = _ptrs(q, _dtypes()[dtype], sh, "q")
    sa = _ptrs(sq, torch.float32, sh, "sq")
    p0 = None
    if phi0 is not None:
        p0 = (C.c_double * max(len(q), 1))(*[float(x) for x in phi0])
    _check(getattr(lib(), fn)(*vel, len(q), qa, sa, p0, nx, ny, nz, float(dx), float(dy),
                              *_prof(prof), float(dt), _stream(stream)), fn)


def monc_step_workspace_bytes(nx, ny, nz, nscal):
    return int(lib().monc_step_workspace_bytes(nx, ny, nz, nscal))


def monc_step_static(state_in, state_out, dx, dy, prof, dt, budgets, stream=None):
    """monc_step with budgets and no workspace (the library's static scratch)."""
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    nscal = len(state_in) - 3
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    b = _ptr(budgets, torch.float64, (MONC_NBUDGET,), "budgets")
    rc = lib().monc_step_static(ia, oa, nscal, nx, ny, nz, float(dx), float(dy), *_prof(prof),
                                float(dt), b, _stream(stream))
    _check(rc, "monc_step_static")


def monc_step(state_in, state_out, dx, dy, prof, dt, budgets=None, workspace=None,
              stream=None, mixed=False, phi0=None):
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    nscal = len(state_in) - 3
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    b = None if budgets is None else _ptr(budgets, torch.float64, (MONC_NBUDGET,), "budgets")
    ws = None if workspace is None else _ptr(workspace, None, None, "workspace")
    if workspace is not None:
        need = monc_step_workspace_bytes(nx, ny, nz, nscal)
        if workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
    if mixed:
        p0 = (C.c_double * max(nscal, 1))(*([float(x) for x in phi0] if phi0 is not None
                                            else [0.0] * max(nscal, 1)))
        rc = lib().monc_step_mixed(ia, oa, nscal, p0, nx, ny, nz, float(dx), float(dy),
                                   *_prof(prof), float(dt), b, ws, _stream(stream))
        _check(rc, "monc_step_mixed")
    else:
        rc = lib().monc_step(ia, oa, nscal, nx, ny, nz, float(dx), float(dy), *_prof(prof),
                             float(dt), b, ws, _stream(stream))
        _check(rc, "monc_step")


class DynParams(C.Structure):
    """monc_dyn_params: Coriolis parameter, geostrophic wind, gravity, theta reference."""
    _fields_ = [("fcor", C.c_double), ("ug", C.c_double), ("vg", C.c_double),
                ("grav", C.c_double), ("th0", C.c_double)]


def _dyn(p):
    if isinstance(p, DynParams):
        return C.byref(p)
    return C.byref(DynParams(*[float(x) for x in p]))


def monc_dyn_tend(u, v, theta, su, sv, sw, params, stream=None):
    """Coriolis and buoyancy source terms; params = (fcor, ug, vg, grav, th0)."""
    torch = _torch()
    nx, ny, nz = _grid(u)
    sh = tuple(u.shape)
    args = [_ptr(t, torch.float64, sh, n) for t, n in
            zip((u, v, theta, su, sv, sw), ("u", "v", "theta", "su", "sv", "sw"))]
    rc = lib().monc_dyn_tend(*args, nx, ny, nz, _dyn(params), _stream(stream))
    _check(rc, "monc_dyn_tend")


def monc_combine_step(state_in, ta, tb, state_out, dt, stream=None):
    """state_out[f] = state_in[f] + dt (ta[f] + tb[f]); tb may be None or hold None."""
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    n = len(state_in)
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    aa = _ptrs(ta, torch.float64, sh, "ta")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    ba = None
    if tb is not None:
        ba = (C.c_void_p * n)()
        for f, t in enumerate(tb):
            ba[f] = None if t is None else _ptr(t, torch.float64, sh, f"tb[{f}]").value
    rc = lib().monc_combine_step(n, ia, aa, ba, oa, nx, ny, nz, float(dt), _stream(stream))
    _check(rc, "monc_combine_step")


def monc_hybrid_step(state_in, state_out, tend, dyn_tend, dx, dy, prof, dt, params,
                     stream=None, side_stream=None):
    """Advection source terms on `stream`, Coriolis and buoyancy on `side_stream`,
    then one combine pass (state_out = state_in + dt (s_adv + s_dyn))."""
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    nscal = len(state_in) - 3
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    ta = _ptrs(tend, torch.float64, sh, "tend")
    da = _ptrs(dyn_tend, torch.float64, sh, "dyn_tend")
    s_main = _stream(stream)
    s_side = s_main if side_stream is None else _stream(side_stream)
    rc = lib().monc_hybrid_step(ia, oa, ta, da, nscal, nx, ny, nz, float(dx), float(dy),
                                *_prof(prof), float(dt), _dyn(params), s_main, s_side)
    _check(rc, "monc_hybrid_step")


def monc_step_dyn(state_in, state_out, dx, dy, prof, dt, params, stream=None):
    """One pass: PW + TVD + Coriolis + buoyancy, then the step."""
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    nscal = len(state_in) - 3
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    rc = lib().monc_step_dyn(ia, oa, nscal, nx, ny, nz, float(dx), float(dy), *_prof(prof),
                             float(dt), _dyn(params), _stream(stream))
    _check(rc, "monc_step_dyn")


def monc_step_pw_scalars(state_in, state_out, dx, dy, prof, dt, stream=None):
    """The FP64 step with the scalars advected by the centred (PW) flux form."""
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    nscal = len(state_in) - 3
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    rc = lib().monc_step_pw_scalars(ia, oa, nscal, nx, ny, nz, float(dx), float(dy),
                                    *_prof(prof), float(dt), _stream(stream))
    _check(rc, "monc_step_pw_scalars")


def monc_advect_tvd_momentum(u, v, w, su, sv, sw, dx, dy, prof, dt, cmax=None,
                             stream=None):
    """TVD momentum source terms; cmax (float64 device tensor of one element,
    optional) receives the largest Courant number of the momentum faces."""
    torch = _torch()
    nx, ny, nz = _grid(u)
    sh = tuple(u.shape)
    ps = [_ptr(t, torch.float64, sh, n) for t, n in zip((u, v, w, su, sv, sw),
                                                       ("u", "v", "w", "su", "sv", "sw"))]
    cm = C.c_void_p(None) if cmax is None else _ptr(cmax, torch.float64, (1,), "cmax")
    _check(lib().monc_advect_tvd_momentum(*ps, nx, ny, nz, float(dx), float(dy), *_prof(prof),
                                          float(dt), cm, _stream(stream)),
           "monc_advect_tvd_momentum")


def monc_step_tvd_momentum(state_in, state_out, dx, dy, prof, dt, cmax=None, stream=None):
    """The FP64 step with TVD for momentum and scalars."""
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    nscal = len(state_in) - 3
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    cm = C.c_void_p(None) if cmax is None else _ptr(cmax, torch.float64, (1,), "cmax")
    rc = lib().monc_step_tvd_momentum(ia, oa, nscal, nx, ny, nz, float(dx), float(dy),
                                      *_prof(prof), float(dt), cm, _stream(stream))
    _check(rc, "monc_step_tvd_momentum")


def monc_step_mixed(state_in, state_out, phi0, dx, dy, prof, dt, budgets=None,
                    workspace=None, stream=None):
    monc_step(state_in, state_out, dx, dy, prof, dt, budgets, workspace, stream,
              mixed=True, phi0=phi0)


def monc_cast_working(dtype, src, work, offset=None, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(src[0])
    sh = tuple(src[0].shape)
    sa = _ptrs(src, torch.float64, sh, "src")
    wa = _ptrs(work, _dtypes()[dtype], sh, "work")
    off = None
    if offset is not None:
        off = (C.c_double * len(src))(*[float(x) for x in offset])
    _check(lib().monc_cast_working(dtype, len(src), sa, wa, off, nx, ny, nz,
                                   _stream(stream)), "monc_cast_working")


MONC_CEIL_READ, MONC_CEIL_WRITE, MONC_CEIL_COPY = 0, 1, 2


def monc_stream_ceiling(mode, src, dst, nbytes, blocks, stream=None):
    """Streaming ceiling kernel: src, dst are device tensors (src may be None
    for MONC_CEIL_WRITE); nbytes bytes are read, written or copied."""
    sp = src.data_ptr() if src is not None else None
    _check(lib().monc_stream_ceiling(mode, sp, dst.data_ptr(), nbytes, blocks,
                                     _stream(stream)), "monc_stream_ceiling")


def monc_ceiling_sink_bytes(blocks):
    return int(lib().monc_ceiling_sink_bytes(blocks))


def monc_budgets_check(host_budgets):
    import numpy as np
    arr = np.ascontiguousarray(host_budgets, dtype=np.float64)
    return int(lib().monc_budgets_check(arr.ctypes.data_as(DPTR)))


def budgets_dict(b, nscal):
    """Name the entries of a host budgets array."""
    names = ["C_u", "C_v", "C_w", "P_u", "Q_u", "P_v", "Q_v", "P_w", "Q_w", "courant",
             "nonfinite"]
    out = {n: float(b[q]) for q, n in enumerate(names)}
    for s in range(nscal):
        out[f"C_s{s}"] = float(b[B_SCALAR0 + 3 * s])
        out[f"M_s{s}"] = float(b[B_SCALAR0 + 3 * s + 1])
        out[f"min_s{s}"] = float(b[B_SCALAR0 + 3 * s + 2])
    return out


# ---------------------------------------------------------------------------
# Batched ensemble
# ---------------------------------------------------------------------------
class MoncMember(C.Structure):
    """Mirror of the C struct monc_member."""
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double),
                ("rdz", C.c_void_p), ("rho", C.c_void_p), ("rhon", C.c_void_p),
                ("state", (C.c_void_p * (3 + MONC_MAX_SCALARS)) * 2),
                ("phi0", C.c_double * MONC_MAX_SCALARS)]


class Ensemble:
    """An ensemble plan.  members: list of dicts with keys state0, state1 (lists
    of 3+nscal float64 device tensors in the padded layout), prof (rdz, rho,
    rhon device tensors), dx, dy, dt, phi0 (list of nscal floats).  The plan
    keeps references to the tensors until close()."""

    def __init__(self, members, nscal, tune_cache=None, tune=True):
        torch = _torch()
        self._keep = members
        arr = (MoncMember * len(members))()
        for m, mem in enumerate(members):
            nx, ny, nz = _grid(mem["state0"][0])
            sh = tuple(mem["state0"][0].shape)
            M = arr[m]
            M.nx, M.ny, M.nz = nx, ny, nz
            M.dx, M.dy, M.dt = float(mem["dx"]), float(mem["dy"]), float(mem["dt"])
            M.rdz, M.rho, M.rhon = [p.value for p in _prof(mem["prof"])]
            for p, key in enumerate(("state0", "state1")):
                for f, t in enumerate(mem[key]):
                    M.state[p][f] = _ptr(t, torch.float64, sh, f"{key}[{f}]").value
            for q, v in enumerate(mem.get("phi0", [0.0] * nscal)):
                M.phi0[q] = float(v)
        plan = C.c_void_p()
        cache = tune_cache.encode() if tune_cache else None
        _check(lib().monc_ensemble_create(C.cast(arr, C.c_void_p), len(members), nscal, cache,
                                          1 if tune else 0, C.byref(plan)),
               "monc_ensemble_create")
        self._plan = plan
        self.nscal = nscal

    def run(self, nsteps, stream=None):
        _check(lib().monc_ensemble_run(self._plan, int(nsteps), _stream(stream)),
               "monc_ensemble_run")

    def set_budgets(self, budgets):
        """Attach a float64 device tensor of shape (nslots, nmembers,
        MONC_NBUDGET) (step t of a run writes slot t), or detach with None."""
        torch = _torch()
        if budgets is None:
            _check(lib().monc_ensemble_set_budgets(self._plan, None, 0),
                   "monc_ensemble_set_budgets")
            self._budgets = None
            return
        n = len(self._keep)
        if (budgets.dtype != torch.float64 or not budgets.is_cuda or budgets.dim() != 3
                or tuple(budgets.shape[1:]) != (n, MONC_NBUDGET) or not budgets.is_contiguous()):
            raise ValueError(f"budgets must be a contiguous float64 device tensor of shape "
                             f"(nslots, {n}, {MONC_NBUDGET})")
        _check(lib().monc_ensemble_set_budgets(self._plan, budgets.data_ptr(),
                                               int(budgets.shape[0])),
               "monc_ensemble_set_budgets")
        self._budgets = budgets

    def step(self, stream=None):
        _check(lib().monc_ensemble_step(self._plan, _stream(stream)), "monc_ensemble_step")

    @property
    def parity(self):
        return int(lib().monc_ensemble_parity(self._plan))

    def info(self):
        ti, grid, nit = (C.c_int * 2)(), (C.c_int * 2)(), (C.c_int * 2)()
        lib().monc_ensemble_info(self._plan, ti, grid, nit)
        return {"ti": list(ti), "grid": list(grid), "nitems": list(nit)}

    def close(self):
        if self._plan:
            lib().monc_ensemble_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Learned coarse-grid correction
# ---------------------------------------------------------------------------
MONC_MLP_NIN, MONC_MLP_K, MONC_MLP_H, MONC_MLP_NOUT = 300, 320, 64, 4
MONC_MLP_NPARAM = (MONC_MLP_H * MONC_MLP_K + MONC_MLP_H + MONC_MLP_H * MONC_MLP_H + MONC_MLP_H
                   + MONC_MLP_NOUT * MONC_MLP_H + MONC_MLP_NOUT)
MONC_MLP_WPACK = MONC_MLP_H * MONC_MLP_K + MONC_MLP_H * MONC_MLP_H + 32 * MONC_MLP_H


def _dbl(vals):
    vals = [float(x) for x in vals]
    return (C.c_double * len(vals))(*vals)


def _opt(t):
    return None if t is None else _ptr(t)


def monc_restrict4(fine, coarse, prof, prof_c, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(fine[0])
    fa = _ptrs(fine, torch.float64, tuple(fine[0].shape), "fine")
    ca = _ptrs(coarse, torch.float64, tuple(coarse[0].shape), "coarse")
    nz_c = nz // 4
    pc = [_ptr(p, torch.float64, (nz_c,), n) for p, n in zip(prof_c, ("rdz_c", "rho_c", "rhon_c"))]
    _check(lib().monc_restrict4(len(fine) - 3, fa, ca, nx, ny, nz, *_prof(prof), *pc,
                                _stream(stream)), "monc_restrict4")


def monc_mlp_features(state, norm, orient, cells, X, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(state[0])
    sa = _ptrs(state, torch.float64, tuple(state[0].shape), "state")
    n = nx * ny * nz if cells is None else cells.numel()
    cp = None if cells is None else _ptr(cells, torch.int32, None, "cells")
    _check(lib().monc_mlp_features(sa, nx, ny, nz, _dbl(norm), int(orient), cp, n,
                                   _ptr(X, None, None, "X"), _stream(stream)), "monc_mlp_features")


def monc_mlp_pack(params, wpack, stream=None):
    _check(lib().monc_mlp_pack(_ptr(params), _ptr(wpack), _stream(stream)), "monc_mlp_pack")


def monc_mlp_infer(state, norm, orient, params, wpack, Y, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(state[0])
    sa = _ptrs(state, torch.float64, tuple(state[0].shape), "state")
    rows = nx * ny * nz * (2 if int(orient) == 2 else 1)
    _ptr(Y, torch.float32, (rows, 4), "Y")
    _check(lib().monc_mlp_infer(sa, nx, ny, nz, _dbl(norm), int(orient), _ptr(params),
                                _ptr(wpack), _ptr(Y), _stream(stream)), "monc_mlp_infer")


def monc_mlp_forward(X, m, params, wpack, Y, H1=None, H2=None, Z1=None, Z2=None, stream=None):
    _check(lib().monc_mlp_forward(_ptr(X), int(m), _ptr(params), _ptr(wpack), _ptr(Y), _opt(H1),
                                  _opt(H2), _opt(Z1), _opt(Z2), _stream(stream)),
           "monc_mlp_forward")


def monc_mlp_backward_workspace_bytes(m):
    return int(lib().monc_mlp_backward_workspace_bytes(int(m)))


def monc_mlp_backward(X, H1, H2, Z1, Z2, dY, m, wpack, grad, workspace, stream=None):
    _check(lib().monc_mlp_backward(_ptr(X), _ptr(H1), _ptr(H2), _ptr(Z1), _ptr(Z2), _ptr(dY),
                                   int(m), _ptr(wpack), _ptr(grad), _ptr(workspace),
                                   _stream(stream)), "monc_mlp_backward")


def monc_mlp_loss_workspace_bytes(b):
    return int(lib().monc_mlp_loss_workspace_bytes(int(b)))


def monc_mlp_loss(Y4, b, cells, c0, c1, tend, dt, scale, prof_c, inv_count, dY4, loss,
                  workspace, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(c0[0])
    sh = tuple(c0[0].shape)
    a0, a1, at = (_ptrs(x, torch.float64, sh, n) for x, n in ((c0, "c0"), (c1, "c1"), (tend, "tend")))
    rdz, rho, rhon = prof_c
    _check(lib().monc_mlp_loss(_ptr(Y4), int(b), _ptr(cells, torch.int32), a0, a1, at, nx, ny, nz,
                               float(dt), _dbl(scale), _ptr(rho), _ptr(rhon), float(inv_count),
                               _ptr(dY4), _ptr(loss), _ptr(workspace), _stream(stream)),
           "monc_mlp_loss")


def monc_mlp_adam(params, m1, m2, grad, t, lr, b1, b2, eps, wpack, stream=None):
    _check(lib().monc_mlp_adam(_ptr(params), _ptr(m1), _ptr(m2), _ptr(grad), int(t), float(lr),
                               float(b1), float(b2), float(eps), _ptr(wpack), _stream(stream)),
           "monc_mlp_adam")


def monc_mlp_train_workspace_bytes(b):
    return int(lib().monc_mlp_train_workspace_bytes(int(b)))


def monc_mlp_train_step(c0, c1, tend, norm, cells, dt, scale, prof_c, inv_count, params, m1, m2,
                        t, lr, b1, b2, eps, wpack, grad, loss, workspace, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(c0[0])
    sh = tuple(c0[0].shape)
    a0, a1, at = (_ptrs(x, torch.float64, sh, n) for x, n in ((c0, "c0"), (c1, "c1"), (tend, "tend")))
    rdz, rho, rhon = prof_c
    _check(lib().monc_mlp_train_step(a0, a1, at, nx, ny, nz, _dbl(norm),
                                     _ptr(cells, torch.int32, None, "cells"), cells.numel(),
                                     float(dt), _dbl(scale), _ptr(rho), _ptr(rhon),
                                     float(inv_count), _ptr(params), _ptr(m1), _ptr(m2), int(t),
                                     float(lr), float(b1), float(b2), float(eps), _ptr(wpack),
                                     _ptr(grad), _ptr(loss), _ptr(workspace), _stream(stream)),
           "monc_mlp_train_step")


def monc_correct_step_workspace_bytes(nx, ny, nz):
    return int(lib().monc_correct_step_workspace_bytes(int(nx), int(ny), int(nz)))


def monc_correct_step(state_in, tend, gx, gy, state_out, dx, dy, scale, prof_c, dt, growth,
                      flags, workspace, stream=None):
    torch = _torch()
    nx, ny, nz = _grid(state_in[0])
    sh = tuple(state_in[0].shape)
    ia = _ptrs(state_in, torch.float64, sh, "state_in")
    ta = _ptrs(tend, torch.float64, sh, "tend")
    oa = _ptrs(state_out, torch.float64, sh, "state_out")
    rdz, rho, rhon = prof_c
    _check(lib().monc_correct_step(ia, ta, _ptr(gx), _ptr(gy), oa, nx, ny, nz, float(dx),
                                   float(dy), _dbl(scale), _ptr(rdz), _ptr(rho), _ptr(rhon),
                                   float(dt), float(growth), _ptr(flags, torch.int32),
                                   _ptr(workspace), _stream(stream)), "monc_correct_step")

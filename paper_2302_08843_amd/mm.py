"""Thin ctypes binding of the C ABI in include/mm.h.

Every function here only marshals arguments: device buffers come from torch
tensors (``tensor.data_ptr()``), the stream from torch's current stream, and
all arithmetic runs in libmmx.so.  If the library is missing this module
raises -- there is no fallback.

Vector fields are torch tensors of shape (3, nz, ny, nx) (component-major, x
fastest), dtype float32 for MM_FP32 plans and float64 for MM_FP64 plans, on
the plan's device.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmx.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EHIP, MM_ENONFINITE, MM_EDTMIN, MM_ENOTCONV, MM_EBUSY = (
    0, -1, -2, -3, -4, -5, -6, -7)
MM_FP32, MM_FP64 = 0, 1
MM_DEMAG, MM_EXCH, MM_ANIS, MM_ZEEMAN, MM_DMI, MM_OERSTED, MM_ALL = 1, 2, 4, 8, 16, 32, 63
MM_DMI_INTERFACE, MM_DMI_BULK, MM_DMI_D2D = 0, 1, 2

STATUS_NAMES = {0: "MM_OK", -1: "MM_EINVAL", -2: "MM_ENOMEM", -3: "MM_EHIP", -4: "MM_ENONFINITE",
                -5: "MM_EDTMIN", -6: "MM_ENOTCONV", -7: "MM_EBUSY"}

# Every entry point declared in include/mm.h.
EXPORTS = ["mm_opts_default", "mm_plan_create", "mm_plan_destroy", "mm_plan_device_bytes",
           "mm_plan_workspace_bytes", "mm_energy_noalloc",
           "mm_plan_padded", "mm_set_ms", "mm_set_exchange", "mm_set_ku", "mm_set_dmi",
           "mm_oersted", "mm_set_current", "mm_set_drive", "mm_heff", "mm_llg_rhs", "mm_llg_step",
           "mm_relax", "mm_energy", "mm_max_torque", "mm_profile", "mm_profile_read",
           "mm_debug_kernel", "mm_debug_spectrum", "mm_last_error", "mm_heff_vjp",
           "mm_llg_rhs_vjp", "mm_rk4_forward", "mm_rk4_adjoint", "mm_serve_opts_default",
           "mm_serve_create", "mm_serve_submit", "mm_serve_poll", "mm_serve_get_stats",
           "mm_serve_destroy", "mm_serve_clock"]

MM_SERVE_RELAX, MM_SERVE_INTEGRATE = 0, 1
MM_DP45, MM_RKF45 = 0, 1

PASS_NAMES = ["x_fwd", "y_fwd", "mid", "y_inv", "x_inv_local", "rk"]
MM_NPASS = len(PASS_NAMES)


class mm_serve_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int), ("steps_per_launch", C.c_int),
                ("prec", C.c_int), ("demag_p", C.c_int), ("batch", C.c_int)]


class mm_request(C.Structure):
    _fields_ = [("grid", C.c_int * 3), ("cell", C.c_double * 3), ("Ms", C.c_double),
                ("A", C.c_double), ("Ku", C.c_double), ("ku_axis", C.c_double * 3),
                ("alpha", C.c_double), ("h_ext", C.c_double * 3), ("terms", C.c_uint),
                ("kind", C.c_int), ("tol", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("t_end", C.c_double), ("max_steps", C.c_long), ("m", C.c_void_p),
                ("stream", C.c_void_p), ("tag", C.c_long)]


class mm_completion(C.Structure):
    _fields_ = [("tag", C.c_long), ("status", C.c_int), ("accepted", C.c_long),
                ("rejected", C.c_long), ("rhs_evals", C.c_long), ("t", C.c_double),
                ("torque", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


class mm_serve_stats(C.Structure):
    _fields_ = [(n, C.c_long) for n in ("submitted", "admitted", "completed", "queued", "active",
                                        "waited_memory", "waited_slot")] + \
               [(n, C.c_size_t) for n in ("bytes_in_use", "bytes_peak", "budget")] + \
               [(n, C.c_long) for n in ("tensors_built", "plans_created", "plans_reused",
                                        "graph_launches", "max_batch")]


class mm_opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("ku_axis", C.c_double * 3), ("demag_p", C.c_int),
                ("stream", C.c_void_p), ("ku2", C.c_double), ("kc1", C.c_double),
                ("kc2", C.c_double), ("kc_axis1", C.c_double * 3), ("kc_axis2", C.c_double * 3),
                ("dz_layers", C.POINTER(C.c_double)), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class mm_step_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("t_end", C.c_double),
                ("max_steps", C.c_long), ("dt_min", C.c_double), ("renorm", C.c_int),
                ("method", C.c_int)]


class mm_step_stats(C.Structure):
    _fields_ = [("accepted", C.c_long), ("rejected", C.c_long), ("rhs_evals", C.c_long),
                ("t", C.c_double), ("dt", C.c_double), ("err_last", C.c_double)]


def _destroy_plan(fn, handle):
    # fn is the library's mm_plan_destroy, held by the finalizer itself
    _PLANS.pop(handle, None)
    fn(C.c_void_p(handle))


def _destroy_server(fn, handle):
    fn(C.c_void_p(handle))


class MMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """Load libmmx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmmx.so is not built: run `python -m paper_2302_08843_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.mm_opts_default.argtypes = [C.POINTER(mm_opts)]
        L.mm_opts_default.restype = None
        L.mm_plan_create.argtypes = [C.POINTER(vp), ip, dp, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.POINTER(mm_opts)]
        L.mm_plan_destroy.argtypes = [vp]
        L.mm_plan_destroy.restype = None
        L.mm_plan_device_bytes.argtypes = [vp]
        L.mm_plan_device_bytes.restype = C.c_size_t
        L.mm_plan_workspace_bytes.argtypes = [ip, C.c_int]
        L.mm_plan_workspace_bytes.restype = C.c_size_t
        L.mm_plan_padded.argtypes = [vp, ip]
        L.mm_plan_padded.restype = None
        L.mm_set_ms.argtypes = [vp, vp]
        L.mm_set_exchange.argtypes = [vp, vp]
        L.mm_set_ku.argtypes = [vp, vp]
        L.mm_set_dmi.argtypes = [vp, C.c_int, C.c_double, vp]
        L.mm_oersted.argtypes = [vp, vp, vp]
        L.mm_set_current.argtypes = [vp, vp, C.c_double]
        L.mm_set_drive.argtypes = [vp, dp, C.c_double, vp]
        L.mm_heff.argtypes = [vp, vp, dp, C.c_uint, C.c_double, vp]
        L.mm_llg_rhs.argtypes = [vp, vp, dp, C.c_uint, C.c_double, vp]
        L.mm_llg_step.argtypes = [vp, vp, dp, C.c_uint, dp, dp, C.POINTER(mm_step_opts),
                                  C.POINTER(mm_step_stats)]
        L.mm_relax.argtypes = [vp, vp, dp, C.c_uint, C.c_double, C.c_long, C.c_double,
                               C.POINTER(mm_step_stats)]
        L.mm_energy.argtypes = [vp, vp, dp, C.c_uint, C.c_double, dp]
        L.mm_max_torque.argtypes = [vp, vp, dp, C.c_uint, C.c_double, dp]
        L.mm_profile.argtypes = [vp, C.c_int]
        L.mm_profile_read.argtypes = [vp, dp, C.POINTER(C.c_long)]
        L.mm_debug_kernel.argtypes = [vp, C.c_int, vp]
        L.mm_debug_spectrum.argtypes = [vp, C.c_int, vp]
        L.mm_serve_opts_default.argtypes = [C.POINTER(mm_serve_opts)]
        L.mm_serve_opts_default.restype = None
        L.mm_serve_create.argtypes = [C.POINTER(vp), C.POINTER(mm_serve_opts)]
        L.mm_serve_submit.argtypes = [vp, C.POINTER(mm_request)]
        L.mm_serve_poll.argtypes = [vp, C.POINTER(mm_completion), C.c_int, C.POINTER(C.c_int)]
        L.mm_serve_get_stats.argtypes = [vp, C.POINTER(mm_serve_stats)]
        L.mm_serve_destroy.argtypes = [vp]
        L.mm_serve_destroy.restype = None
        L.mm_serve_clock.argtypes = []
        L.mm_serve_clock.restype = C.c_double
        L.mm_heff_vjp.argtypes = [vp, vp, vp, C.c_uint, vp, vp]
        L.mm_llg_rhs_vjp.argtypes = [vp, vp, dp, C.c_uint, C.c_double, vp, vp, vp]
        L.mm_rk4_forward.argtypes = [vp, vp, dp, C.c_uint, C.c_double, C.c_double, C.c_long, vp,
                                     C.c_long, vp, dp]
        L.mm_rk4_adjoint.argtypes = [vp, vp, dp, C.c_uint, C.c_double, C.c_double, C.c_long, vp,
                                     C.c_long, vp, vp, dp]
        L.mm_last_error.restype = C.c_char_p
        L.mm_energy_noalloc.argtypes = [vp, vp, dp, C.c_uint, C.c_double, dp]
        for name in ("mm_plan_create", "mm_energy_noalloc", "mm_set_ms", "mm_set_exchange", "mm_set_ku", "mm_set_dmi", "mm_oersted",
                     "mm_set_current",
                     "mm_set_drive", "mm_heff", "mm_llg_rhs",
                     "mm_llg_step", "mm_relax", "mm_energy", "mm_max_torque", "mm_profile",
                     "mm_profile_read", "mm_debug_kernel", "mm_debug_spectrum", "mm_heff_vjp",
                     "mm_llg_rhs_vjp", "mm_rk4_forward", "mm_rk4_adjoint", "mm_serve_create",
                     "mm_serve_submit", "mm_serve_poll", "mm_serve_get_stats"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != MM_OK:
        raise MMError(status, lib().mm_last_error().decode())
    return status


def _vec3(v):
    if v is None:
        return None
    a = (C.c_double * 3)(*[float(x) for x in np.asarray(v, dtype=np.float64).reshape(3)])
    return a


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


# Plans created through this module: handle value -> (grid, dtype name, device
# index), so that every tensor handed to the library is checked against the
# plan it is meant for before any call (a wrong dtype, shape or device would
# otherwise make the kernels read or write out of bounds).
_PLANS = {}


def _plan_info(plan):
    info = _PLANS.get(plan.value if isinstance(plan, C.c_void_p) else plan)
    if info is None:
        raise ValueError("unknown plan handle")
    return info


def _expect(t, name, dtype, device, shape):
    """Raise ValueError unless t is a contiguous tensor of `dtype` on CUDA
    device `device` with exactly `shape`."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s (got %s)" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if not t.is_cuda or t.device.index != device:
        raise ValueError("%s must live on cuda:%d (got %s)" % (name, device, t.device))
    return C.c_void_p(t.data_ptr())


def _vec(plan, t, name):
    """A vector field (3, nz, ny, nx) of the plan's precision."""
    grid, dt, dev = _plan_info(plan)
    import torch

    nx, ny, nz = grid
    return _expect(t, name, getattr(torch, dt), dev, (3, nz, ny, nx))


def _cellf(plan, t, name, dtype=None):
    """A scalar per-cell field (nz, ny, nx) of the plan's precision (or dtype)."""
    grid, dt, dev = _plan_info(plan)
    import torch

    nx, ny, nz = grid
    return _expect(t, name, dtype if dtype is not None else getattr(torch, dt), dev, (nz, ny, nx))


def _ovec(plan, t, name):
    return None if t is None else _vec(plan, t, name)


def _ocellf(plan, t, name, dtype=None):
    return None if t is None else _cellf(plan, t, name, dtype)


# ---------------------------------------------------------------------------
# Functions with the C names (argument marshalling only)
# ---------------------------------------------------------------------------

def mm_opts_default():
    o = mm_opts()
    lib().mm_opts_default(C.byref(o))
    return o


def mm_plan_create(grid, cell, Ms, A, Ku, alpha, opts=None):
    h = C.c_void_p()
    g = (C.c_int * 3)(*[int(v) for v in grid])
    d = (C.c_double * 3)(*[float(v) for v in cell])
    _check(lib().mm_plan_create(C.byref(h), g, d, float(Ms), float(A), float(Ku), float(alpha),
                                C.byref(opts) if opts is not None else None))
    import torch

    prec = opts.prec if opts is not None else MM_FP64
    _PLANS[h.value] = (tuple(int(v) for v in grid), "float32" if prec == MM_FP32 else "float64",
                       torch.cuda.current_device() if torch.cuda.is_available() else -1)
    return h


def mm_plan_destroy(plan):
    _PLANS.pop(plan.value if isinstance(plan, C.c_void_p) else plan, None)
    lib().mm_plan_destroy(plan)


def mm_heff(plan, m, h_ext, terms, t, h_out):
    _check(lib().mm_heff(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t),
                         _vec(plan, h_out, "h_out")))


def mm_llg_rhs(plan, m, h_ext, terms, t, dmdt_out):
    _check(lib().mm_llg_rhs(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t),
                            _vec(plan, dmdt_out, "dmdt_out")))


def mm_set_ms(plan, Ms_cell):
    _check(lib().mm_set_ms(plan, _ocellf(plan, Ms_cell, "Ms_cell")))


def mm_set_exchange(plan, A_cell):
    _check(lib().mm_set_exchange(plan, _ocellf(plan, A_cell, "A_cell")))


def mm_set_ku(plan, Ku_cell):
    _check(lib().mm_set_ku(plan, _ocellf(plan, Ku_cell, "Ku_cell")))


def mm_set_dmi(plan, kind, D, D_cell):
    _check(lib().mm_set_dmi(plan, int(kind), float(D), _ocellf(plan, D_cell, "D_cell")))


def mm_oersted(plan, j, h_out):
    _check(lib().mm_oersted(plan, _vec(plan, j, "j"), _vec(plan, h_out, "h_out")))


def mm_set_current(plan, j, freq):
    _check(lib().mm_set_current(plan, _ovec(plan, j, "j"), float(freq)))


def mm_set_drive(plan, amp, freq, mask):
    import torch

    _check(lib().mm_set_drive(plan, _vec3(amp), float(freq),
                              _ocellf(plan, mask, "mask", torch.uint8)))


def mm_llg_step(plan, m, h_ext, terms, t, dt, opts):
    pm = _vec(plan, m, "m")
    tt, dd = C.c_double(t), C.c_double(dt)
    st = mm_step_stats()
    status = lib().mm_llg_step(plan, pm, _vec3(h_ext), int(terms), C.byref(tt), C.byref(dd),
                               C.byref(opts), C.byref(st))
    return status, tt.value, dd.value, st


def mm_relax(plan, m, h_ext, terms, tol, max_steps, rtol):
    pm = _vec(plan, m, "m")
    st = mm_step_stats()
    status = lib().mm_relax(plan, pm, _vec3(h_ext), int(terms), float(tol), int(max_steps),
                            float(rtol), C.byref(st))
    return status, st


def mm_energy(plan, m, h_ext, terms, t):
    E = (C.c_double * 6)()
    _check(lib().mm_energy(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t), E))
    return np.array(list(E))


def mm_energy_noalloc(plan, m, h_ext, terms, t):
    E = (C.c_double * 6)()
    _check(lib().mm_energy_noalloc(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t),
                                   E))
    return np.array(list(E))


def mm_max_torque(plan, m, h_ext, terms, t):
    out = C.c_double()
    _check(lib().mm_max_torque(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t),
                               C.byref(out)))
    return out.value


def mm_profile(plan, enable):
    _check(lib().mm_profile(plan, int(bool(enable))))


def mm_profile_read(plan):
    ms = (C.c_double * MM_NPASS)()
    cnt = (C.c_long * MM_NPASS)()
    _check(lib().mm_profile_read(plan, ms, cnt))
    return {PASS_NAMES[i]: (ms[i], cnt[i]) for i in range(MM_NPASS)}


def _padded_f64(plan, t, name, spectrum):
    import torch

    P = mm_plan_padded(plan)
    Px, Py, Pz = P
    shape = ((Pz // 2 + 1, Py // 2 + 1, Px // 2 + 1 if Px > 1 else 1) if spectrum
             else (Pz, Py, Px))
    return _expect(t, name, torch.float64, _plan_info(plan)[2], shape)


def mm_debug_kernel(plan, s, out):
    _check(lib().mm_debug_kernel(plan, int(s), _padded_f64(plan, out, "out", False)))


def mm_debug_spectrum(plan, s, out):
    _check(lib().mm_debug_spectrum(plan, int(s), _padded_f64(plan, out, "out", True)))


def _ckpt(plan, ck, nsteps, ckpt_every, name):
    """Checkpoints (K, 3, nz, ny, nx) with K >= ceil(nsteps / ckpt_every), the
    number the library reads or writes (argument errors such as a
    non-positive step count are left to the library)."""
    if ck is None:
        return None
    grid, dt, dev = _plan_info(plan)
    import torch

    nx, ny, nz = grid
    nck = 1
    if int(ckpt_every) > 0:
        nck = max((int(nsteps) + int(ckpt_every) - 1) // int(ckpt_every), 1)
    shape = (max(int(ck.shape[0]), nck) if isinstance(ck, torch.Tensor) and ck.dim() == 5 else nck,
             3, nz, ny, nx)
    if isinstance(ck, torch.Tensor) and ck.dim() == 5 and int(ck.shape[0]) < nck:
        raise ValueError("%s holds %d checkpoints, %d needed" % (name, int(ck.shape[0]), nck))
    return _expect(ck, name, getattr(torch, dt), dev, shape)


def mm_heff_vjp(plan, m, w, terms, grad_m, grad_ms):
    _check(lib().mm_heff_vjp(plan, _vec(plan, m, "m"), _vec(plan, w, "w"), int(terms),
                             _vec(plan, grad_m, "grad_m"), _ocellf(plan, grad_ms, "grad_ms")))


def mm_llg_rhs_vjp(plan, m, h_ext, terms, t, w, grad_m, grad_ms):
    _check(lib().mm_llg_rhs_vjp(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t),
                                _vec(plan, w, "w"), _vec(plan, grad_m, "grad_m"),
                                _ocellf(plan, grad_ms, "grad_ms")))


def mm_rk4_forward(plan, m, h_ext, terms, t0, dt, nsteps, region, ckpt_every, ckpt):
    import torch

    loss = C.c_double()
    _check(lib().mm_rk4_forward(plan, _vec(plan, m, "m"), _vec3(h_ext), int(terms), float(t0),
                                float(dt), int(nsteps), _ocellf(plan, region, "region", torch.uint8),
                                int(ckpt_every), _ckpt(plan, ckpt, nsteps, ckpt_every, "ckpt"),
                                C.byref(loss)))
    return loss.value


def mm_rk4_adjoint(plan, ckpt, h_ext, terms, t0, dt, nsteps, region, ckpt_every, grad_ms,
                   grad_m0):
    import torch

    loss = C.c_double()
    if ckpt is None:
        raise ValueError("ckpt is required")
    _check(lib().mm_rk4_adjoint(plan, _ckpt(plan, ckpt, nsteps, ckpt_every, "ckpt"), _vec3(h_ext),
                                int(terms), float(t0), float(dt), int(nsteps),
                                _ocellf(plan, region, "region", torch.uint8), int(ckpt_every),
                                _ocellf(plan, grad_ms, "grad_ms"), _ovec(plan, grad_m0, "grad_m0"),
                                C.byref(loss)))
    return loss.value


def mm_serve_opts_default():
    o = mm_serve_opts()
    lib().mm_serve_opts_default(C.byref(o))
    return o


def mm_serve_create(opts=None):
    h = C.c_void_p()
    _check(lib().mm_serve_create(C.byref(h), None if opts is None else C.byref(opts)))
    return h


def mm_serve_submit(server, req):
    _check(lib().mm_serve_submit(server, C.byref(req)))


def mm_serve_poll(server, max_out=256):
    buf = (mm_completion * max_out)()
    n = C.c_int()
    _check(lib().mm_serve_poll(server, buf, int(max_out), C.byref(n)))
    return [buf[i] for i in range(n.value)]


def mm_serve_get_stats(server):
    st = mm_serve_stats()
    _check(lib().mm_serve_get_stats(server, C.byref(st)))
    return st


def mm_serve_destroy(server):
    lib().mm_serve_destroy(server)


def mm_serve_clock():
    return float(lib().mm_serve_clock())


def mm_plan_padded(plan):
    P = (C.c_int * 3)()
    lib().mm_plan_padded(plan, P)
    return tuple(P)


def mm_plan_device_bytes(plan):
    return int(lib().mm_plan_device_bytes(plan))


def mm_plan_workspace_bytes(grid, prec):
    g = (C.c_int * 3)(*[int(v) for v in grid])
    return int(lib().mm_plan_workspace_bytes(g, int(prec)))


# ---------------------------------------------------------------------------
# Convenience object (same calls, holds the handle and the tensor dtype)
# ---------------------------------------------------------------------------

class Plan:
    """A plan on the current CUDA (HIP) device; see mm_plan_create."""

    def __init__(self, grid, cell, Ms, A=0.0, Ku=0.0, alpha=0.5, prec="fp64", ku_axis=(0, 0, 1),
                 demag_p=20, stream=None, Ku2=0.0, Kc1=0.0, Kc2=0.0, kc_axes=((1, 0, 0), (0, 1, 0)),
                 layers=None, workspace=None):
        """workspace: optional device tensor (any dtype, contiguous, at least
        mm_plan_workspace_bytes(grid, prec) bytes) that holds the plan's
        persistent buffers; the plan keeps a reference to it."""
        import torch

        self.grid = tuple(int(v) for v in grid)
        self.cell = tuple(float(v) for v in cell)
        self.prec = MM_FP32 if prec in ("fp32", MM_FP32, "f32") else MM_FP64
        self.dtype = torch.float32 if self.prec == MM_FP32 else torch.float64
        self.device = torch.device("cuda", torch.cuda.current_device())
        o = mm_opts_default()
        o.prec = self.prec
        for a in range(3):
            o.ku_axis[a] = float(ku_axis[a])
        o.demag_p = int(demag_p)
        o.stream = _stream_handle(stream)
        o.ku2, o.kc1, o.kc2 = float(Ku2), float(Kc1), float(Kc2)
        for a in range(3):
            o.kc_axis1[a] = float(kc_axes[0][a])
            o.kc_axis2[a] = float(kc_axes[1][a])
        self._stream = stream
        self.layers = None
        if layers is not None:
            # thin layers of unequal height (read during creation only)
            self.layers = np.ascontiguousarray(np.asarray(layers, dtype=np.float64))
            assert self.layers.shape == (self.grid[2],), "one height per layer"
            o.dz_layers = self.layers.ctypes.data_as(C.POINTER(C.c_double))
        self.workspace = workspace
        if workspace is not None:
            if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or \
                    not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            o.workspace = C.c_void_p(workspace.data_ptr())
            o.workspace_bytes = workspace.numel() * workspace.element_size()
        self.handle = mm_plan_create(self.grid, self.cell, Ms, A, Ku, alpha, o)
        nx, ny, nz = self.grid
        self.shape = (3, nz, ny, nx)
        # destroyed through the ABI when collected or, at the latest, at
        # interpreter exit (finalizers run before module teardown)
        self._fin = weakref.finalize(self, _destroy_plan, lib().mm_plan_destroy, self.handle.value)

    def close(self):
        """Release the plan's device memory now."""
        self._fin()
        self.handle = None

    def _t(self, a):
        import torch

        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=self.dtype).contiguous()

    def empty(self):
        import torch

        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    def _v(self, a):
        """A vector field as a (3, nz, ny, nx) tensor of the plan's dtype."""
        return self._t(a).reshape(self.shape)

    def heff(self, m, h_ext=None, terms=MM_ALL, t=0.0, out=None):
        m = self._v(m)
        out = self.empty() if out is None else out
        mm_heff(self.handle, m, h_ext, terms, t, out)
        return out

    def llg_rhs(self, m, h_ext=None, terms=MM_ALL, t=0.0, out=None):
        m = self._v(m)
        out = self.empty() if out is None else out
        mm_llg_rhs(self.handle, m, h_ext, terms, t, out)
        return out

    def set_ms(self, Ms_cell):
        import torch

        if Ms_cell is None:
            mm_set_ms(self.handle, None)
            return
        nx, ny, nz = self.grid
        mm_set_ms(self.handle, self._t(Ms_cell).reshape(nz, ny, nx).contiguous())
        torch.cuda.current_stream().synchronize()

    def set_exchange(self, A_cell):
        """Per-cell exchange constant (None: the uniform A of the plan)."""
        import torch

        if A_cell is None:
            mm_set_exchange(self.handle, None)
            return
        nx, ny, nz = self.grid
        mm_set_exchange(self.handle, self._t(A_cell).reshape(nz, ny, nx).contiguous())
        torch.cuda.current_stream().synchronize()

    def set_ku(self, Ku_cell):
        """Per-cell first-order uniaxial constant (None: the uniform Ku)."""
        import torch

        if Ku_cell is None:
            mm_set_ku(self.handle, None)
            return
        nx, ny, nz = self.grid
        mm_set_ku(self.handle, self._t(Ku_cell).reshape(nz, ny, nx).contiguous())
        torch.cuda.current_stream().synchronize()

    def set_dmi(self, D, kind=MM_DMI_INTERFACE):
        """DMI of type `kind` with a uniform (scalar) or per-cell strength D
        in J/m^2; D=None or 0 removes it."""
        import torch

        if D is None or (np.ndim(D) == 0 and not hasattr(D, "device")):
            mm_set_dmi(self.handle, kind, 0.0 if D is None else float(D), None)
            return
        nx, ny, nz = self.grid
        mm_set_dmi(self.handle, kind, 0.0, self._t(D).reshape(nz, ny, nx).contiguous())
        torch.cuda.current_stream().synchronize()

    def oersted(self, j, out=None):
        """Oersted field of the current density j (A/m^2, shape (3, nz, ny, nx))."""
        j = self._v(j)
        out = self.empty() if out is None else out
        mm_oersted(self.handle, j, out)
        return out

    def set_current(self, j, freq=0.0):
        """Current density for the MM_OERSTED term (None removes it)."""
        import torch

        if j is None:
            mm_set_current(self.handle, None, 0.0)
            return
        mm_set_current(self.handle, self._v(j), freq)
        torch.cuda.current_stream().synchronize()

    def set_drive(self, amp, freq, mask):
        import torch

        if mask is None:
            mm_set_drive(self.handle, None, 0.0, None)
            return
        nx, ny, nz = self.grid
        mk = torch.as_tensor(np.asarray(mask, dtype=np.uint8)).to(self.device).reshape(
            nz, ny, nx).contiguous()
        mm_set_drive(self.handle, amp, freq, mk)
        torch.cuda.current_stream().synchronize()

    def llg_step(self, m, h_ext=None, terms=MM_ALL, t=0.0, dt=-1.0, rtol=1e-6, atol=None,
                 t_end=float("inf"), max_steps=1 << 40, renorm=False, dt_min=0.0, check=True,
                 method=MM_DP45):
        """Advance m (a plan-dtype device tensor, updated in place)."""
        o = mm_step_opts(rtol=rtol, atol=rtol if atol is None else atol, t_end=t_end,
                         max_steps=max_steps, dt_min=dt_min, renorm=int(bool(renorm)),
                         method=int(method))
        status, t, dt, st = mm_llg_step(self.handle, m, h_ext, terms, t, dt, o)
        if check:
            _check(status)
        return status, t, dt, _stats(st)

    def relax(self, m, h_ext=None, terms=MM_ALL, tol=1e-5, max_steps=50000, rtol=1e-4):
        status, st = mm_relax(self.handle, m, h_ext, terms, tol, max_steps, rtol)
        return status, _stats(st)

    def energy(self, m, h_ext=None, terms=MM_ALL, t=0.0):
        return mm_energy(self.handle, self._v(m), h_ext, terms, t)

    def max_torque(self, m, h_ext=None, terms=MM_ALL, t=0.0):
        return mm_max_torque(self.handle, self._v(m), h_ext, terms, t)

    def padded(self):
        return mm_plan_padded(self.handle)

    def profile(self, enable=True):
        mm_profile(self.handle, enable)

    def profile_read(self):
        """{pass name: (total ms, launches)} since profiling was enabled."""
        return mm_profile_read(self.handle)

    def device_bytes(self):
        return mm_plan_device_bytes(self.handle)

    def debug_kernel(self, s):
        import torch

        Px, Py, Pz = self.padded()
        out = torch.empty((Pz, Py, Px), dtype=torch.float64, device=self.device)
        mm_debug_kernel(self.handle, s, out)
        return out

    def heff_vjp(self, m, w, terms=MM_ALL, want_ms=True):
        """(H^T w, d(w.h)/dMs) for the linear terms in `terms`."""
        m, w = self._v(m), self._v(w)
        gm = self.empty()
        gms = self._scalar_field() if want_ms else None
        mm_heff_vjp(self.handle, m, w, terms, gm, gms)
        return gm, gms

    def llg_rhs_vjp(self, m, w, h_ext=None, terms=MM_ALL, t=0.0, want_ms=True):
        """(J^T w, d(w.f)/dMs) of the LLG right-hand side at (m, t)."""
        m, w = self._v(m), self._v(w)
        gm = self.empty()
        gms = self._scalar_field() if want_ms else None
        mm_llg_rhs_vjp(self.handle, m, h_ext, terms, t, w, gm, gms)
        return gm, gms

    def _scalar_field(self):
        import torch

        nx, ny, nz = self.grid
        return torch.empty((nz, ny, nx), dtype=self.dtype, device=self.device)

    def _region(self, region):
        import torch

        if region is None:
            return None
        nx, ny, nz = self.grid
        if isinstance(region, torch.Tensor):
            return region.to(device=self.device, dtype=torch.uint8).reshape(nz, ny, nx).contiguous()
        return torch.as_tensor(np.ascontiguousarray(region, dtype=np.uint8)).to(
            self.device).reshape(nz, ny, nx).contiguous()

    def rk4(self, m, dt, nsteps, region=None, h_ext=None, terms=MM_ALL, t0=0.0, ckpt_every=0):
        """Fixed-step RK4 (m advanced in place).  Returns (loss, checkpoints or
        None); checkpoints are the states before every ckpt_every-th step."""
        import torch

        ck = None
        if ckpt_every > 0:
            nck = (int(nsteps) + ckpt_every - 1) // ckpt_every
            ck = torch.empty((max(nck, 1),) + self.shape, dtype=self.dtype, device=self.device)
        loss = mm_rk4_forward(self.handle, m, h_ext, terms, t0, dt, nsteps, self._region(region),
                              ckpt_every, ck)
        return loss, ck

    def rk4_adjoint(self, ckpt, dt, nsteps, region, h_ext=None, terms=MM_ALL, t0=0.0,
                    ckpt_every=50, want_m0=True):
        """(loss, dL/dMs, dL/dm0) of the RK4 region loss, from checkpoints."""
        gms = self._scalar_field()
        gm0 = self.empty() if want_m0 else None
        loss = mm_rk4_adjoint(self.handle, ckpt, h_ext, terms, t0, dt, nsteps,
                              self._region(region), ckpt_every, gms, gm0)
        return loss, gms, gm0

    def debug_spectrum(self, s):
        import torch

        Px, Py, Pz = self.padded()
        hx = Px // 2 + 1 if Px > 1 else 1
        out = torch.empty((Pz // 2 + 1, Py // 2 + 1, hx), dtype=torch.float64, device=self.device)
        mm_debug_spectrum(self.handle, s, out)
        return out


def _stats(st):
    return dict(accepted=st.accepted, rejected=st.rejected, rhs_evals=st.rhs_evals, t=st.t,
                dt=st.dt, err_last=st.err_last)


class RegionLoss:
    """Differentiable map Ms (per cell) -> time-averaged region m_z after RK4
    integration, for gradient-based inverse design (Sec. 5.2).  `apply(Ms)`
    returns a 0-d tensor whose backward runs the discrete adjoint on the GPU.
    The plan keeps the checkpoint segment between calls."""

    def __init__(self, plan, m0, dt, nsteps, region, h_ext=None, terms=MM_ALL, t0=0.0,
                 ckpt_every=50):
        self.plan, self.m0 = plan, plan._v(m0)
        self.dt, self.nsteps, self.region = float(dt), int(nsteps), plan._region(region)
        self.h_ext, self.terms, self.t0, self.every = h_ext, terms, float(t0), int(ckpt_every)

    def apply(self, Ms):
        import torch

        outer = self

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, ms):
                p = outer.plan
                p.set_ms(ms.detach())
                m = outer.m0.clone()
                loss, ck = p.rk4(m, outer.dt, outer.nsteps, outer.region, outer.h_ext,
                                 outer.terms, outer.t0, outer.every)
                ctx.save_for_backward(ms)
                ctx.ck = ck
                return torch.tensor(loss, dtype=torch.float64, device=ms.device)

            @staticmethod
            def backward(ctx, gout):
                (ms,) = ctx.saved_tensors
                p = outer.plan
                p.set_ms(ms.detach())
                _, gms, _ = p.rk4_adjoint(ctx.ck, outer.dt, outer.nsteps, outer.region,
                                          outer.h_ext, outer.terms, outer.t0, outer.every,
                                          want_m0=False)
                return (gout.to(gms.dtype) * gms).reshape(ms.shape)

        return _Fn.apply(Ms)


class Server:
    """Request server (mm_serve_*): submit relaxations / integrations with
    device-resident start states, poll for completions.  Results are written
    into each request's state tensor in place."""

    def __init__(self, budget=0, max_active=16, steps_per_launch=8, prec="fp32", demag_p=20,
                 batch=8):
        import torch

        o = mm_serve_opts_default()
        o.hbm_budget = int(budget)
        o.max_active = int(max_active)
        o.steps_per_launch = int(steps_per_launch)
        o.batch = int(batch)
        o.prec = MM_FP32 if prec in ("fp32", MM_FP32, "f32") else MM_FP64
        o.demag_p = int(demag_p)
        self.prec = o.prec
        self.dtype = torch.float32 if o.prec == MM_FP32 else torch.float64
        self.handle = mm_serve_create(o)
        self._held = {}
        self._fin = weakref.finalize(self, _destroy_server, lib().mm_serve_destroy,
                                     self.handle.value)

    def close(self):
        """Wait for the active requests and release the server now."""
        self._fin()
        self.handle = None

    def submit(self, m, grid, cell, Ms, A=0.0, Ku=0.0, ku_axis=(0, 0, 1), alpha=1.0, h_ext=None,
               terms=MM_ALL, kind=MM_SERVE_RELAX, tol=1e-5, rtol=1e-6, atol=None, t_end=0.0,
               max_steps=50000, tag=0):
        """m: contiguous (3, nz, ny, nx) device tensor of the server dtype,
        kept alive by the server until its completion is polled."""
        nx, ny, nz = (int(v) for v in grid)
        _expect(m, "m", self.dtype, m.device.index if m.is_cuda else -2, (3, nz, ny, nx))
        r = mm_request()
        for a in range(3):
            r.grid[a] = int(grid[a])
            r.cell[a] = float(cell[a])
            r.ku_axis[a] = float(ku_axis[a])
            r.h_ext[a] = 0.0 if h_ext is None else float(h_ext[a])
        r.Ms, r.A, r.Ku, r.alpha = float(Ms), float(A), float(Ku), float(alpha)
        r.terms, r.kind, r.tol = int(terms), int(kind), float(tol)
        r.rtol = float(rtol)
        r.atol = float(rtol if atol is None else atol)
        r.t_end, r.max_steps = float(t_end), int(max_steps)
        r.m = C.c_void_p(m.data_ptr())
        r.stream = _stream_handle(None)  # the server waits for the caller's stream
        r.tag = int(tag)
        mm_serve_submit(self.handle, r)
        self._held[int(tag)] = m

    def poll(self):
        """List of completion dicts (tag, status, accepted, rejected,
        rhs_evals, t, torque, t_submit, t_admit, t_done)."""
        out = []
        for c in mm_serve_poll(self.handle):
            d = {f: getattr(c, f) for f, _ in mm_completion._fields_}
            self._held.pop(int(c.tag), None)
            out.append(d)
        return out

    def stats(self):
        st = mm_serve_get_stats(self.handle)
        return {f: getattr(st, f) for f, _ in mm_serve_stats._fields_}

    @staticmethod
    def clock():
        return mm_serve_clock()


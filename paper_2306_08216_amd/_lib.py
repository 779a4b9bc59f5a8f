"""ctypes binding of libmdf.so: the C ABI of include/mdf.h under the same names.

This module only marshals arguments.  It raises ImportError when the HIP
library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdf.so")

MDF_OK, MDF_EINVAL, MDF_ESTATE, MDF_EDEVICE, MDF_EUNSTABLE = 0, -1, -2, -3, -4
MDF_BC_PERIODIC, MDF_BC_WALL = 0, 1

STATUS_NAMES = {0: "MDF_OK", -1: "MDF_EINVAL", -2: "MDF_ESTATE", -3: "MDF_EDEVICE", -4: "MDF_EUNSTABLE"}

_dp = C.POINTER(C.c_double)


class mdf_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("lx", C.c_double), ("ly", C.c_double),
        ("nu", C.c_double),
        ("pl_n", C.c_double), ("nu_min", C.c_double), ("nu_max", C.c_double),
        ("cfl", C.c_double), ("c", C.c_double), ("eta", C.c_double), ("s_ratio", C.c_double),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32),
        ("lid_u", C.c_double),
        ("fx", C.c_double), ("fy", C.c_double),
        ("inv_dx_x", _dp), ("inv_dx_y", _dp),
        ("dx_min", C.c_double),
        ("force_x", _dp), ("force_y", _dp),
        ("force_omega", C.c_double), ("force_phase", C.c_double), ("force_harmonic", C.c_int32),
        ("metric", _dp),
        ("mass_source", _dp),
    ]


# every exported symbol of include/mdf.h, with (restype, argtypes)
SIGNATURES = {
    "mdf_workspace_size": (C.c_size_t, [C.POINTER(mdf_params)]),
    "mdf_init": (C.c_int, [C.POINTER(mdf_params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                           C.c_void_p, C.POINTER(C.c_void_p)]),
    "mdf_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "mdf_moments": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mdf_derived": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32]),
    "mdf_diagnostics": (C.c_int, [C.c_void_p, _dp]),
    "mdf_save": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mdf_load": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mdf_set_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "mdf_set_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mdf_autotune": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "mdf_set_partition_costs": (C.c_int, [C.c_void_p, C.c_double, C.c_double]),
    "mdf_plan_segments": (C.c_int32, [C.POINTER(mdf_params), C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_int32), C.c_int32]),
    "mdf_dt": (C.c_double, [C.c_void_p]),
    "mdf_steps": (C.c_int64, [C.c_void_p]),
    "mdf_last_error": (C.c_char_p, [C.c_void_p]),
    "mdf_destroy": (None, [C.c_void_p]),
    "mdf_cnn_param_count": (C.c_int32, []),
    "mdf_cnn_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "mdf_cnn_forward": (C.c_int, [C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                  C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "mdf_cnn_forward_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_double,
                                          C.c_double, C.c_void_p, C.c_void_p]),
    "mdf_cnn_backward": (C.c_int, [C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mdf_cnn_layer_io": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mdf_cnn_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_float,
                               C.c_float, C.c_float, C.c_int32, C.c_void_p]),
    "mdf_closure_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "mdf_closure_begin": (C.c_int, [C.c_void_p]),
    "mdf_closure_apply_async": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]),
    "mdf_closure_stats": (C.c_int, [C.c_void_p, _dp]),
    "mdf_batch_workspace_size": (C.c_size_t, [C.POINTER(mdf_params), C.c_int32]),
    "mdf_batch_init": (C.c_int, [C.POINTER(mdf_params), C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    "mdf_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "mdf_batch_step_graph": (C.c_int, [C.c_void_p, C.c_int64]),
    "mdf_batch_set_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "mdf_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "mdf_batch_moments": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mdf_batch_save": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mdf_batch_derived": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint32]),
    "mdf_batch_diagnostics": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "mdf_batch_dt": (C.c_double, [C.c_void_p, C.c_int32]),
    "mdf_batch_steps": (C.c_int64, [C.c_void_p]),
    "mdf_batch_workgroups": (C.c_int32, [C.c_void_p]),
    "mdf_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "mdf_batch_destroy": (None, [C.c_void_p]),
    "mdf_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mdf_stability": (C.c_int, [C.POINTER(mdf_params), C.c_double, C.c_double, C.c_int32, _dp, _dp]),
}

_lib = None


def lib():
    """Load libmdf.so (built by __graft_entry__.build()); fail loudly if absent.
    The environment variable MDF_LIBRARY names another build of the same
    sources to load instead (the checking build libmdf_poison.so)."""
    global _lib
    if _lib is None:
        path = os.environ.get("MDF_LIBRARY", LIB_PATH)
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MdfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, ctx=None):
    if status != MDF_OK:
        msg = lib().mdf_last_error(ctx)
        raise MdfError(status, msg.decode() if msg else "")
    return status


# thin wrappers with the C names -------------------------------------------

def mdf_workspace_size(p: mdf_params) -> int:
    return lib().mdf_workspace_size(C.byref(p))


def mdf_init(p: mdf_params, u0: int, v0: int, p0: int, workspace: int, ws_bytes: int, stream: int) -> int:
    out = C.c_void_p()
    check(lib().mdf_init(C.byref(p), u0, v0, p0, workspace, ws_bytes, stream, C.byref(out)))
    return out.value


def mdf_step(ctx: int, n: int):
    return check(lib().mdf_step(ctx, int(n)), ctx)


def mdf_moments(ctx: int, u: int, v: int, p: int):
    return check(lib().mdf_moments(ctx, u, v, p), ctx)


def mdf_derived(ctx: int, out: int, mask: int):
    return check(lib().mdf_derived(ctx, out, int(mask)), ctx)


def mdf_diagnostics(ctx: int, out8):
    """out8: ctypes (c_double * 8). Returns the status (MDF_EUNSTABLE is returned, not raised)."""
    s = lib().mdf_diagnostics(ctx, out8)
    if s not in (MDF_OK, MDF_EUNSTABLE):
        check(s, ctx)
    return s


def mdf_save(ctx: int, f: int):
    return check(lib().mdf_save(ctx, f), ctx)


def mdf_load(ctx: int, f: int):
    return check(lib().mdf_load(ctx, f), ctx)


def mdf_set_kernel(ctx: int, variant: int, tile_w: int = 0, seg_h: int = 0, prefetch: int = 0):
    return check(lib().mdf_set_kernel(ctx, int(variant), int(tile_w), int(seg_h), int(prefetch)), ctx)


def mdf_plan_segments(p: mdf_params, variant: int, tile_w: int, slots: int, cap: int = 8192):
    """(strip, ys0, ys1) rows of the balanced partition, as a list of tuples."""
    buf = (C.c_int32 * (3 * cap))()
    n = lib().mdf_plan_segments(C.byref(p), int(variant), int(tile_w), int(slots), buf, int(cap))
    return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n)]


def mdf_autotune(ctx: int, steps: int):
    out = (C.c_double * 6)()
    check(lib().mdf_autotune(ctx, int(steps), out), ctx)
    return tuple(out)


def mdf_set_partition_costs(ctx: int, x_wall_scale: float, y_wall_scale: float):
    return check(lib().mdf_set_partition_costs(ctx, float(x_wall_scale), float(y_wall_scale)), ctx)


def mdf_set_fields(ctx: int, u0: int, v0: int, p0: int):
    return check(lib().mdf_set_fields(ctx, u0, v0, p0), ctx)


def mdf_dt(ctx: int) -> float:
    return lib().mdf_dt(ctx)


def mdf_steps(ctx: int) -> int:
    return lib().mdf_steps(ctx)


def mdf_last_error(ctx) -> str:
    s = lib().mdf_last_error(ctx)
    return s.decode() if s else ""


def mdf_destroy(ctx: int):
    lib().mdf_destroy(ctx)


# batches ---------------------------------------------------------------------

def bcheck(status: int, b=None):
    if status != MDF_OK:
        msg = lib().mdf_batch_last_error(b)
        raise MdfError(status, msg.decode() if msg else "")
    return status


def mdf_batch_workspace_size(ps, count: int) -> int:
    return lib().mdf_batch_workspace_size(ps, int(count))


def mdf_batch_init(ps, count: int, u0s, v0s, p0s, workspace: int, ws_bytes: int, stream: int) -> int:
    arr = C.c_void_p * count
    out = C.c_void_p()
    bcheck(lib().mdf_batch_init(ps, int(count), arr(*u0s), arr(*v0s), arr(*p0s), workspace, ws_bytes, stream,
                                C.byref(out)))
    return out.value


def mdf_batch_step(b: int, n: int):
    return bcheck(lib().mdf_batch_step(b, int(n)), b)


def mdf_batch_step_graph(b: int, n: int):
    return bcheck(lib().mdf_batch_step_graph(b, int(n)), b)


def mdf_batch_set_kernel(b: int, variant: int, tile_w: int, prefetch: int, rounds: int):
    return bcheck(lib().mdf_batch_set_kernel(b, int(variant), int(tile_w), int(prefetch), int(rounds)), b)


def mdf_batch_autotune(b: int, steps: int):
    choice = (C.c_int32 * 4)()
    bcheck(lib().mdf_batch_autotune(b, int(steps), choice), b)
    return tuple(choice)


def mdf_batch_moments(b: int, i: int, u: int, v: int, p: int):
    return bcheck(lib().mdf_batch_moments(b, int(i), u, v, p), b)


def mdf_batch_save(b: int, i: int, f: int):
    return bcheck(lib().mdf_batch_save(b, int(i), f), b)


def mdf_batch_derived(b: int, i: int, out: int, mask: int):
    return bcheck(lib().mdf_batch_derived(b, int(i), out, int(mask)), b)


def mdf_batch_diagnostics(b: int, i: int, out8):
    """Returns the status (MDF_OK or MDF_EUNSTABLE); out8 is filled either way."""
    st = lib().mdf_batch_diagnostics(b, int(i), out8)
    if st not in (MDF_OK, MDF_EUNSTABLE):
        bcheck(st, b)
    return st


def mdf_stream_copy(src: int, dst: int, nbytes: int, stream: int):
    return check(lib().mdf_stream_copy(src, dst, int(nbytes), stream))


def mdf_batch_dt(b: int, i: int) -> float:
    return lib().mdf_batch_dt(b, int(i))


def mdf_batch_steps(b: int) -> int:
    return lib().mdf_batch_steps(b)


def mdf_batch_workgroups(b: int) -> int:
    return lib().mdf_batch_workgroups(b)


def mdf_batch_last_error(b) -> str:
    s = lib().mdf_batch_last_error(b)
    return s.decode() if s else ""


def mdf_batch_destroy(b: int):
    lib().mdf_batch_destroy(b)


# learned closure -------------------------------------------------------------

def mdf_cnn_param_count() -> int:
    return lib().mdf_cnn_param_count()


def mdf_cnn_workspace_size(batch: int, h: int, w: int) -> int:
    return lib().mdf_cnn_workspace_size(int(batch), int(h), int(w))


def mdf_cnn_forward(ws: int, ws_bytes: int, params: int, batch: int, h: int, w: int, uv: int, in_scale: float,
                    out_scale: float, duv: int, stream: int):
    return check(lib().mdf_cnn_forward(ws, ws_bytes, params, int(batch), int(h), int(w), uv, float(in_scale),
                                       float(out_scale), duv, stream))


def mdf_cnn_forward_noalloc(params: int, batch: int, h: int, w: int, uv: int, in_scale: float, out_scale: float,
                            duv: int, stream: int):
    return check(lib().mdf_cnn_forward_noalloc(params, int(batch), int(h), int(w), uv, float(in_scale),
                                               float(out_scale), duv, stream))


def mdf_cnn_backward(ws: int, ws_bytes: int, params: int, batch: int, h: int, w: int, target: int,
                     out_scale: float, grad: int, loss: int, stream: int):
    return check(lib().mdf_cnn_backward(ws, ws_bytes, params, int(batch), int(h), int(w), target, float(out_scale),
                                        grad, loss, stream))


def mdf_cnn_layer_io(ws: int, ws_bytes: int, batch: int, h: int, w: int, layer: int, in_bf16, z, g_bf16, g,
                     stream: int):
    return check(lib().mdf_cnn_layer_io(ws, ws_bytes, int(batch), int(h), int(w), int(layer), in_bf16, z, g_bf16, g,
                                        stream))


def mdf_cnn_adam(params: int, grad: int, m: int, v: int, n: int, lr: float, beta1: float, beta2: float, eps: float,
                 step: int, stream: int):
    return check(lib().mdf_cnn_adam(params, grad, m, v, int(n), float(lr), float(beta1), float(beta2), float(eps),
                                    int(step), stream))


def mdf_closure_apply(ctx: int, du: int, dv: int, ke_ref: float, div_factor: float):
    ke, div, fb = C.c_double(), C.c_double(), C.c_int32()
    check(lib().mdf_closure_apply(ctx, du, dv, float(ke_ref), float(div_factor), C.byref(ke), C.byref(div),
                                  C.byref(fb)), ctx)
    return ke.value, div.value, bool(fb.value)


def mdf_closure_begin(ctx: int):
    return check(lib().mdf_closure_begin(ctx), ctx)


def mdf_closure_apply_async(ctx: int, du: int, dv: int, div_factor: float):
    return check(lib().mdf_closure_apply_async(ctx, du, dv, float(div_factor)), ctx)


def mdf_closure_stats(ctx: int):
    """(ke_ref, fall-backs, windows) since mdf_closure_begin; synchronises."""
    out = (C.c_double * 3)()
    check(lib().mdf_closure_stats(ctx, out), ctx)
    return out[0], int(out[1]), int(out[2])


def mdf_stability(p: mdf_params, u0: float, v0: float, nk: int):
    """(rho[nk, nk], (max rho, theta_x, theta_y)) of the von Neumann screen."""
    import numpy as np
    rho = np.empty((int(nk), int(nk)), dtype=np.float64)
    worst = (C.c_double * 3)()
    check(lib().mdf_stability(C.byref(p), float(u0), float(v0), int(nk), rho.ctypes.data_as(_dp), worst))
    return rho, (worst[0], worst[1], worst[2])

"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loaded by tests/, the smoke check and the CPU baseline of the benchmark; the
product path never imports it.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
LIB_OMP_PATH = os.path.join(HERE, "liborc_omp.so")

_dp = C.POINTER(C.c_double)


class OrcParams(C.Structure):
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
        ("track_rho0", C.c_int32),
        ("flux_source", C.c_int32),
    ]


_libs = {}
_override = None


def lib(kind: str = "serial"):
    """The oracle library: "serial" (liborc.so) or "omp" (liborc_omp.so, the
    same sources with OpenMP over the node loops).  Inside using_library()
    every kind resolves to that library."""
    path = _override or (LIB_OMP_PATH if kind == "omp" else LIB_PATH)
    if path not in _libs:
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        _libs[path] = _declare(C.CDLL(path))
    return _libs[path]


@contextlib.contextmanager
def using_library(path: str):
    """Route every oracle call made inside the block (and by Oracle objects
    created inside it) to the library at `path` (a differently built copy of
    the oracle sources, e.g. one with a planted mistake)."""
    global _override
    old = _override
    _override = os.path.abspath(path)
    try:
        yield lib()
    finally:
        _override = old


def _declare(L):
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcParams), _dp, _dp, _dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int32]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_steps.restype = C.c_int64
        L.orc_steps.argtypes = [C.c_void_p]
        for name in ("orc_get_f", "orc_derived", "orc_diagnostics"):
            getattr(L, name).argtypes = [C.c_void_p, _dp]
        L.orc_set_f.argtypes = [C.c_void_p, _dp]
        L.orc_fields.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.orc_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_node_moments.argtypes = [C.c_double, _dp, _dp, _dp, _dp]
        L.orc_collision_matrices.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        L.cnn_param_count.restype = C.c_int32
        L.cnn_bf16.restype = C.c_double
        L.cnn_bf16.argtypes = [C.c_double]
        L.cnn_conv3x3.argtypes = [C.c_int32] * 5 + [_dp, _dp, _dp, _dp]
        L.cnn_forward.argtypes = [_dp, C.c_int32, C.c_int32, C.c_int32, _dp, _dp]
        L.cnn_loss_grad.restype = C.c_double
        L.cnn_loss_grad.argtypes = [_dp, C.c_int32, C.c_int32, C.c_int32, _dp, _dp, _dp]
        L.cnn_apply_correction.argtypes = [C.c_int32, C.c_int32, C.c_double, _dp, _dp, _dp]
        L.orc_collide_step1.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_mixed_derivative.argtypes = [C.c_void_p, _dp, C.c_int32, C.c_int32, _dp]
        L.orc_wall_update.argtypes = [C.c_void_p, _dp]
        L.orc_powerlaw_nu.restype = C.c_double
        L.orc_powerlaw_nu.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_set_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_rho0.restype = C.c_int32
        L.orc_rho0.argtypes = [C.c_void_p, _dp]
        L.orc_form_pressure.restype = C.c_double
        L.orc_form_pressure.argtypes = [C.c_void_p, _dp, C.c_int32, C.c_double]
        return L


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _params(prob):
    keep = []
    gx = None if prob.inv_dx_x is None else np.ascontiguousarray(prob.inv_dx_x, dtype=np.float64)
    gy = None if prob.inv_dx_y is None else np.ascontiguousarray(prob.inv_dx_y, dtype=np.float64)
    ffx = getattr(prob, "force_x", None)
    ffy = getattr(prob, "force_y", None)
    ffx = None if ffx is None else np.ascontiguousarray(ffx, dtype=np.float64)
    ffy = None if ffy is None else np.ascontiguousarray(ffy, dtype=np.float64)
    for a in (ffx, ffy):
        assert a is None or a.shape == (prob.ny, prob.nx)
    met = getattr(prob, "metric", None)
    met = None if met is None else np.ascontiguousarray(met, dtype=np.float64)
    assert met is None or met.shape == (4, prob.ny, prob.nx)
    rs = getattr(prob, "mass_source", None)
    rs = None if rs is None else np.ascontiguousarray(rs, dtype=np.float64)
    assert rs is None or rs.shape == (prob.ny, prob.nx)
    keep += [gx, gy, ffx, ffy, met, rs]
    p = OrcParams(prob.nx, prob.ny, prob.lx, prob.ly, prob.nu, prob.pl_n, prob.nu_min, prob.nu_max,
                  prob.cfl, prob.c, prob.eta, prob.s_ratio, prob.bc_x, prob.bc_y, prob.lid_u,
                  prob.fx, prob.fy, _ptr(gx), _ptr(gy), prob.dx_min, _ptr(ffx), _ptr(ffy),
                  prob.force_omega, prob.force_phase, int(prob.force_harmonic), _ptr(met),
                  _ptr(rs), int(getattr(prob, "track_rho0", 0)), int(getattr(prob, "flux_source", 0)))
    return p, keep


class Oracle:
    """One oracle run of a problems.Problem.  threads > 0 runs it on the OpenMP
    build with that many threads (results identical to the sequential build)."""

    def __init__(self, prob, threads: int = 0):
        self.prob = prob
        self._L = lib("omp" if threads > 0 else "serial")
        if threads > 0:
            self.threads = self._L.orc_set_threads(int(threads))
        else:
            self.threads = 1
        self._p, self._keep = _params(prob)
        u0 = np.ascontiguousarray(prob.u0, dtype=np.float64)
        v0 = np.ascontiguousarray(prob.v0, dtype=np.float64)
        p0 = np.ascontiguousarray(prob.p0, dtype=np.float64)
        self._h = self._L.orc_create(C.byref(self._p), _ptr(u0), _ptr(v0), _ptr(p0))
        if not self._h:
            raise ValueError("oracle rejected the problem parameters")
        self.nx, self.ny = prob.nx, prob.ny

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def dt(self) -> float:
        return self._L.orc_dt(self._h)

    @property
    def steps(self) -> int:
        return self._L.orc_steps(self._h)

    def step(self, n: int = 1):
        self._L.orc_step(self._h, int(n))
        return self

    def f(self) -> np.ndarray:
        out = np.empty((10, self.ny, self.nx))
        self._L.orc_get_f(self._h, _ptr(out))
        return out

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (10, self.ny, self.nx)
        self._L.orc_set_f(self._h, _ptr(f))

    def fields(self, which: int) -> np.ndarray:
        """Intermediate field of the last step: 0 f_hat^+, 1 f_bar^+, 2 f_bar(t+h), 3 f(t+h)."""
        out = np.empty((10, self.ny, self.nx))
        self._L.orc_fields(self._h, int(which), _ptr(out))
        return out

    def moments(self):
        u = np.empty((self.ny, self.nx))
        v = np.empty_like(u)
        p = np.empty_like(u)
        self._L.orc_moments(self._h, _ptr(u), _ptr(v), _ptr(p))
        return u, v, p

    def rho0(self) -> np.ndarray:
        """rho0 of the tracked alpha = 0 equation (needs prob.track_rho0)."""
        out = np.empty((self.ny, self.nx))
        if self._L.orc_rho0(self._h, _ptr(out)) != 0:
            raise ValueError("the alpha = 0 equation is not tracked in this run")
        return out

    def form_pressure(self, phi: np.ndarray, form: int, R: float) -> float:
        """Pressure of eq. 2.3.23 with source R for one node's stored form phi (10 values)."""
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        assert phi.shape == (10,)
        return self._L.orc_form_pressure(self._h, _ptr(phi), int(form), float(R))

    def derived(self) -> np.ndarray:
        out = np.empty((14, self.ny, self.nx))
        self._L.orc_derived(self._h, _ptr(out))
        return out

    def diagnostics(self) -> np.ndarray:
        out = np.empty(8)
        self._L.orc_diagnostics(self._h, _ptr(out))
        return out

    def mixed_derivative(self, plane: np.ndarray, axis: int, sign: int) -> np.ndarray:
        plane = np.ascontiguousarray(plane, dtype=np.float64)
        out = np.empty_like(plane)
        self._L.orc_mixed_derivative(self._h, _ptr(plane), axis, sign, _ptr(out))
        return out

    def wall_update(self, field: np.ndarray) -> np.ndarray:
        field = np.array(field, dtype=np.float64, order="C", copy=True)
        self._L.orc_wall_update(self._h, _ptr(field))
        return field

    def collide_step1(self, fhat_node: np.ndarray):
        fh = np.ascontiguousarray(fhat_node, dtype=np.float64)
        a = np.empty(10)
        b = np.empty(10)
        self._L.orc_collide_step1(self._h, _ptr(fh), _ptr(a), _ptr(b))
        return a, b

    def powerlaw_nu(self, gam_hat: float, theta: float) -> float:
        return self._L.orc_powerlaw_nu(self._h, gam_hat, theta)


def feq(c: float, u: float, v: float, P: float) -> np.ndarray:
    out = np.empty(10)
    lib().orc_feq(c, u, v, P, _ptr(out))
    return out


def node_moments(c: float, phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    u, v, P = C.c_double(), C.c_double(), C.c_double()
    lib().orc_node_moments(c, _ptr(phi), C.byref(u), C.byref(v), C.byref(P))
    return u.value, v.value, P.value


def collision_matrices(s: float, sp: float, dt: float):
    out = np.empty(125)
    lib().orc_collision_matrices(s, sp, dt, _ptr(out))
    m = out.reshape(5, 5, 5)
    return {"Lt": m[0], "ImL": m[1], "Ib": m[2], "Cinv": m[3], "Ainv": m[4]}


# ---- closure network (plain FP64 definitions; see cnn_oracle.c) ------------

CNN_CHANNELS = (2, 32, 32, 32, 2)


def cnn_param_count() -> int:
    return lib().cnn_param_count()


def cnn_bf16(v: float) -> float:
    return lib().cnn_bf16(float(v))


def cnn_bf16_array(a: np.ndarray) -> np.ndarray:
    f = np.vectorize(lib().cnn_bf16, otypes=[np.float64])
    return f(np.asarray(a, dtype=np.float64))


def cnn_conv3x3(a: np.ndarray, w: np.ndarray, bias: Optional[np.ndarray] = None) -> np.ndarray:
    """a: [B, H, W, cin]; w: [9, cin, cout]; periodic 3x3 convolution -> [B, H, W, cout]."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    B, H, W, cin = a.shape
    cout = w.shape[2]
    z = np.empty((B, H, W, cout))
    b = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    lib().cnn_conv3x3(B, H, W, cin, cout, _ptr(a), _ptr(w), None if b is None else _ptr(b), _ptr(z))
    return z


def cnn_forward(params: np.ndarray, x: np.ndarray) -> np.ndarray:
    """x: [B, H, W, 2] -> y: [B, H, W, 2]."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    B, H, W, _ = x.shape
    y = np.empty((B, H, W, 2))
    lib().cnn_forward(_ptr(params), B, H, W, _ptr(x), _ptr(y))
    return y


def cnn_loss_grad(params: np.ndarray, x: np.ndarray, target: np.ndarray):
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(target, dtype=np.float64)
    B, H, W, _ = x.shape
    g = np.empty(cnn_param_count())
    loss = lib().cnn_loss_grad(_ptr(params), B, H, W, _ptr(x), _ptr(t), _ptr(g))
    return loss, g


def cnn_apply_correction(f: np.ndarray, du: np.ndarray, dv: np.ndarray, c: float = 1.0) -> np.ndarray:
    """f: dense [10, ny, nx] state; returns f + f^eq(u + du, P) - f^eq(u, P)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    ny, nx = f.shape[1:]
    du = np.ascontiguousarray(du, dtype=np.float64)
    dv = np.ascontiguousarray(dv, dtype=np.float64)
    lib().cnn_apply_correction(nx, ny, float(c), _ptr(du), _ptr(dv), _ptr(f))
    return f


def cnn_layer_slices():
    """(weight slice, bias slice, cin, cout) of each layer in the flat parameter vector."""
    out, o = [], 0
    for l in range(4):
        cin, cout = CNN_CHANNELS[l], CNN_CHANNELS[l + 1]
        nw = 9 * cin * cout
        out.append((slice(o, o + nw), slice(o + nw, o + nw + cout), cin, cout))
        o += nw + cout
    return out

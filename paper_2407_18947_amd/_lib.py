"""Thin ctypes binding of librtcc3.so (declared in include/rtcc3.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory (complex128 tensors) and the
stream; no computation happens here.  If the library is missing the calls
raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "librtcc3.so")

RTCC3_OK, RTCC3_EINVAL, RTCC3_ENOMEM, RTCC3_EDEVICE, RTCC3_ESTATE, RTCC3_EDIVERGED = 0, -1, -2, -3, -4, -5
RTCC3_FP64, RTCC3_FP32, RTCC3_BF16X3, RTCC3_BF16X2 = 0, 1, 2, 3
RTCC3_OPT_TRIPLES, RTCC3_OPT_PRECISION, RTCC3_OPT_WINDOW_BLOCKS, RTCC3_OPT_SINGLE_STREAM = 1, 2, 3, 4
RTCC3_OPT_GRAPH, RTCC3_OPT_AUTOTUNE, RTCC3_OPT_TANGENT = 5, 6, 7

EXPORTS = [
    "rtcc3_create", "rtcc3_set_state", "rtcc3_get_state", "rtcc3_rhs", "rtcc3_rhs_terms", "rtcc3_propagate",
    "rtcc3_propagate_batch",
    "rtcc3_dipole", "rtcc3_set_option", "rtcc3_last_timing", "rtcc3_zgemm_selftest",
    "rtcc3_zgemm_selftest_noalloc", "rtcc3_tuning_summary", "rtcc3_tuning_report", "rtcc3_rhs_tangent",
    "rtcc3_propagate_tangent", "rtcc3_get_state_tangent", "rtcc3_last_error", "rtcc3_destroy",
]

_lib = None


class RTCC3Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtcc3 error {code}: {msg}")
        self.code = code


def load():
    """Load librtcc3.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIBPATH)
    P, I, D, VP = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    L.rtcc3_create.argtypes = [I, I, VP, I, VP, VP, I, VP, P(VP)]
    L.rtcc3_set_state.argtypes = [VP, VP, I]
    L.rtcc3_get_state.argtypes = [VP, VP, I]
    L.rtcc3_rhs.argtypes = [VP, VP, VP, VP]
    L.rtcc3_rhs_terms.argtypes = [VP, VP, VP, VP, I]
    L.rtcc3_propagate.argtypes = [VP, I, D, VP, VP]
    L.rtcc3_propagate_batch.argtypes = [VP, I, I, D, VP, VP]
    L.rtcc3_dipole.argtypes = [VP, VP, VP]
    L.rtcc3_set_option.argtypes = [VP, I, I]
    L.rtcc3_last_timing.argtypes = [VP, VP]
    L.rtcc3_tuning_summary.argtypes = [VP, VP]
    L.rtcc3_tuning_report.argtypes = [VP, VP, I]
    L.rtcc3_zgemm_selftest.argtypes = [I, I, I, I, VP, VP, VP]
    L.rtcc3_zgemm_selftest_noalloc.argtypes = [I, I, I, I, VP, VP, VP]
    L.rtcc3_rhs_tangent.argtypes = [VP, VP, VP, VP, VP, VP, VP, VP, VP]
    L.rtcc3_propagate_tangent.argtypes = [VP, I, D, VP, VP, D, VP, VP, VP]
    L.rtcc3_get_state_tangent.argtypes = [VP, VP, I]
    L.rtcc3_last_error.argtypes = [VP]
    L.rtcc3_last_error.restype = ctypes.c_char_p
    L.rtcc3_destroy.argtypes = [VP]
    L.rtcc3_destroy.restype = None
    for name in EXPORTS:
        if name not in ("rtcc3_last_error", "rtcc3_destroy"):
            getattr(L, name).restype = I
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())  # torch tensor


def _check(rc, ctx=None):
    if rc != RTCC3_OK:
        msg = load().rtcc3_last_error(ctx)
        raise RTCC3Error(rc, msg.decode() if msg else "")


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _c128(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


# ---------------------------------------------------------------- same names as the C ABI
def rtcc3_create(o, v, fock, B, dipole, precision=RTCC3_FP64, stream=None):
    L = load()
    fock, B, dipole = _f64(fock), _f64(B), _f64(dipole)
    naux = B.shape[0]
    out = ctypes.c_void_p()
    rc = L.rtcc3_create(o, v, _ptr(fock), naux, _ptr(B), _ptr(dipole), precision, stream, ctypes.byref(out))
    _check(rc, None)
    return out


def rtcc3_set_state(ctx, y):
    if isinstance(y, np.ndarray) or not hasattr(y, "data_ptr"):
        yh = _c128(y)
        _check(load().rtcc3_set_state(ctx, _ptr(yh), 0), ctx)
    else:
        _check(load().rtcc3_set_state(ctx, _ptr(y), 1), ctx)


def rtcc3_get_state(ctx, n):
    y = np.empty(n, dtype=np.complex128)
    _check(load().rtcc3_get_state(ctx, _ptr(y), 0), ctx)
    return y


def rtcc3_rhs(ctx, E, y_dev, dy_dev):
    E = _f64(E)
    _check(load().rtcc3_rhs(ctx, _ptr(E), _ptr(y_dev), _ptr(dy_dev)), ctx)


def rtcc3_rhs_terms(ctx, E, y_dev, terms_dev, with_triples=1):
    E = _f64(E)
    _check(load().rtcc3_rhs_terms(ctx, _ptr(E), _ptr(y_dev), _ptr(terms_dev), int(with_triples)), ctx)


def rtcc3_propagate(ctx, steps, dt, field, mu=None):
    """Returns the dipole series [(steps+1), 3]; `mu` (optional) receives it even
    when the call raises (EDIVERGED leaves the entries after the last finite
    state NaN)."""
    field = _f64(field)
    if field.shape != (2 * steps + 1, 3):
        raise ValueError("field must have shape (2*steps+1, 3)")
    if mu is None:
        mu = np.empty((steps + 1, 3), dtype=np.complex128)
    if mu.shape != (steps + 1, 3) or mu.dtype != np.complex128 or not mu.flags.c_contiguous:
        raise ValueError("mu must be a contiguous complex128 array of shape (steps+1, 3)")
    _check(load().rtcc3_propagate(ctx, int(steps), float(dt), _ptr(field), _ptr(mu)), ctx)
    return mu


def rtcc3_propagate_batch(ctxs, steps, dt, fields, mus=None):
    """Propagates the contexts together; returns their dipole series (list of
    [(steps+1), 3]); `mus` (optional list) receives them even when the call raises."""
    n = len(ctxs)
    fields = [_f64(f) for f in fields]
    if len(fields) != n or any(f.shape != (2 * steps + 1, 3) for f in fields):
        raise ValueError("one field of shape (2*steps+1, 3) per context")
    if mus is None:
        mus = [np.empty((steps + 1, 3), dtype=np.complex128) for _ in range(n)]
    carr = (ctypes.c_void_p * n)(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    farr = (ctypes.c_void_p * n)(*[f.ctypes.data for f in fields])
    marr = (ctypes.c_void_p * n)(*[m.ctypes.data for m in mus])
    _check(load().rtcc3_propagate_batch(carr, n, int(steps), float(dt), farr, marr), None)
    return mus


def rtcc3_dipole(ctx, E):
    E = _f64(E)
    out = np.empty(3, dtype=np.complex128)
    _check(load().rtcc3_dipole(ctx, _ptr(E), _ptr(out)), ctx)
    return out


def rtcc3_set_option(ctx, option, value):
    _check(load().rtcc3_set_option(ctx, int(option), int(value)), ctx)


def rtcc3_rhs_tangent(ctx, E, Edot, y_dev, ydot_dev, dy_dev, dydot_dev):
    """Fills dy_dev and dydot_dev; returns (mu[3], mudot[3])."""
    E, Edot = _f64(E), _f64(Edot)
    mu = np.empty(3, dtype=np.complex128)
    mudot = np.empty(3, dtype=np.complex128)
    _check(load().rtcc3_rhs_tangent(ctx, _ptr(E), _ptr(Edot), _ptr(y_dev), _ptr(ydot_dev), _ptr(dy_dev),
                                    _ptr(dydot_dev), _ptr(mu), _ptr(mudot)), ctx)
    return mu, mudot


def rtcc3_propagate_tangent(ctx, steps, dt, field, field_dot=None, kappa_dot=0.0, ydot0=None):
    """Returns (mu, mudot), each [(steps+1), 3]."""
    field = _f64(field)
    if field.shape != (2 * steps + 1, 3):
        raise ValueError(f"field must have shape {(2 * steps + 1, 3)}")
    fd = None if field_dot is None else _f64(field_dot)
    if fd is not None and fd.shape != field.shape:
        raise ValueError("field_dot must have the field's shape")
    yd = None if ydot0 is None else _c128(ydot0)
    mu = np.empty((steps + 1, 3), dtype=np.complex128)
    mudot = np.empty((steps + 1, 3), dtype=np.complex128)
    _check(load().rtcc3_propagate_tangent(ctx, int(steps), float(dt), _ptr(field), _ptr(fd), float(kappa_dot),
                                          _ptr(yd), _ptr(mu), _ptr(mudot)), ctx)
    return mu, mudot


def rtcc3_get_state_tangent(ctx, n):
    y = np.empty(n, dtype=np.complex128)
    _check(load().rtcc3_get_state_tangent(ctx, _ptr(y), 0), ctx)
    return y


def rtcc3_last_timing(ctx):
    out = np.zeros(6)
    _check(load().rtcc3_last_timing(ctx, _ptr(out)), ctx)
    return out


def rtcc3_tuning_summary(ctx):
    out = np.zeros(2, dtype=np.int32)
    _check(load().rtcc3_tuning_summary(ctx, _ptr(out)), ctx)
    return int(out[0]), int(out[1])


def rtcc3_tuning_report(ctx, max_records=4096):
    """Rows (M, N, K, batch, heuristic split, chosen split, heuristic ms, chosen ms)."""
    out = np.zeros((max_records, 8))
    n = load().rtcc3_tuning_report(ctx, _ptr(out), max_records)
    if n < 0:
        _check(n, ctx)
    return out[: min(n, max_records)]


def rtcc3_zgemm_selftest(A, B, precision=RTCC3_FP64):
    A, B = _c128(A), _c128(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.empty((M, N), dtype=np.complex128)
    _check(load().rtcc3_zgemm_selftest(M, N, K, precision, _ptr(A), _ptr(B), _ptr(C)), None)
    return C


def rtcc3_zgemm_selftest_noalloc(A, B, precision=RTCC3_FP64):
    A, B = _c128(A), _c128(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.empty((M, N), dtype=np.complex128)
    _check(load().rtcc3_zgemm_selftest_noalloc(M, N, K, precision, _ptr(A), _ptr(B), _ptr(C)), None)
    return C


def rtcc3_last_error(ctx=None):
    m = load().rtcc3_last_error(ctx)
    return m.decode() if m else ""


def rtcc3_destroy(ctx):
    if ctx:
        load().rtcc3_destroy(ctx)


class Context:
    """Owning wrapper of an rtcc3 context for one system."""

    def __init__(self, system, precision=RTCC3_FP64, stream=None):
        self.o, self.v = system.o, system.v
        self.n = self.o + self.v
        self.ylen = 2 * (self.o * self.v + self.o ** 2 * self.v ** 2)
        self.ctx = rtcc3_create(self.o, self.v, system.fock, system.B, system.mu, precision, stream)

    def close(self):
        if self.ctx:
            rtcc3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, y):
        rtcc3_set_state(self.ctx, y)

    def get_state(self):
        return rtcc3_get_state(self.ctx, self.ylen)

    def set_option(self, option, value):
        rtcc3_set_option(self.ctx, option, value)

    def propagate(self, steps, dt, field):
        self.last_dipoles = np.empty((steps + 1, 3), dtype=np.complex128)
        return rtcc3_propagate(self.ctx, steps, dt, field, self.last_dipoles)

    def dipole(self, E):
        return rtcc3_dipole(self.ctx, E)

    def propagate_tangent(self, steps, dt, field, field_dot=None, kappa_dot=0.0, ydot0=None):
        return rtcc3_propagate_tangent(self.ctx, steps, dt, field, field_dot, kappa_dot, ydot0)

    def get_state_tangent(self):
        return rtcc3_get_state_tangent(self.ctx, self.ylen)

    def terms_size(self):
        o, v, n = self.o, self.v, self.n
        return 4 * (o * v + o * o * v * v) + n * n + 3

    def split_terms(self, t):
        o, v, n = self.o, self.v, self.n
        ov, oovv = o * v, o * o * v * v
        out, p = {}, 0
        for name, sh in [("R1", (o, v)), ("R2", (o, o, v, v)), ("G1", (o, v)), ("G2", (o, o, v, v)),
                         ("X1", (o, v)), ("X2", (o, o, v, v)), ("Y1", (o, v)), ("Y2", (o, o, v, v)),
                         ("D", (n, n)), ("mu", (3,))]:
            k = int(np.prod(sh))
            out[name] = t[p:p + k].reshape(sh)
            p += k
        return out

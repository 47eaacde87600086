"""Python access to the plain FP64 CPU oracle (``liboracle.so``, built from
``oracle.c`` by :func:`build`).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FREE, FREE_CONTINUOUS, PERIODIC, PERIODIC_CONTINUOUS = 0, 1, 2, 3
_ERRORS = {-1: "EINVAL", -2: "EBOX", -3: "ENEUTRAL", -4: "ENONFINITE", -5: "ENOMEM"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({_ERRORS.get(code, '?')})")
        self.code = code


def build(verbose=False):
    """Compile liboracle.so with gcc (plain -O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    global _lib
    _lib = None


class _Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("order", ctypes.c_int), ("boundary", ctypes.c_int),
                ("origin", ctypes.c_double * 3), ("box", ctypes.c_double),
                ("split_d", ctypes.c_double), ("node_shrink", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_nodes.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.orc_lagrange.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, _D]
        L.orc_shift_1d.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_replace.argtypes = [ctypes.c_int, ctypes.c_double, _D, ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_shift_3d.argtypes = [ctypes.c_int, _D, _D, _D, _D, _D]
        L.orc_bilinear.argtypes = [ctypes.c_int, ctypes.c_double, _D, ctypes.c_double, _D,
                                   ctypes.c_double, _D, _D]
        L.orc_bilinear.restype = ctypes.c_double
        L.orc_bilinear_matrix.argtypes = [ctypes.c_int, ctypes.c_double, _D, ctypes.c_double, _D,
                                          ctypes.c_double, _D]
        L.orc_direct.argtypes = [ctypes.c_int, _D, _D, ctypes.c_int, _I, _D, _D]
        L.orc_ewald.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _D, _D]
        L.orc_split_count.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _D, _I, _I]
        L.orc_fmm.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_fmm_pairwise.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _D, _D, _D, _D]
        L.orc_periodic_root.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.orc_periodic_root_alpha.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def params(levels, order, boundary=FREE, origin=(0.0, 0.0, 0.0), box=1.0, split_d=0.0,
           node_shrink=1.0):
    p = _Params()
    p.levels, p.order, p.boundary = levels, order, boundary
    p.origin = (ctypes.c_double * 3)(*origin)
    p.box, p.split_d, p.node_shrink = box, split_d, node_shrink
    return p


def nodes(n, sigma=1.0):
    t = np.zeros(n)
    lib().orc_nodes(n, sigma, _dp(t))
    return t


def lagrange(a, x):
    a = _f64(a)
    n = a.size
    g, dg = np.zeros(n), np.zeros(n)
    lib().orc_lagrange(n, _dp(a), float(x), _dp(g), _dp(dg))
    return g, dg


def shift_1d(a, at):
    a, at = _f64(a), _f64(at)
    n = a.size
    G = np.zeros((n, n))
    lib().orc_shift_1d(n, _dp(a), _dp(at), _dp(G))
    return G


def replace(n, lo, side, pos, q, sigma=1.0):
    pos, q, lo = _f64(pos).reshape(-1, 3), _f64(q).ravel(), _f64(lo)
    phi = np.zeros(n ** 3)
    lib().orc_replace(n, sigma, _dp(lo), float(side), q.size, _dp(pos), _dp(q), _dp(phi))
    return phi


def shift_3d(n, Gx, Gy, Gz, v):
    Gx, Gy, Gz, v = _f64(Gx), _f64(Gy), _f64(Gz), _f64(v)
    out = np.zeros(n ** 3)
    lib().orc_shift_3d(n, _dp(Gx), _dp(Gy), _dp(Gz), _dp(v), _dp(out))
    return out


def bilinear(n, lo1, s1, lo2, s2, v, w, sigma=1.0):
    return lib().orc_bilinear(n, sigma, _dp(_f64(lo1)), float(s1), _dp(_f64(lo2)), float(s2),
                              _dp(_f64(v)), _dp(_f64(w)))


def bilinear_matrix(n, lo1, s1, lo2, s2, sigma=1.0):
    K = np.zeros((n ** 3, n ** 3))
    lib().orc_bilinear_matrix(n, sigma, _dp(_f64(lo1)), float(s1), _dp(_f64(lo2)), float(s2), _dp(K))
    return K


def direct(pos, q, targets=None):
    pos, q = _f64(pos), _f64(q)
    N = q.size
    if targets is None:
        nt, tp = N, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int32)
        nt, tp = targets.size, targets.ctypes.data_as(_I)
    phi, field = np.zeros(nt), np.zeros((nt, 3))
    _check(lib().orc_direct(N, _dp(pos), _dp(q), nt, tp, _dp(phi), _dp(field)))
    return phi, field


def ewald(pos, q, box=1.0, origin=(0.0, 0.0, 0.0), alpha=None, nreal=1, nrecip=None, targets=None):
    """Tin-foil Ewald potential and field.  Defaults give ~1e-15 relative
    truncation error: alpha = 5/box, real images |m| <= 1 around the minimum
    image, reciprocal |k| <= 12 (units of 2 pi / box)."""
    pos, q = _f64(pos), _f64(q)
    N = q.size
    alpha = 5.0 / box if alpha is None else alpha
    nrecip = 12 if nrecip is None else nrecip
    if targets is None:
        nt, tp = N, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int32)
        nt, tp = targets.size, targets.ctypes.data_as(_I)
    phi, field = np.zeros(nt), np.zeros((nt, 3))
    _check(lib().orc_ewald(N, _dp(pos), _dp(q), _dp(_f64(origin)), box, alpha, nreal, nrecip, nt, tp,
                           _dp(phi), _dp(field)))
    return phi, field


def split_count(pos, levels, order, boundary, box=1.0, origin=(0.0, 0.0, 0.0), split_d=0.0):
    p = params(levels, order, boundary, origin, box, split_d)
    pos = _f64(pos)
    ns, nf = ctypes.c_int(), ctypes.c_int()
    _check(lib().orc_split_count(ctypes.byref(p), pos.shape[0], _dp(pos), ctypes.byref(ns), ctypes.byref(nf)))
    return ns.value, nf.value


def fmm(pos, q, levels, order, boundary=FREE, box=1.0, origin=(0.0, 0.0, 0.0), split_d=0.0,
        node_shrink=1.0, dump_levels=False):
    """The replacement FMM (Sec. 2.2 + Sec. 2.3 + Sec. 4.2) in FP64.
    Returns dict(phi, field, field_paper, energy[, phi_levels, L_levels])."""
    p = params(levels, order, boundary, origin, box, split_d, node_shrink)
    pos, q = _f64(pos), _f64(q)
    N = q.size
    phi, field, fpap = np.zeros(N), np.zeros((N, 3)), np.zeros((N, 3))
    E = ctypes.c_double()
    PL = LL = None
    if dump_levels:
        total = sum(8 ** l for l in range(levels + 1))
        PL, LL = np.zeros(total * order ** 3), np.zeros(total * order ** 3)
    _check(lib().orc_fmm(ctypes.byref(p), N, _dp(pos), _dp(q), _dp(phi), _dp(field), _dp(fpap),
                         ctypes.byref(E), _dp(PL), _dp(LL)))
    out = dict(phi=phi, field=field, field_paper=fpap, energy=E.value)
    if dump_levels:
        n3 = order ** 3
        offs = np.cumsum([0] + [8 ** l for l in range(levels + 1)])
        out["phi_levels"] = [PL[offs[l] * n3: offs[l + 1] * n3].reshape(-1, n3) for l in range(levels + 1)]
        out["L_levels"] = [LL[offs[l] * n3: offs[l + 1] * n3].reshape(-1, n3) for l in range(levels + 1)]
    return out


def fmm_pairwise(pos, q, levels, order, boundary=FREE, box=1.0, origin=(0.0, 0.0, 0.0), split_d=0.0,
                 node_shrink=1.0):
    p = params(levels, order, boundary, origin, box, split_d, node_shrink)
    pos, q = _f64(pos), _f64(q)
    N = q.size
    phi = np.zeros(N)
    E = ctypes.c_double()
    _check(lib().orc_fmm_pairwise(ctypes.byref(p), N, _dp(pos), _dp(q), _dp(phi), ctypes.byref(E)))
    return dict(phi=phi, energy=E.value)


def periodic_root(n, sigma=1.0, alpha=None):
    T = np.zeros((n ** 3, n ** 3))
    if alpha is None:
        lib().orc_periodic_root(n, sigma, _dp(T))
    else:
        lib().orc_periodic_root_alpha(n, sigma, alpha, _dp(T))
    return T

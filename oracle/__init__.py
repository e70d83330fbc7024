"""Python access to the CPU oracle (direct QBX, brute-force expansions) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import
this package. It wraps ``oracle.c`` through ctypes and works on host numpy arrays only.

Kinds: 1 = single layer S, 2 = double layer D, 3 = S(dens1) - D(dens2) (Green's formula).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

S, D, S_MINUS_D = 1, 2, 3

_lib = None


def load(path: str):
    """Load an oracle shared library and declare its signatures."""
    L = C.CDLL(path)
    dp, i64, i32 = C.POINTER(C.c_double), C.c_int64, C.c_int
    L.oracle_qbx_coeffs.argtypes = [i32, i64, dp, dp, dp, dp, dp, i64, dp, i32, dp]
    L.oracle_qbx_eval.argtypes = [i32, i64, dp, dp, dp, dp, dp, i64, dp, i32, i64, dp,
                                  C.POINTER(C.c_int32), dp]
    L.oracle_point_potential.argtypes = [i32, i64, dp, dp, dp, dp, dp, i64, dp, dp]
    L.oracle_qbx_normal_derivative.argtypes = [i64, dp, dp, dp, dp, i64, dp, i32, i64, dp, dp,
                                               C.POINTER(C.c_int32), dp]
    L.oracle_multipole.argtypes = [i32, i64, dp, dp, dp, dp, dp, C.c_double, C.c_double, i32,
                                   dp]
    L.oracle_local.argtypes = L.oracle_multipole.argtypes
    L.oracle_eval_multipole.argtypes = [i32, dp, C.c_double, C.c_double, i64, dp, dp]
    L.oracle_eval_local.argtypes = L.oracle_eval_multipole.argtypes
    L.oracle_num_threads.argtypes = []
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = load(_build.LIB)
    return _lib


def _d(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _sources(geom_or_src, dens1, dens2):
    g = geom_or_src
    src = (_f64(g.src_xy), _f64(g.src_nrm), _f64(g.src_w))
    return src, _f64(dens1), _f64(dens2)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def qbx_eval(geom, kind, dens1, dens2=None, p_qbx=8, tgt_xy=None, tgt_ctr=None):
    """Direct QBX at the geometry's targets (or given targets/association)."""
    (sxy, snrm, sw), d1, d2 = _sources(geom, dens1, dens2)
    cxy = _f64(geom.ctr_xy)
    txy = _f64(geom.tgt_xy if tgt_xy is None else tgt_xy)
    tc = np.ascontiguousarray(geom.tgt_ctr if tgt_ctr is None else tgt_ctr, dtype=np.int32)
    out = np.empty(txy.shape[0])
    rc = lib().oracle_qbx_eval(kind, sxy.shape[0], _d(sxy), _d(snrm), _d(sw), _d(d1), _d(d2),
                               cxy.shape[0], _d(cxy), p_qbx, txy.shape[0], _d(txy),
                               tc.ctypes.data_as(C.POINTER(C.c_int32)), _d(out))
    if rc != 0:
        raise RuntimeError(f"oracle_qbx_eval failed ({rc})")
    return out


def qbx_coeffs(geom, kind, dens1, dens2=None, p_qbx=8, ctr_xy=None):
    """Unscaled QBX coefficients alpha_m, shape (n_ctr, p+1) complex."""
    (sxy, snrm, sw), d1, d2 = _sources(geom, dens1, dens2)
    cxy = _f64(geom.ctr_xy if ctr_xy is None else ctr_xy).reshape(-1, 2)
    out = np.empty((cxy.shape[0], p_qbx + 1, 2))
    rc = lib().oracle_qbx_coeffs(kind, sxy.shape[0], _d(sxy), _d(snrm), _d(sw), _d(d1), _d(d2),
                                 cxy.shape[0], _d(cxy), p_qbx, _d(out))
    if rc != 0:
        raise RuntimeError(f"oracle_qbx_coeffs failed ({rc})")
    return out[..., 0] + 1j * out[..., 1]


def qbx_normal_derivative(geom, dens, p_qbx=8, tgt_xy=None, tgt_nrm=None, tgt_ctr=None):
    """S' dens (the single layer potential's normal derivative along the target normals) by
    direct QBX at the geometry's targets (or the given ones); on-surface targets with two
    centers average the one-sided limits."""
    (sxy, snrm, sw), d1, _ = _sources(geom, dens, None)
    cxy = _f64(geom.ctr_xy)
    txy = _f64(geom.tgt_xy if tgt_xy is None else tgt_xy).reshape(-1, 2)
    tn = _f64(geom.tgt_nrm if tgt_nrm is None else tgt_nrm).reshape(-1, 2)
    tc = np.ascontiguousarray(geom.tgt_ctr if tgt_ctr is None else tgt_ctr, dtype=np.int32)
    out = np.empty(txy.shape[0])
    rc = lib().oracle_qbx_normal_derivative(sxy.shape[0], _d(sxy), _d(snrm), _d(sw), _d(d1),
                                            cxy.shape[0], _d(cxy), p_qbx, txy.shape[0], _d(txy),
                                            _d(tn), tc.ctypes.data_as(C.POINTER(C.c_int32)),
                                            _d(out))
    if rc != 0:
        raise RuntimeError(f"oracle_qbx_normal_derivative failed ({rc})")
    return out


def point_potential(geom, kind, dens1, dens2=None, tgt_xy=None):
    (sxy, snrm, sw), d1, d2 = _sources(geom, dens1, dens2)
    txy = _f64(geom.tgt_xy if tgt_xy is None else tgt_xy).reshape(-1, 2)
    out = np.empty(txy.shape[0])
    rc = lib().oracle_point_potential(kind, sxy.shape[0], _d(sxy), _d(snrm), _d(sw), _d(d1),
                                      _d(d2), txy.shape[0], _d(txy), _d(out))
    if rc != 0:
        raise RuntimeError(f"oracle_point_potential failed ({rc})")
    return out


def multipole(geom, kind, dens1, dens2, center, p):
    (sxy, snrm, sw), d1, d2 = _sources(geom, dens1, dens2)
    out = np.empty((p + 1, 2))
    rc = lib().oracle_multipole(kind, sxy.shape[0], _d(sxy), _d(snrm), _d(sw), _d(d1), _d(d2),
                                float(center[0]), float(center[1]), p, _d(out))
    if rc != 0:
        raise RuntimeError("oracle_multipole failed")
    return out[:, 0] + 1j * out[:, 1]


def local(geom, kind, dens1, dens2, center, p):
    (sxy, snrm, sw), d1, d2 = _sources(geom, dens1, dens2)
    out = np.empty((p + 1, 2))
    rc = lib().oracle_local(kind, sxy.shape[0], _d(sxy), _d(snrm), _d(sw), _d(d1), _d(d2),
                            float(center[0]), float(center[1]), p, _d(out))
    if rc != 0:
        raise RuntimeError("oracle_local failed")
    return out[:, 0] + 1j * out[:, 1]


def _coef_arr(coef):
    c = np.asarray(coef, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1))


def eval_multipole(coef, center, xy):
    a = _coef_arr(coef)
    xy = _f64(xy).reshape(-1, 2)
    out = np.empty(xy.shape[0])
    lib().oracle_eval_multipole(a.shape[0] - 1, _d(a), float(center[0]), float(center[1]),
                                xy.shape[0], _d(xy), _d(out))
    return out


def eval_local(coef, center, xy):
    b = _coef_arr(coef)
    xy = _f64(xy).reshape(-1, 2)
    out = np.empty(xy.shape[0])
    lib().oracle_eval_local(b.shape[0] - 1, _d(b), float(center[0]), float(center[1]),
                            xy.shape[0], _d(xy), _d(out))
    return out

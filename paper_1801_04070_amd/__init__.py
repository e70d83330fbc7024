"""MI355X-native GIGAQBX: QBX-coupled FMM for 2-D Laplace layer potentials (HIP, gfx950).

The compute path is the C-ABI library ``libgigaqbx.so`` (``include/gigaqbx.h``); this module only
marshals arguments to it. PyTorch supplies device memory and the HIP stream. There is no CPU
fallback: importing :class:`QBXFMM` on a device context without the built library raises.

Functions with the ABI's names (``gq_create`` ... ``gq_last_error``) are re-exported from the
loaded library; :class:`QBXFMM` wraps a context for torch tensors.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (GQ_S, GQ_D, GQ_S_MINUS_D, GQ_S_AND_D, GQ_SP, GQ_MEM_HOST, GQ_MEM_DEVICE, GQ_FP64,
                   GQ_MIXED_FP32, gq_params, gq_stats)

__all__ = ["QBXFMM", "GQError", "library", "associate_targets", "GQ_S", "GQ_D", "GQ_S_MINUS_D", "GQ_S_AND_D", "GQ_SP",
           "default_params"]

_L = None


def library():
    """The loaded C library (raises ImportError if it is not built)."""
    global _L
    if _L is None:
        # torch first: the library then binds to the HIP runtime torch already loaded, so device
        # pointers, streams and the device list are shared by one runtime in the process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        _L = _lib.load()
    return _L


def __getattr__(name):
    if name in _lib.EXPORTED or name in _lib.EXPORTED_MLP:
        return getattr(library(), name)
    raise AttributeError(name)


def associate_targets(ctr_xy, ctr_r, tgt_xy, slack: float = 0.2, far_factor: float = 3.0):
    """gq_associate_targets on host arrays: returns (tgt_ctr (n_tgt, 2) int32, n_gap)."""
    L = library()
    c = np.ascontiguousarray(ctr_xy, dtype=np.float64).reshape(-1, 2)
    r = np.ascontiguousarray(ctr_r, dtype=np.float64)
    t = np.ascontiguousarray(tgt_xy, dtype=np.float64).reshape(-1, 2)
    out = np.empty((t.shape[0], 2), dtype=np.int32)
    gap = C.c_int64()
    st = L.gq_associate_targets(len(r), c.ctypes.data, r.ctypes.data, t.shape[0], t.ctypes.data,
                                float(slack), float(far_factor), out.ctypes.data, C.byref(gap))
    if st != 0:
        raise GQError(st, L.gq_associate_last_error().decode())
    return out, gap.value


class GQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def default_params(**kw) -> gq_params:
    p = gq_params()
    library().gq_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _ptr(a):
    """Device or host address of a torch tensor or numpy array."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class QBXFMM:
    """One library context. ``device=-1`` gives a host-only context (tree and lists only)."""

    def __init__(self, device: int = 0, stream=None):
        self._L = library()
        self.device = device
        h = C.c_void_p()
        if device >= 0:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            sp = C.c_void_p(stream.cuda_stream)
        else:
            sp = None
        st = self._L.gq_create(C.byref(h), device, sp)
        if st != 0:
            raise GQError(st, self._L.gq_last_error(None).decode())
        self._h = h
        self.n_src = self.n_ctr = self.n_tgt = 0

    def _check(self, st):
        if st != 0:
            raise GQError(st, self._L.gq_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.gq_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._check(self._L.gq_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def set_geometry(self, src_xy, src_nrm, src_w, ctr_xy, ctr_r, tgt_xy, tgt_ctr):
        """Arrays are host numpy (float64 / int32) or device torch tensors (all of one kind)."""
        arrs = [src_xy, src_nrm, src_w, ctr_xy, ctr_r, tgt_xy, tgt_ctr]
        if all(isinstance(a, np.ndarray) for a in arrs):
            mem = GQ_MEM_HOST
            arrs = [np.ascontiguousarray(a, dtype=np.int32 if i == 6 else np.float64)
                    for i, a in enumerate(arrs)]
        else:
            mem = GQ_MEM_DEVICE
            arrs = [a.contiguous() for a in arrs]
        self._keep = arrs
        src_xy, src_nrm, src_w, ctr_xy, ctr_r, tgt_xy, tgt_ctr = arrs
        self.n_src, self.n_ctr, self.n_tgt = len(src_w), len(ctr_r), tgt_xy.shape[0]
        self._check(self._L.gq_set_geometry(
            self._h, mem, self.n_src, _ptr(src_xy), _ptr(src_nrm), _ptr(src_w), self.n_ctr,
            _ptr(ctr_xy), _ptr(ctr_r), self.n_tgt, _ptr(tgt_xy), _ptr(tgt_ctr)))
        self._keep = None

    def set_geometry_batch(self, geoms):
        """Several independent geometries (objects with the fields of ``gq_inputs.Geometry``,
        host arrays, tgt_ctr local to each geometry) in one context; outputs and densities are
        concatenated in the same order."""
        cat = lambda name, dt: np.ascontiguousarray(
            np.concatenate([getattr(g, name) for g in geoms]), dtype=dt)
        off = lambda n: np.concatenate([[0], np.cumsum([n(g) for g in geoms])]).astype(np.int64)
        so = off(lambda g: len(g.src_w))
        co = off(lambda g: len(g.ctr_r))
        to = off(lambda g: g.tgt_xy.shape[0])
        arrs = [cat("src_xy", np.float64), cat("src_nrm", np.float64), cat("src_w", np.float64),
                cat("ctr_xy", np.float64).reshape(-1, 2), cat("ctr_r", np.float64),
                cat("tgt_xy", np.float64).reshape(-1, 2), cat("tgt_ctr", np.int32).reshape(-1, 2)]
        self.n_src, self.n_ctr, self.n_tgt = int(so[-1]), int(co[-1]), int(to[-1])
        self.geom_offsets = {"src": so, "ctr": co, "tgt": to}
        self._check(self._L.gq_set_geometry_batch(
            self._h, GQ_MEM_HOST, len(geoms), so.ctypes.data, co.ctypes.data, to.ctypes.data,
            self.n_src, *[_ptr(a) for a in arrs[:3]], self.n_ctr, _ptr(arrs[3]), _ptr(arrs[4]),
            self.n_tgt, _ptr(arrs[5]), _ptr(arrs[6])))

    def set_geometry_from(self, geom):
        """Geometry object with the fields of ``gq_inputs.Geometry`` (host arrays)."""
        self.set_geometry(geom.src_xy, geom.src_nrm, geom.src_w, geom.ctr_xy, geom.ctr_r,
                          geom.tgt_xy, geom.tgt_ctr)

    def build(self, params: gq_params | None = None, **kw) -> dict:
        p = params if params is not None else default_params(**kw)
        self._check(self._L.gq_build(self._h, C.byref(p)))
        got = gq_params()
        self._check(self._L.gq_get_params(self._h, C.byref(got)))
        self.params = got
        return self.stats()

    def stats(self) -> dict:
        s = gq_stats()
        self._check(self._L.gq_get_stats(self._h, C.byref(s)))
        d = {name: getattr(s, name) for name, _ in gq_stats._fields_}
        d["root_lo"] = tuple(s.root_lo)
        d["model_ops"] = dict(zip(_lib.GQ_OP_NAMES, list(s.model_ops)))
        return d

    _TREE_TYPES = {
        _lib.GQ_TREE_BOX_LEVEL: (np.int32, 1), _lib.GQ_TREE_BOX_PARENT: (np.int32, 1),
        _lib.GQ_TREE_BOX_CHILD: (np.int32, 4), _lib.GQ_TREE_BOX_IJ: (np.int64, 2),
        _lib.GQ_TREE_BOX_SRC_RANGE: (np.int64, 2), _lib.GQ_TREE_BOX_CTR_RANGE: (np.int64, 2),
        _lib.GQ_TREE_SRC_ORDER: (np.int64, 1), _lib.GQ_TREE_CTR_ORDER: (np.int64, 1),
    }

    def tree_array(self, what: int) -> np.ndarray:
        n = C.c_int64()
        self._check(self._L.gq_get_tree_array(self._h, what, None, C.byref(n)))
        if what in self._TREE_TYPES:
            dt, w = self._TREE_TYPES[what]
        else:
            dt, w = (np.int64, 1) if what % 2 == 1 else (np.int32, 1)
        out = np.empty(n.value, dtype=dt)
        self._check(self._L.gq_get_tree_array(self._h, what, out.ctypes.data, C.byref(n)))
        return out.reshape(-1, w) if w > 1 else out

    def lists(self) -> dict:
        """All interaction lists as {name: (starts, entries)}."""
        names = {"list1": _lib.GQ_LIST1_START, "list2": _lib.GQ_LIST2_START,
                 "list3c": _lib.GQ_LIST3C_START, "list3f": _lib.GQ_LIST3F_START,
                 "list4c": _lib.GQ_LIST4C_START, "list4f": _lib.GQ_LIST4F_START}
        return {k: (self.tree_array(v), self.tree_array(v + 1)) for k, v in names.items()}

    def autotune(self, kind: int, dens, reps: int = 5) -> tuple:
        """Tune the work-item shapes on this context (gq_autotune); returns (params, ms)."""
        d = dens.reshape(-1, dens.shape[-1])[0].contiguous()
        ms = C.c_double()
        self._check(self._L.gq_autotune(self._h, kind, _ptr(d), d.shape[0], reps, C.byref(ms)))
        p = gq_params()
        self._check(self._L.gq_get_params(self._h, C.byref(p)))
        self.params = p
        return p, ms.value

    def set_qbx_orders(self, orders):
        """Per-center QBX orders (caller order), or None for the uniform build order."""
        if orders is None:
            self._check(self._L.gq_set_qbx_orders(self._h, GQ_MEM_HOST, None))
            return
        if isinstance(orders, np.ndarray):
            o = np.ascontiguousarray(orders, dtype=np.int32)
            self._check(self._L.gq_set_qbx_orders(self._h, GQ_MEM_HOST, o.ctypes.data))
        else:
            import torch
            o = orders.to(torch.int32).contiguous()
            self._check(self._L.gq_set_qbx_orders(self._h, GQ_MEM_DEVICE, o.data_ptr()))

    def set_target_normals(self, tgt_nrm):
        """Unit normals of the targets for GQ_SP: host numpy (n_tgt, 2) or a device tensor."""
        if isinstance(tgt_nrm, np.ndarray):
            a = np.ascontiguousarray(tgt_nrm, dtype=np.float64).reshape(-1, 2)
            self._nrm_keep = a
            self._check(self._L.gq_set_target_normals(self._h, GQ_MEM_HOST, a.shape[0],
                                                      a.ctypes.data))
        else:
            a = tgt_nrm.contiguous()
            self._nrm_keep = a
            self._check(self._L.gq_set_target_normals(self._h, GQ_MEM_DEVICE, a.shape[0],
                                                      a.data_ptr()))

    def expansions(self, what: int, slot: int = 0) -> np.ndarray:
        """Box expansions of the last evaluation (gq_get_expansions): (n_boxes, p_fmm + 1)
        complex, scaled by the box side (a_k / s^k, b_k s^k)."""
        n = C.c_int64()
        self._check(self._L.gq_get_expansions(self._h, what, slot, None, C.byref(n)))
        out = np.empty(2 * n.value, dtype=np.float64)
        self._check(self._L.gq_get_expansions(self._h, what, slot, out.ctypes.data, C.byref(n)))
        c = out[0::2] + 1j * out[1::2]
        return c.reshape(-1, self.params.p_fmm + 1)

    def center_orders(self) -> np.ndarray:
        """The compiled QBX order each center runs at (caller order)."""
        out = np.empty(self.n_ctr, dtype=np.int32)
        self._check(self._L.gq_get_center_orders(self._h, out.ctypes.data))
        return out

    def box_orders(self) -> np.ndarray:
        n = C.c_int64()
        self._check(self._L.gq_get_box_orders(self._h, None, C.byref(n)))
        out = np.empty(n.value, dtype=np.int32)
        self._check(self._L.gq_get_box_orders(self._h, out.ctypes.data, C.byref(n)))
        return out

    def set_profiling(self, enable: bool = True):
        self._check(self._L.gq_set_profiling(self._h, int(enable)))

    def stage_times(self) -> dict:
        """{(kind, stage_name): (total_ms, launches)} since the last call (synchronises)."""
        n = 3 * _lib.GQ_N_STAGES
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._check(self._L.gq_get_stage_times(self._h, ms, cnt))
        out = {}
        for k in range(3):
            for s, name in enumerate(_lib.GQ_STAGE_NAMES):
                i = k * _lib.GQ_N_STAGES + s
                if cnt[i]:
                    out[(k + 1, name)] = (ms[i], cnt[i])
        return out

    def graph(self, kind: int, dens1, dens2=None, out=None):
        """Capture ``eval(kind, dens1, dens2, out)`` into a HIP graph (see gq_graph_create);
        returns (EvalGraph, out). The tensors must stay alive while the graph is used."""
        import torch
        d1 = dens1.reshape(-1, dens1.shape[-1]) if dens1.dim() == 1 else dens1
        d2 = None if dens2 is None else (dens2.reshape(-1, dens2.shape[-1]) if dens2.dim() == 1
                                         else dens2)
        if d1.stride(-1) != 1 or (d2 is not None and d2.stride(-1) != 1):
            raise ValueError("densities must have unit stride along a row")
        if out is None:
            rows = d1.shape[0] * (2 if kind == GQ_S_AND_D else 1)
            out = torch.empty((rows, self.n_tgt), dtype=torch.float64, device=d1.device)
        h = C.c_void_p()
        self._check(self._L.gq_graph_create(self._h, kind, d1.shape[0], _ptr(d1), d1.stride(0),
                                            _ptr(d2), 0 if d2 is None else d2.stride(0),
                                            _ptr(out), out.stride(0), C.byref(h)))
        return EvalGraph(self, h, (d1, d2, out)), out

    def device_math(self, fn: int, x):
        """The library's device log (GQ_MATH_LOG) or reciprocal (GQ_MATH_RCP) of a float64 CUDA
        tensor, elementwise (gq_device_math); returns a new tensor."""
        import torch
        x = x.contiguous()
        out = torch.empty_like(x)
        self._check(self._L.gq_device_math(self._h, fn, x.numel(), _ptr(x), _ptr(out)))
        return out

    def eval(self, kind: int, dens1, dens2=None, out=None, direct: bool = False,
             noalloc: bool = False):
        """Evaluate on the device. dens1/dens2: torch float64 CUDA tensors (n_src,) or
        (n_dens, n_src); returns a tensor (n_tgt,) or (n_dens, n_tgt); for GQ_S_AND_D
        (2 n_dens, n_tgt), the S rows first. direct: gq_eval_direct; noalloc: gq_eval_noalloc
        (pass ``out`` as well to keep the call free of allocations)."""
        import torch
        squeeze = dens1.dim() == 1

        def rows(t):
            # keep a row-strided 2-D view (unit stride along a row), else copy
            t = t.reshape(-1, t.shape[-1]) if t.dim() == 1 else t
            return t if t.stride(-1) == 1 else t.contiguous()

        d1 = rows(dens1)
        d2 = None if dens2 is None else rows(dens2)
        n_dens = d1.shape[0]
        if out is None:
            rows = n_dens * (2 if kind == GQ_S_AND_D else 1)
            out = torch.empty((rows, self.n_tgt), dtype=torch.float64, device=d1.device)
        fn = (self._L.gq_eval_direct if direct else
              self._L.gq_eval_noalloc if noalloc else self._L.gq_eval)
        self._check(fn(self._h, kind, n_dens, _ptr(d1), d1.stride(0), _ptr(d2),
                       0 if d2 is None else d2.stride(0), _ptr(out), out.stride(0)))
        return out[0] if squeeze and kind != GQ_S_AND_D else out


class EvalGraph:
    """A captured evaluation; ``launch()`` replays it on the context's stream."""

    def __init__(self, fmm: QBXFMM, handle, keep):
        self._fmm, self._h, self._keep = fmm, handle, keep

    def launch(self):
        self._fmm._check(self._fmm._L.gq_graph_launch(self._h))

    def close(self):
        if self._h is not None and self._h.value:
            self._fmm._L.gq_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

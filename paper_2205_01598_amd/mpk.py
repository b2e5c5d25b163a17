"""Python face of the MPK library: thin wrappers over the C-ABI.

PyTorch only supplies device memory (tensors) and streams; every step of the
computation runs in the library's HIP kernels or its C++ planner.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import check, default_options, lib


def _csr_struct(n, rowptr, col, val):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    s = _lib.mpk_csr(int(n), int(rowptr[-1]) if len(rowptr) else 0,
                     rowptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                     col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return s, (rowptr, col, val)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(int(t.data_ptr()))


def _check_vec(t, name: str, numel: int, at_least: bool = False, device: bool = True):
    """A device buffer the kernels read or write: a contiguous float64 GPU
    tensor of ``numel`` elements (or more with ``at_least``).  Raises
    ValueError before anything reaches the library."""
    if t is None:
        raise ValueError(f"{name}: a tensor is required")
    if not hasattr(t, "data_ptr") or not hasattr(t, "is_cuda"):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if str(t.dtype) != "torch.float64":
        raise ValueError(f"{name}: dtype must be torch.float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    n = t.numel()
    if (n < numel) if at_least else (n != numel):
        want = f"at least {numel}" if at_least else f"{numel}"
        raise ValueError(f"{name}: expected {want} elements, got {n}")
    if device and not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU (cuda) tensor")


def _check_rec(rec, powers: int, nk: int):
    """Host coefficient arrays hold an entry per power (two for complex
    coef and coef0); y_prev and acc are N x k device buffers."""
    for nm in ("alpha", "beta", "gamma"):
        if len(getattr(rec, nm)) < powers:
            raise ValueError(f"recurrence {nm}: needs {powers} entries, got {len(getattr(rec, nm))}")
    w = 2 if rec.complex_pairs else 1
    if rec.coef is not None and len(rec.coef) < w * powers:
        raise ValueError(f"recurrence coef: needs {w * powers} entries, got {len(rec.coef)}")
    if rec.coef0 is not None and len(rec.coef0) < w:
        raise ValueError(f"recurrence coef0: needs {w} entries, got {len(rec.coef0)}")
    for nm in ("y_prev", "acc"):
        if getattr(rec, nm) is not None:
            _check_vec(getattr(rec, nm), nm, nk, device=False)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _f64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Recurrence:
    """Three-term recurrence epilogue (see ``mpk_recurrence`` in include/mpk.h)."""

    def __init__(self, alpha, beta=None, gamma=None, coef=None, complex_pairs=False,
                 y_prev=None, acc=None, coef0=None):
        p = len(alpha)
        self.alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        self.beta = np.ascontiguousarray(beta if beta is not None else np.zeros(p), dtype=np.float64)
        self.gamma = np.ascontiguousarray(gamma if gamma is not None else np.zeros(p), dtype=np.float64)
        self.coef = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64)
        self.complex_pairs = bool(complex_pairs)
        self.y_prev = y_prev
        self.acc = acc
        self.coef0 = None if coef0 is None else np.ascontiguousarray(np.atleast_1d(coef0), dtype=np.float64)

    def struct(self):
        return _lib.mpk_recurrence(
            _f64p(self.alpha), _f64p(self.beta), _f64p(self.gamma),
            _f64p(self.coef) if self.coef is not None else None,
            int(self.complex_pairs),
            int(self.y_prev.data_ptr()) if self.y_prev is not None else None,
            int(self.acc.data_ptr()) if self.acc is not None else None,
            _f64p(self.coef0) if self.coef0 is not None else None)


class Plan:
    """``mpk_plan``: preprocessing (levels, level groups, Lp schedule, tiles)
    plus the device copy of the renumbered matrix."""

    def __init__(self, A, p: int, cache_bytes: int, *, upload: bool = True, **opts):
        self._h = None
        s, keep = _csr_struct(A.n, A.rowptr, A.col, A.val)
        o = default_options(**opts)
        h = ctypes.c_void_p()
        check(lib().mpk_plan_create(ctypes.byref(s), int(p), int(cache_bytes), ctypes.byref(o),
                                    ctypes.byref(h)))
        self._h = h
        self.n = int(A.n)
        self.nnz = int(s.nnz)
        self.p = int(p)
        self.nrhs = int(o.nrhs)
        if upload:
            self.upload()

    @classmethod
    def from_device(cls, rowptr, col, val, p: int, cache_bytes: int, *, upload: bool = True, **opts):
        """``mpk_plan_create_device``: plan a CSR held in GPU tensors
        (int64 rowptr[n+1], int32 col[nnz], float64 val[nnz]; rows sorted,
        pattern symmetric, at most 4096 entries per row).  Levels, renumbering
        and P A P^T run on the GPU and the renumbered matrix stays there."""
        arrays = ((rowptr, "rowptr", "torch.int64"), (col, "col", "torch.int32"), (val, "val", "torch.float64"))
        for t, name, dt in arrays:
            if not hasattr(t, "data_ptr") or not hasattr(t, "is_cuda"):
                raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
            if str(t.dtype) != dt:
                raise ValueError(f"{name}: dtype must be {dt}, got {t.dtype}")
            if not t.is_contiguous():
                raise ValueError(f"{name}: must be contiguous")
        for t, name, _ in arrays:
            if not t.is_cuda:
                raise ValueError(f"{name}: must be a GPU (cuda) tensor")
        n = rowptr.numel() - 1
        if n < 0:
            raise ValueError("rowptr: needs n + 1 >= 1 entries")
        if val.numel() != col.numel():
            raise ValueError(f"val: expected {col.numel()} elements (one per column index), got {val.numel()}")
        s = _lib.mpk_csr(int(n), int(col.numel()),
                         ctypes.cast(int(rowptr.data_ptr()), ctypes.POINTER(ctypes.c_int64)),
                         ctypes.cast(int(col.data_ptr()), ctypes.POINTER(ctypes.c_int32)),
                         ctypes.cast(int(val.data_ptr()), ctypes.POINTER(ctypes.c_double)))
        o = default_options(**opts)
        h = ctypes.c_void_p()
        self = cls.__new__(cls)
        self._h = None
        check(lib().mpk_plan_create_device(ctypes.byref(s), int(p), int(cache_bytes), ctypes.byref(o),
                                           ctypes.byref(h)))
        self._h = h
        self.n = int(n)
        self.nnz = int(col.numel())
        self.p = int(p)
        self.nrhs = int(o.nrhs)
        if upload:
            self.upload()
        return self

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib._lib is not None:
            lib().mpk_plan_destroy(self._h)
            self._h = None

    def upload(self):
        check(lib().mpk_plan_upload(self._h))

    def retune(self, p: int, cache_bytes: int, **opts):
        """New p / cache budget / launch options on the same BFS levels."""
        o = default_options(**opts)
        check(lib().mpk_plan_retune(self._h, int(p), int(cache_bytes), ctypes.byref(o)))
        self.p = int(p)
        self.nrhs = int(o.nrhs)
        return self

    def info(self) -> dict:
        i = _lib.mpk_plan_info()
        check(lib().mpk_plan_query(self._h, ctypes.byref(i)))
        d = {name: getattr(i, name) for name, _ in i._fields_}
        d["phase_seconds"] = list(d["phase_seconds"])
        return d

    def arrays(self):
        inf = self.info()
        n, L, G = inf["n"], inf["n_levels"], inf["n_groups"]
        perm = np.empty(n, np.int32)
        lp = np.empty(L + 1, np.int32)
        gp = np.empty(G + 1, np.int32)
        sch = np.empty(3 * G * self.p, np.int32)
        P = ctypes.POINTER(ctypes.c_int32)
        check(lib().mpk_plan_arrays(self._h, perm.ctypes.data_as(P), lp.ctypes.data_as(P),
                                    gp.ctypes.data_as(P), sch.ctypes.data_as(P)))
        return perm, lp, gp, sch.reshape(-1, 3)

    def matrix(self):
        rowptr = np.empty(self.n + 1, np.int64)
        col = np.empty(self.nnz, np.int32)
        val = np.empty(self.nnz, np.float64)
        check(lib().mpk_plan_matrix(self._h, rowptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _f64p(val)))
        return rowptr, col, val

    def tiles(self):
        inf = self.info()
        T, W = inf["n_tiles"], inf["n_tickets"]
        tr = np.empty(T + 1, np.int32)
        lo = np.empty(T, np.int32)
        hi = np.empty(T, np.int32)
        work = np.empty(W, np.int32)
        P = ctypes.POINTER(ctypes.c_int32)
        check(lib().mpk_plan_tiles(self._h, tr.ctypes.data_as(P), lo.ctypes.data_as(P),
                                   hi.ctypes.data_as(P), work.ctypes.data_as(P)))
        return tr, lo, hi, work

    def tile_deps(self, line_closed: bool = False):
        T = self.info()["n_tiles"]
        d = np.empty(6 * T, np.int32)
        check(lib().mpk_plan_tile_deps(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(line_closed)))
        return d.reshape(T, 6)

    def units(self):
        """Refined plans (recursion_stages > 0, Sec. 4.4): (unit_ptr,
        unit_stage, dep_ptr, dep_rng) as numpy arrays; dep_rng has shape
        (n_dep_ranges, 2), inclusive tile ranges."""
        info = self.info()
        U, T, R = info["n_units"], info["n_tiles"], info["n_dep_ranges"]
        up, us = np.empty(U + 1, np.int32), np.empty(U, np.int32)
        dp, dr = np.empty(T + 1, np.int32), np.empty(2 * R, np.int32)
        P = ctypes.POINTER(ctypes.c_int32)
        check(lib().mpk_plan_units(self._h, up.ctypes.data_as(P), us.ctypes.data_as(P), dp.ctypes.data_as(P),
                                   dr.ctypes.data_as(P)))
        return up, us, dp, dr.reshape(R, 2)

    # -- device calls ------------------------------------------------------------
    def permute(self, x, out, to_plan: bool, stream=None):
        k = 1 if x.dim() == 1 else x.shape[-1]
        _check_vec(x, "in", self.n * k)
        _check_vec(out, "out", self.n * k)
        check(lib().mpk_permute(self._h, _ptr(x), _ptr(out), int(k), int(to_plan), _stream(stream)))
        return out

    def _run_args(self, X, Y, rec, powers):
        powers = self.p if powers is None else int(powers)
        if not 1 <= powers <= self.p:
            raise ValueError(f"powers must be in [1, {self.p}], got {powers}")
        nk = self.n * self.nrhs
        if rec is not None:
            _check_rec(rec, powers, nk)
        _check_vec(X, "X", nk, device=False)
        _check_vec(Y, "Y", powers * nk, at_least=True, device=False)
        for nm, t in (("X", X), ("Y", Y)) + ((("y_prev", rec.y_prev), ("acc", rec.acc)) if rec else ()):
            if t is not None and not t.is_cuda:
                raise ValueError(f"{nm}: must be a GPU (cuda) tensor")
        return powers, (ctypes.byref(rec.struct()) if rec is not None else None)

    def run(self, X, Y, rec: Recurrence | None = None, stream=None, powers: int | None = None):
        """y_1..y_powers (default: all p) of X into Y (plan order)."""
        powers, r = self._run_args(X, Y, rec, powers)
        if powers == self.p:
            check(lib().mpk_run(self._h, _ptr(X), _ptr(Y), r, _stream(stream)))
        else:
            check(lib().mpk_run_first(self._h, powers, _ptr(X), _ptr(Y), r, _stream(stream)))
        return Y

    def run_baseline(self, X, Y, rec: Recurrence | None = None, stream=None, powers: int | None = None):
        powers, r = self._run_args(X, Y, rec, powers)
        if powers == self.p:
            check(lib().mpk_run_baseline(self._h, _ptr(X), _ptr(Y), r, _stream(stream)))
        else:
            check(lib().mpk_run_baseline_first(self._h, powers, _ptr(X), _ptr(Y), r, _stream(stream)))
        return Y

    def run_sync(self, X, Y, granularity: str = "wavefront", stream=None):
        """Level-blocked MPK with a kernel launch per Lp node ("node") or per
        wavefront of independent nodes ("wavefront") instead of
        point-to-point flags."""
        g = {"node": 0, "wavefront": 1}[granularity]
        self._run_args(X, Y, None, None)
        check(lib().mpk_run_sync(self._h, _ptr(X), _ptr(Y), g, _stream(stream)))
        return Y

    def status(self, stream=None):
        check(lib().mpk_plan_status(self._h, _stream(stream)))


class Spmv:
    """``mpk_spmv``: baseline SpMV on a matrix in its given order."""

    def __init__(self, A, **opts):
        self._h = None
        s, keep = _csr_struct(A.n, A.rowptr, A.col, A.val)
        o = default_options(**opts)
        h = ctypes.c_void_p()
        check(lib().spmv_create(ctypes.byref(s), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.n = int(A.n)
        self.nrhs = int(o.nrhs)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib._lib is not None:
            lib().spmv_destroy(self._h)
            self._h = None

    def run(self, x, y, stream=None):
        _check_vec(x, "x", self.n * self.nrhs)
        _check_vec(y, "y", self.n * self.nrhs)
        check(lib().spmv_run(self._h, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def powers(self, p: int, X, Y, stream=None):
        _check_vec(X, "X", self.n * self.nrhs)
        _check_vec(Y, "Y", int(p) * self.n * self.nrhs, at_least=True)
        check(lib().spmv_powers_run(self._h, int(p), _ptr(X), _ptr(Y), _stream(stream)))
        return Y


def bw_probe(buf, reps: int, workgroups: int, sink, stream=None, loads_per_thread: int = 0, parts: int = 1):
    """Load-only read probe over the whole tensor ``buf``; loads_per_thread
    > 0 selects ``mpk_bw_probe_ex`` (that many loads in flight per thread,
    buffer cut into ``parts`` per-XCD parts)."""
    nbytes = buf.numel() * buf.element_size()
    if loads_per_thread:
        check(lib().mpk_bw_probe_ex(_ptr(buf), int(nbytes), int(reps), int(workgroups), int(loads_per_thread),
                                    int(parts), _ptr(sink), _stream(stream)))
    else:
        check(lib().mpk_bw_probe(_ptr(buf), int(nbytes), int(reps), int(workgroups), _ptr(sink),
                                 _stream(stream)))


def xcd_ids(ids, workgroups: int, spin: int = 0, stream=None):
    """Hardware XCD of every workgroup of a launch (``mpk_xcd_ids``) into the
    int32 device tensor ``ids``."""
    check(lib().mpk_xcd_ids(_ptr(ids), int(workgroups), int(spin), _stream(stream)))
    return ids


def hop_probe(flags, peer: int, scope: int, iters: int, max_polls: int, out, stream=None):
    """Round trips of a flag between workgroups 0 and ``peer`` (``mpk_hop_probe``)
    into ``out``; returns the wall-clock tick rate in kHz."""
    khz = ctypes.c_int32(0)
    check(lib().mpk_hop_probe(_ptr(flags), int(peer), int(scope), int(iters), int(max_polls), _ptr(out),
                              ctypes.byref(khz), _stream(stream)))
    return khz.value

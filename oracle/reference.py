"""Plain CPU oracle for the level-blocked MPK (arXiv 2205.01598).

TEST INFRASTRUCTURE ONLY.  Nothing here is on the product path; the product
library must never import this module.  It is slow on purpose: plain loops in
C (``oracle.c``) and plain Python/numpy, FP64 throughout unless a function says
otherwise, with no blocking, fusion or reordering beyond what the paper's
definition states.

Functions and the passages they follow
  spmv_powers        Sec. 3 / Sec. 3.1 (Fig. 2): the MPK computes y_p = A^p x
                     for p = 1..p_m and stores every y_p; the baseline is p_m
                     back-to-back CRS SpMVs.  This is the exact target every
                     MPK variant must reproduce (level blocking only reorders
                     these operations, Sec. 4.2).  threads > 1 shares the rows
                     of every SpMV among OpenMP threads (static schedule, the
                     paper's baseline, Sec. 6); each row is still summed in
                     stored order, so the result is the same bit for bit.
  permute_symmetric  P A P^T of the Sec. 4.1 renumbering (the permuted
                     matrix the MPK runs on).
  round_values       values as FP32 / BF16 storage holds them, as FP64; with
                     spmv_powers the FP64-arithmetic mixed-precision variant
  spmv_powers_lowp   the same product with matrix values stored in FP32 or
                     BF16 and FP32 accumulation (an extension, not in the
                     paper; parity for it is tolerance-based, not exact).
  bfs_levels         Eq. (3) levels and the Sec. 4.1 renumbering (levels
                     numbered consecutively, L(i-1) before L(i)).
  peripheral_root    root choice for Eq. (3); the paper uses vertex 0 in its
                     example (Sec. 4.1) and leaves the choice open otherwise.
  level_nnz          nonzeros per level, the N_nz(T) of Eq. (5).
  level_groups       greedy level groups of Sec. 4.3, criterion Eq. (5).
  lp_schedule        diagonal traversal of the Lp diagram, Sec. 4.2 / Fig. 6.
  cheb_coefficients  Chebyshev expansion coefficients of exp(-i H dt)
                     (Sec. 7, Eq. (6)-(8); the coefficient formula is the
                     standard Jacobi-Anger expansion the paper cites).
  cheb_propagate     one Chebyshev time step, Eq. (7)-(8).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.orc_spmv_powers.restype = ctypes.c_int
    lib.orc_spmv_powers.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int32,
                                    ctypes.c_int32, _f64p, _f64p]
    lib.orc_spmv_powers_omp.restype = ctypes.c_int
    lib.orc_spmv_powers_omp.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int32,
                                        ctypes.c_int32, _f64p, _f64p, ctypes.c_int32]
    lib.orc_spmv_powers_lowp.restype = ctypes.c_int
    lib.orc_spmv_powers_lowp.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, _f64p, _f64p]
    lib.orc_round_values.restype = ctypes.c_int
    lib.orc_round_values.argtypes = [ctypes.c_int64, _f64p, ctypes.c_int32, _f64p]
    lib.orc_bfs_distances.restype = ctypes.c_int
    lib.orc_bfs_distances.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i64p]
    lib.orc_peripheral_root.restype = ctypes.c_int64
    lib.orc_peripheral_root.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64]
    lib.orc_bfs_levels.restype = ctypes.c_int64
    lib.orc_bfs_levels.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p, _i64p]
    _lib = lib
    return lib


def _arrs(A):
    rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return rowptr, col, val


def _p(a, t):
    return a.ctypes.data_as(t)


# ----------------------------------------------------------------------------
# powers
# ----------------------------------------------------------------------------

def spmv_powers(A, x, p: int, threads: int = 1) -> np.ndarray:
    """y_q = A y_{q-1}, y_0 = x, for q = 1..p (Sec. 3.1, Fig. 2), FP64.

    ``x`` has shape (n,) or (n, k) (k right-hand sides, row-major).  Returns an
    array of shape (p, n) or (p, n, k) holding y_1..y_p.  ``threads`` > 1
    runs the rows of each SpMV on that many OpenMP threads with the same
    per-row arithmetic (identical result).
    """
    rowptr, col, val = _arrs(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = 1 if x.ndim == 1 else x.shape[1]
    y = np.empty((p, A.n * k), dtype=np.float64)
    if threads > 1:
        rc = _load().orc_spmv_powers_omp(A.n, _p(rowptr, _i64p), _p(col, _i32p), _p(val, _f64p),
                                         k, p, _p(x, _f64p), _p(y, _f64p), int(threads))
    else:
        rc = _load().orc_spmv_powers(A.n, _p(rowptr, _i64p), _p(col, _i32p), _p(val, _f64p),
                                     k, p, _p(x, _f64p), _p(y, _f64p))
    if rc != 0:
        raise ValueError("orc_spmv_powers failed")
    return y.reshape((p, A.n) if x.ndim == 1 else (p, A.n, k))


def spmv_powers_lowp(A, x, p: int, vdtype: str) -> np.ndarray:
    """Mixed-precision powers: values rounded to ``vdtype`` ('f32' or 'bf16'),
    each input vector rounded to FP32, products summed in FP32, each power
    stored as FP64 (the stored value is the FP32 sum, exactly)."""
    code = {"f32": 1, "bf16": 2}[vdtype]
    rowptr, col, val = _arrs(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = 1 if x.ndim == 1 else x.shape[1]
    y = np.empty((p, A.n * k), dtype=np.float64)
    rc = _load().orc_spmv_powers_lowp(A.n, _p(rowptr, _i64p), _p(col, _i32p), _p(val, _f64p),
                                      code, k, p, _p(x, _f64p), _p(y, _f64p))
    if rc != 0:
        raise ValueError("orc_spmv_powers_lowp failed")
    return y.reshape((p, A.n) if x.ndim == 1 else (p, A.n, k))


def round_values(A, vdtype: str):
    """A with its values rounded as FP32 ('f32') or BF16 ('bf16') storage
    holds them (round to nearest even; BF16 via FP32), widened back to FP64.
    spmv_powers on the result is the FP64-arithmetic variant of the
    mixed-precision product: reduced storage, FP64 products and sums."""
    code = {"f32": 1, "bf16": 2}[vdtype]
    rowptr, col, val = _arrs(A)
    out = np.empty(A.nnz, dtype=np.float64)
    if _load().orc_round_values(A.nnz, _p(val, _f64p), code, _p(out, _f64p)):
        raise ValueError("orc_round_values failed")
    return type(A)(A.n, A.rowptr, A.col, out)


# ----------------------------------------------------------------------------
# levels, groups, schedule
# ----------------------------------------------------------------------------

def bfs_distances(A, root: int) -> np.ndarray:
    """Unweighted graph distance from ``root`` in the graph of A + A^T
    (-1 outside root's component)."""
    rowptr, col, _ = _arrs(A)
    d = np.empty(A.n, dtype=np.int64)
    if _load().orc_bfs_distances(A.n, _p(rowptr, _i64p), _p(col, _i32p), int(root), _p(d, _i64p)):
        raise ValueError("bad root")
    return d


def peripheral_root(A, start: int = 0) -> int:
    """George-Liu pseudo-peripheral vertex reached from ``start``."""
    rowptr, col, _ = _arrs(A)
    r = _load().orc_peripheral_root(A.n, _p(rowptr, _i64p), _p(col, _i32p), int(start))
    if r < 0:
        raise ValueError("peripheral_root failed")
    return int(r)


def bfs_levels(A, root_mode: int = 0):
    """BFS levels (Eq. 3) and the renumbering of Sec. 4.1.

    root_mode 0: v_root = 0 (the choice of the worked example in Sec. 4.1);
    root_mode 1: the pseudo-peripheral vertex reached from vertex 0.
    Returns (perm, level_ptr): perm[new] = old (int32), level_ptr int64[L+1].
    """
    rowptr, col, _ = _arrs(A)
    n = A.n
    if n == 0:
        return np.zeros(0, np.int32), np.zeros(1, np.int64)
    root = 0 if root_mode == 0 else peripheral_root(A, 0)
    perm = np.empty(n, dtype=np.int32)
    lp = np.empty(n + 1, dtype=np.int64)
    L = _load().orc_bfs_levels(n, _p(rowptr, _i64p), _p(col, _i32p), root,
                               _p(perm, _i32p), _p(lp, _i64p))
    if L < 0:
        raise ValueError("orc_bfs_levels failed")
    return perm, lp[: L + 1].copy()


def level_nnz(A, perm, level_ptr) -> np.ndarray:
    """Stored nonzeros of A in the rows of each level (int64)."""
    rowlen = np.diff(np.asarray(A.rowptr, dtype=np.int64))
    out = np.zeros(len(level_ptr) - 1, dtype=np.int64)
    for i in range(len(level_ptr) - 1):
        rows = np.asarray(perm[level_ptr[i]:level_ptr[i + 1]], dtype=np.int64)
        out[i] = int(rowlen[rows].sum())
    return out


def level_groups(lnnz, p: int, cache_bytes: int, f: float = 0.5,
                 bytes_per_nnz: int = 12) -> np.ndarray:
    """Greedy level groups, Eq. (5): (p+1) * N_nz(T) * b < f*C.

    Starting from the first ungrouped level, levels are added while the
    accumulated group still satisfies Eq. (5) with strict '<'; a level that
    violates Eq. (5) on its own becomes a group of its own.  The budget f*C is
    taken as floor(f*C) bytes and every comparison is in integers.  Returns
    group_ptr (int64[G+1], indices into the level list).
    """
    budget = int(np.floor(float(f) * float(cache_bytes)))
    L = len(lnnz)
    gptr = [0]
    i = 0
    while i < L:
        acc = int(lnnz[i])
        j = i + 1
        while j < L and (p + 1) * (acc + int(lnnz[j])) * bytes_per_nnz < budget:
            acc += int(lnnz[j])
            j += 1
        gptr.append(j)
        i = j
    return np.asarray(gptr, dtype=np.int64)


def lp_schedule(G: int, p: int) -> np.ndarray:
    """Diagonal traversal of the Lp diagram (Sec. 4.2, Fig. 6).

    Diagonals d = i + p' run left to right (d = 1 .. G+p-1); inside one
    diagonal the power p' rises from max(1, d-(G-1)) to min(d, p) and the
    node is (i = d - p', p').  Returns int64[G*p, 3] rows (d, p', i); the row
    index is the execution step, counted from 0.
    """
    out = []
    for d in range(1, G + p):
        for q in range(max(1, d - (G - 1)), min(d, p) + 1):
            out.append((d, q, d - q))
    return np.asarray(out, dtype=np.int64).reshape(-1, 3)


def permute_symmetric(A, perm):
    """P A P^T with perm[new] = old (Sec. 4.1): entry (i, j) of the result is
    A[perm[i], perm[j]].  Every stored entry (r, c, v) of A moves to
    (iperm[r], iperm[c], v); the entries are then ordered by (new row, new
    column) with a stable sort, so duplicates keep their stored order.
    Returns (rowptr int64[n+1], col int32[nnz], val float64[nnz])."""
    n = A.n
    iperm = np.empty(n, dtype=np.int64)
    iperm[np.asarray(perm, dtype=np.int64)] = np.arange(n)
    old_rowptr = np.asarray(A.rowptr, dtype=np.int64)
    new_row = iperm[np.repeat(np.arange(n, dtype=np.int64), np.diff(old_rowptr))]
    new_col = iperm[np.asarray(A.col, dtype=np.int64)]
    order = np.lexsort((new_col, new_row))  # stable: last key is the primary one
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(new_row, minlength=n), out=rowptr[1:])
    return rowptr, new_col[order].astype(np.int32), np.asarray(A.val, dtype=np.float64)[order]


# ----------------------------------------------------------------------------
# Chebyshev time propagation (Sec. 7)
# ----------------------------------------------------------------------------

def cheb_coefficients(M: int, r_dt: float, c_dt: float = 0.0) -> np.ndarray:
    """c_k, k = 0..M, of exp(-i H dt) = sum_k c_k T_k(A) for H = r A + c.

    Jacobi-Anger: exp(-i tau A) = J_0(tau) + 2 sum_{k>=1} (-i)^k J_k(tau) T_k(A),
    times the phase exp(-i c dt).  J_k comes from scipy.special.jv.
    """
    from scipy.special import jv

    k = np.arange(M + 1)
    c = (2.0 - (k == 0)) * ((-1j) ** k) * jv(k, r_dt)
    return c * np.exp(-1j * c_dt)


def cheb_propagate(A, x, coeffs, threads: int = 1) -> np.ndarray:
    """One time step x' = sum_k c_k v_k with v_0 = x, v_1 = A x,
    v_{k+1} = 2 A v_k - v_{k-1} (Eq. 7-8).

    ``x`` is complex, given as (n, 2) [re, im]; A is real, so each product is
    an SpMV on the two real columns.  Returns (n, 2).  ``threads`` is passed
    to spmv_powers (same result)."""
    xc = np.asarray(x, dtype=np.float64)
    M = len(coeffs) - 1
    v_prev = xc.copy()
    acc = coeffs[0].real * v_prev + coeffs[0].imag * np.stack([-v_prev[:, 1], v_prev[:, 0]], 1)
    if M == 0:
        return acc
    v = spmv_powers(A, v_prev, 1, threads)[0]
    acc += coeffs[1].real * v + coeffs[1].imag * np.stack([-v[:, 1], v[:, 0]], 1)
    for k in range(2, M + 1):
        av = spmv_powers(A, v, 1, threads)[0]
        v_next = 2.0 * av - v_prev
        acc += coeffs[k].real * v_next + coeffs[k].imag * np.stack([-v_next[:, 1], v_next[:, 0]], 1)
        v_prev, v = v, v_next
    return acc

def heat_coefficients(M: int, tau: float) -> np.ndarray:
    """c_k, k = 0..M, of exp(-tau (A + I)) = sum_k c_k T_k(A) (Sec. 7, heat
    equation with L = r (A + I) and tau = a dt r).

    From the generating function exp(z cos t) = I_0(z) + 2 sum_k I_k(z) cos(k t)
    at z = -tau, with I_k(-tau) = (-1)^k I_k(tau):
    c_k = (2 - delta_k0) (-1)^k I_k(tau) exp(-tau).  I_k from scipy.special.iv.
    """
    from scipy.special import iv

    k = np.arange(M + 1)
    return (2.0 - (k == 0)) * ((-1.0) ** k) * iv(k, tau) * np.exp(-tau)


def cheb_propagate_real(A, x, coeffs, threads: int = 1) -> np.ndarray:
    """One time step x' = sum_k c_k v_k with real coefficients and a real
    state (n,): v_0 = x, v_1 = A x, v_{k+1} = 2 A v_k - v_{k-1} (Eq. 7-8)."""
    v_prev = np.asarray(x, dtype=np.float64).copy()
    acc = coeffs[0] * v_prev
    if len(coeffs) == 1:
        return acc
    v = spmv_powers(A, v_prev, 1, threads)[0]
    acc = acc + coeffs[1] * v
    for k in range(2, len(coeffs)):
        v_next = 2.0 * spmv_powers(A, v, 1, threads)[0] - v_prev
        acc = acc + coeffs[k] * v_next
        v_prev, v = v, v_next
    return acc


# ----------------------------------------------------------------------------
# recursive refinement of bulky levels (Sec. 4.4)
# ----------------------------------------------------------------------------

def _undirected_adjacency(A):
    """Neighbour lists of the graph of A + A^T without the diagonal (lists of
    original indices)."""
    import scipy.sparse as sp

    S = sp.csr_matrix((np.ones(A.nnz), np.asarray(A.col, np.int64), np.asarray(A.rowptr, np.int64)),
                      shape=(A.n, A.n))
    U = ((S + S.T) != 0).tocsr()
    U.setdiag(False)
    U.eliminate_zeros()
    U.sort_indices()
    return [U.indices[U.indptr[v]:U.indptr[v + 1]] for v in range(A.n)]


def _subgraph_levels(rows, adj, pos):
    """Breadth-first levels of the subgraph induced by ``rows`` (original
    indices listed in the current numbering).  Root: the first row; each
    vertex, taken in the new order, appends its unvisited neighbours inside
    the subgraph in ascending current position; when the frontier is empty
    the first unvisited row (in current order) starts the next level.
    Returns (order, level_ptr) with order a list of original indices."""
    inside = set(int(v) for v in rows)
    seen = set()
    order, lptr = [], [0]
    scan = 0
    while len(order) < len(rows):
        while int(rows[scan]) in seen:
            scan += 1
        root = int(rows[scan])
        seen.add(root)
        frontier = [root]
        order.append(root)
        lptr.append(len(order))
        while frontier:
            nxt = []
            for u in frontier:
                nb = sorted((int(v) for v in adj[u] if int(v) in inside and int(v) not in seen), key=lambda v: pos[v])
                for v in nb:
                    seen.add(v)
                    nxt.append(v)
            if nxt:
                order.extend(nxt)
                lptr.append(len(order))
            frontier = nxt
    return order, lptr


def refine_levels(A, perm, level_ptr, p: int, cache_bytes: int, f: float = 0.5, bytes_per_nnz: int = 12,
                  stages: int = 1, row_weight=None):
    """Recursive level refinement (Sec. 4.4), up to ``stages`` stages (s_m).

    At stage s the levels are grouped by Eq. (5) (``level_groups``); every
    maximal run of consecutive groups that violate Eq. (5) (single bulky
    levels) is replaced by the breadth-first levels of the subgraph it
    induces (``_subgraph_levels``), which are grouped and refined again at
    stage s+1, as long as s+1 <= stages.  Groups that satisfy Eq. (5), and
    violating ones at the last stage, are kept as they are.  Nonzeros per
    level count the whole rows of A.

    ``row_weight`` (per original row) replaces the row lengths in Eq. (5),
    e.g. ones for the vertex-counting cache of the Sec. 4.4 example.

    Returns (perm, unit_ptr, unit_stage): the final numbering (new -> old),
    the row boundaries of the final groups ("units", int64[U+1]) in that
    numbering, and the stage each unit comes from.
    """
    rowlen = (np.diff(np.asarray(A.rowptr, dtype=np.int64)) if row_weight is None
              else np.asarray(row_weight, dtype=np.int64))
    adj = _undirected_adjacency(A)
    pos = np.empty(A.n, dtype=np.int64)
    pos[np.asarray(perm, dtype=np.int64)] = np.arange(A.n)
    budget = int(np.floor(float(f) * float(cache_bytes)))

    def refine(rows, lptr, stage):
        lnnz = np.array([int(rowlen[np.asarray(rows[lptr[i]:lptr[i + 1]], dtype=np.int64)].sum())
                         for i in range(len(lptr) - 1)], dtype=np.int64)
        gptr = level_groups(lnnz, p, cache_bytes, f, bytes_per_nnz)
        gnnz = [int(lnnz[gptr[i]:gptr[i + 1]].sum()) for i in range(len(gptr) - 1)]
        violates = [(p + 1) * g * bytes_per_nnz >= budget for g in gnnz]
        order, units = [], []
        i, G = 0, len(gptr) - 1
        while i < G:
            if stage >= stages or not violates[i]:
                part = list(rows[lptr[gptr[i]]:lptr[gptr[i + 1]]])
                order.extend(part)
                units.append((len(part), stage))
                i += 1
                continue
            j = i
            while j < G and violates[j]:
                j += 1
            region = rows[lptr[gptr[i]]:lptr[gptr[j]]]
            sub_order, sub_lptr = _subgraph_levels(region, adj, pos)
            o2, u2 = refine(sub_order, sub_lptr, stage + 1)
            order.extend(o2)
            units.extend(u2)
            i = j
        return order, units

    order, units = refine([int(v) for v in perm], [int(v) for v in level_ptr], 0)
    unit_ptr = np.zeros(len(units) + 1, dtype=np.int64)
    unit_ptr[1:] = np.cumsum([u[0] for u in units])
    return (np.asarray(order, dtype=np.int32), unit_ptr, np.asarray([u[1] for u in units], dtype=np.int64))

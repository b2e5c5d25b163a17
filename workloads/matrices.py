"""Seeded sparse-matrix and vector generators (inputs only).

Every generator returns a :class:`CSR` with 0-based ``int64`` row pointers,
``int32`` column indices sorted ascending within each row, and ``float64``
values.  Random draws come from ``numpy.random.Generator(PCG64)`` streams that
:func:`seed_streams` spawns from one seed in the fixed order
[permutation, values, vector], so the same seed always yields the same input.

Shapes follow the workloads of the paper: grid stencils (the 2d-7pt worked
example of Sec. 4.1, the HPCG-like 27-point matrix of Table 2, the order-2/4/6
heat-equation stencils of Table 3), the Anderson model Hamiltonian of Sec. 7
(open boundaries, which reproduces the nonzero count Table 3 gives), and
synthetic irregular matrices (random geometric graphs, banded random,
power-law row lengths) that stand in for the SuiteSparse set of Table 2,
which is not available here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Host CSR matrix: ``rowptr`` int64[n+1], ``col`` int32[nnz], ``val`` float64[nnz]."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        np.add.at(d, (rows, self.col.astype(np.int64)), self.val)
        return d


def seed_streams(seed: int):
    """Three independent generators: (permutation, values, vector)."""
    ss = np.random.SeedSequence(int(seed))
    kids = ss.spawn(3)
    return tuple(np.random.Generator(np.random.PCG64(k)) for k in kids)


# ----------------------------------------------------------------------------
# padded (N x m) construction helpers
# ----------------------------------------------------------------------------

def _compress(cols_pad: np.ndarray, vals_pad: np.ndarray, valid: np.ndarray) -> CSR:
    n = cols_pad.shape[0]
    counts = valid.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols_pad[valid].astype(np.int32)
    val = vals_pad[valid].astype(np.float64)
    return CSR(n, rowptr, col, val)


def _relabel_padded(cols_pad, vals_pad, valid, new2old):
    """Symmetric relabelling P A P^T of a padded matrix; columns re-sorted per row."""
    n = cols_pad.shape[0]
    old2new = np.empty(n, dtype=np.int64)
    old2new[new2old] = np.arange(n, dtype=np.int64)
    cols = cols_pad[new2old]
    vals = vals_pad[new2old]
    ok = valid[new2old]
    mapped = np.where(ok, old2new[np.where(ok, cols, 0)], n)
    order = np.argsort(mapped, axis=1, kind="stable")
    mapped = np.take_along_axis(mapped, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    ok = mapped < n
    return mapped, vals, ok


def _grid_offsets(dim: int, offsets):
    """Sort stencil offsets by their linear index so CSR columns come out ascending."""
    return sorted(offsets, key=lambda o: sum(o[d] * (10 ** (3 * d)) for d in range(dim)))


def _grid_stencil(shape, offsets, values_fn):
    """Padded stencil matrix on a box with open (Dirichlet) boundaries.

    ``shape`` = (nx, ny[, nz]) with x fastest.  ``values_fn(valid, is_diag)``
    returns the padded value array.
    """
    dim = len(shape)
    n = int(np.prod(shape))
    offsets = _grid_offsets(dim, offsets)
    m = len(offsets)
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for d in range(dim):
        coords.append(rem % shape[d])
        rem = rem // shape[d]
    strides = [int(np.prod(shape[:d])) for d in range(dim)]
    cols = np.empty((n, m), dtype=np.int64)
    valid = np.ones((n, m), dtype=bool)
    is_diag = np.zeros(m, dtype=bool)
    for j, off in enumerate(offsets):
        lin = 0
        for d in range(dim):
            c = coords[d] + off[d]
            valid[:, j] &= (c >= 0) & (c < shape[d])
            lin += off[d] * strides[d]
        cols[:, j] = idx + lin
        is_diag[j] = all(o == 0 for o in off)
    cols[~valid] = 0
    vals = values_fn(valid, is_diag)
    return cols, vals, valid


def _const_values(diag, off):
    def fn(valid, is_diag):
        v = np.where(is_diag[None, :], float(diag), float(off))
        return np.broadcast_to(v, valid.shape).astype(np.float64) * valid
    return fn


# ----------------------------------------------------------------------------
# stencils
# ----------------------------------------------------------------------------

def stencil_2d(n: int, points: int = 5, diag: float = 4.0, off: float = -1.0) -> CSR:
    """2D stencil on an n x n grid, lexicographic numbering v = y*n + x.

    points = 5: the standard Laplacian pattern.
    points = 7: 5-point plus the anti-diagonal pair (x+1, y-1), (x-1, y+1).
      This is the 2d-7pt pattern of the worked example in Sec. 4: with it a
      BFS from vertex 0 on the 8 x 8 grid gives the 15 levels of Fig. 4.
    points = 9: the full 3 x 3 box.
    """
    base = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    if points == 5:
        offs = base
    elif points == 7:
        offs = base + [(1, -1), (-1, 1)]
    elif points == 9:
        offs = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
    else:
        raise ValueError("points must be 5, 7 or 9")
    cols, vals, valid = _grid_stencil((n, n), offs, _const_values(diag, off))
    return _compress(cols, vals, valid)


def _box27():
    return [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]


def _star(radius):
    offs = [(0, 0, 0)]
    for r in range(1, radius + 1):
        for d in range(3):
            for s in (1, -1):
                o = [0, 0, 0]
                o[d] = s * r
                offs.append(tuple(o))
    return offs


def stencil_3d(n: int, points: int = 7, diag: float | None = None, off: float = -1.0) -> CSR:
    """Constant-coefficient 3D stencil on an n^3 grid (x fastest), open boundaries.

    points = 7 (star), 13, 19 (longer stars) or 27 (3x3x3 box).  The default
    diagonal is (points - 1) * |off|.
    """
    if points == 27:
        offs = _box27()
    elif points in (7, 13, 19):
        offs = _star((points - 1) // 6)
    else:
        raise ValueError("points must be 7, 13, 19 or 27")
    if diag is None:
        diag = (points - 1) * abs(off)
    cols, vals, valid = _grid_stencil((n, n, n), offs, _const_values(diag, off))
    return _compress(cols, vals, valid)


def star_stencil_3d(n: int, order: int) -> CSR:
    """Finite-difference Laplacian of spatial order 2, 4 or 6 on an n^3 grid.

    These are the heat-equation matrices of Table 3 (7, 13 and 19 points per
    interior row); coefficients are the standard central-difference weights.
    """
    weights = {2: [-2.0, 1.0],
               4: [-5.0 / 2, 4.0 / 3, -1.0 / 12],
               6: [-49.0 / 18, 3.0 / 2, -3.0 / 20, 1.0 / 90]}[order]
    radius = order // 2
    offs = _star(radius)

    def fn(valid, is_diag):
        v = np.empty(len(offs))
        for j, o in enumerate(_grid_offsets(3, offs)):
            r = max(abs(c) for c in o)
            v[j] = 3 * weights[0] if r == 0 else weights[r]
        return np.broadcast_to(v, valid.shape) * valid

    cols, vals, valid = _grid_stencil((n, n, n), offs, fn)
    return _compress(cols, vals, valid)


def heat_operator_3d(n: int, order: int):
    """Heat-equation operator of Table 3 scaled for a Chebyshev expansion.

    L = -(finite-difference Laplacian of spatial order 2, 4 or 6 on an n^3
    grid, zero outside) is symmetric positive semidefinite with spectrum in
    [0, 2r], r = half the largest Gershgorin row sum of an interior row (12,
    16 and 163/9 for the three orders).  Returns (A, r) with the stored
    matrix A = L / r - I, whose spectrum lies in [-1, 1].
    """
    S = star_stencil_3d(n, order)
    weights = {2: [-2.0, 1.0],
               4: [-5.0 / 2, 4.0 / 3, -1.0 / 12],
               6: [-49.0 / 18, 3.0 / 2, -3.0 / 20, 1.0 / 90]}[order]
    gersh = 3.0 * (abs(weights[0]) + 2.0 * sum(abs(w) for w in weights[1:]))
    r = gersh / 2.0
    rows = np.repeat(np.arange(S.n), np.diff(S.rowptr))
    val = -S.val / r - (S.col.astype(np.int64) == rows)
    return CSR(S.n, S.rowptr.copy(), S.col.copy(), val), r


def stencil_27pt_random(n: int, seed: int = 0, permute: bool = True):
    """27-point stencil on an n^3 grid with random values and a dominant diagonal.

    Off-diagonal values are U[-1, 1] (drawn per (grid row, offset) in natural
    order from the value stream); a_ii = 1 + sum_j |a_ij|.  With ``permute``
    the matrix is symmetrically relabelled by a random permutation from the
    permutation stream (P A P^T).  Returns (CSR, new2old) where
    ``new2old[r]`` is the natural grid index of row r (identity if not
    permuted).
    """
    rng_perm, rng_val, _ = seed_streams(seed)
    offs = _box27()

    def fn(valid, is_diag):
        v = rng_val.uniform(-1.0, 1.0, size=valid.shape)
        v *= valid
        v[:, is_diag] = 0.0
        dsum = 1.0 + np.abs(v).sum(axis=1)
        v[:, np.nonzero(is_diag)[0][0]] = dsum
        return v

    cols, vals, valid = _grid_stencil((n, n, n), offs, fn)
    N = cols.shape[0]
    if permute:
        new2old = rng_perm.permutation(N).astype(np.int64)
        cols, vals, valid = _relabel_padded(cols, vals, valid, new2old)
    else:
        new2old = np.arange(N, dtype=np.int64)
    return _compress(cols, vals, valid), new2old


def integer_stencil_27pt(n: int, seed: int = 0, permute: bool = True) -> CSR:
    """27-point pattern with integer entries in {-2..2} (diagonal included).

    With x in {-1, 0, 1} every partial sum of A^p x for p <= 8 is an integer
    below 54^8 < 2^53, so FP64 results are exact whatever the summation order.
    """
    rng_perm, rng_val, _ = seed_streams(seed)

    def fn(valid, is_diag):
        return rng_val.integers(-2, 3, size=valid.shape).astype(np.float64) * valid

    cols, vals, valid = _grid_stencil((n, n, n), _box27(), fn)
    if permute:
        new2old = rng_perm.permutation(cols.shape[0]).astype(np.int64)
        cols, vals, valid = _relabel_padded(cols, vals, valid, new2old)
    return _compress(cols, vals, valid)


def anderson_3d(n: int, W: float = 16.0, t: float = -1.0, seed: int = 0,
                scale: float | None = None) -> CSR:
    """Anderson model Hamiltonian on an n^3 lattice with open boundaries.

    Nearest-neighbour hopping ``t`` (7-point pattern) and on-site energies
    U[-W/2, W/2] from the value stream.  The stored matrix is H / scale with
    scale = W/2 + 6|t| by default (a Gershgorin bound, so the spectrum of the
    stored matrix lies in [-1, 1] as the Chebyshev expansion of Sec. 7 needs).
    At n = 200 the pattern has the 55,760,000 nonzeros listed in Table 3.
    """
    _, rng_val, _ = seed_streams(seed)
    if scale is None:
        scale = W / 2.0 + 6.0 * abs(t)
    offs = _star(1)

    def fn(valid, is_diag):
        eps = rng_val.uniform(-W / 2.0, W / 2.0, size=valid.shape[0])
        v = np.where(is_diag[None, :], 0.0, t) * valid
        v[:, np.nonzero(is_diag)[0][0]] = eps
        return v / scale

    cols, vals, valid = _grid_stencil((n, n, n), offs, fn)
    return _compress(cols, vals, valid)


# ----------------------------------------------------------------------------
# irregular matrices
# ----------------------------------------------------------------------------

def _row_major_order(rows: np.ndarray, cols: np.ndarray, n: int) -> np.ndarray:
    """Permutation that sorts entries by (row, column), ties in input order:
    the order of ``np.lexsort((cols, rows))`` for 0 <= rows, cols < n, from
    one stable sort of a combined int64 key (an order of magnitude faster on
    10^8 entries)."""
    return np.argsort(rows.astype(np.int64) * int(n) + cols.astype(np.int64), kind="stable")


def random_geometric(N: int, avg_degree: float = 16.0, seed: int = 0,
                     radius: float | None = None):
    """Random geometric graph: N points U[0,1]^3, edge when distance < r.

    r = (3 * avg_degree / (4 pi N))^(1/3) (closed cube, no wrap-around).  One
    weight w = 1 - U[0,1) in (0, 1] per undirected edge; rows are normalised
    (A_ij = w_ij / sum_j w_ij), so A is row-stochastic; an isolated vertex gets
    A_ii = 1.  Points come from the permutation stream, weights from the value
    stream.  Returns (CSR, points).
    """
    from scipy.spatial import cKDTree

    rng_pts, rng_val, _ = seed_streams(seed)
    if radius is None:
        radius = (3.0 * avg_degree / (4.0 * np.pi * N)) ** (1.0 / 3.0)
    pts = rng_pts.random((N, 3))
    tree = cKDTree(pts)
    pairs = tree.query_pairs(radius, output_type="ndarray").astype(np.int64)
    if pairs.size:
        order = _row_major_order(pairs[:, 0], pairs[:, 1], N)
        pairs = pairs[order]
    w = 1.0 - rng_val.random(pairs.shape[0])
    rows = np.concatenate([pairs[:, 0], pairs[:, 1]])
    cols = np.concatenate([pairs[:, 1], pairs[:, 0]])
    ww = np.concatenate([w, w])
    deg = np.bincount(rows, minlength=N)
    iso = np.nonzero(deg == 0)[0]
    rows = np.concatenate([rows, iso])
    cols = np.concatenate([cols, iso])
    ww = np.concatenate([ww, np.ones(iso.size)])
    order = _row_major_order(rows, cols, N)
    rows, cols, ww = rows[order], cols[order], ww[order]
    rowsum = np.bincount(rows, weights=ww, minlength=N)
    vals = ww / rowsum[rows]
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=rowptr[1:])
    return CSR(N, rowptr, cols.astype(np.int32), vals), pts


def _from_padded_dedup(cols, vals, valid, n):
    """Sort padded rows, drop duplicate columns (keep first value), compress."""
    key = np.where(valid, cols, n)
    order = np.argsort(key, axis=1, kind="stable")
    key = np.take_along_axis(key, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    dup = np.zeros_like(valid)
    dup[:, 1:] = key[:, 1:] == key[:, :-1]
    ok = (key < n) & ~dup
    return _compress(key, vals, ok)


def _dominant_diagonal(csr: CSR) -> CSR:
    rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
    isd = csr.col.astype(np.int64) == rows
    off = np.where(isd, 0.0, np.abs(csr.val))
    dsum = 1.0 + np.bincount(rows, weights=off, minlength=csr.n)
    csr.val[isd] = dsum[rows[isd]]
    return csr


def banded_random(n: int, bandwidth: int, seed: int = 0) -> CSR:
    """Banded random matrix: 2..16 random columns per row in [i-b, i+b].

    Values U[-1, 1]; the diagonal is always present and made dominant
    (a_ii = 1 + sum |a_ij|).
    """
    _, rng_val, rng_x = seed_streams(seed)
    m = 17
    cnt = rng_x.integers(2, 17, size=n)
    offs = rng_x.integers(-bandwidth, bandwidth + 1, size=(n, m))
    idx = np.arange(n, dtype=np.int64)[:, None]
    cols = idx + offs
    cols[:, 0] = idx[:, 0]
    slot = np.arange(m)[None, :]
    valid = (slot <= cnt[:, None]) & (cols >= 0) & (cols < n)
    vals = rng_val.uniform(-1.0, 1.0, size=(n, m))
    csr = _from_padded_dedup(np.where(valid, cols, 0), vals, valid, n)
    return _dominant_diagonal(csr)


def zipf_rows(n: int, exponent: float, seed: int = 0, cap: int = 1024) -> CSR:
    """Power-law row lengths (Zipf, capped) with uniformly random columns.

    Row i gets min(Zipf(exponent), cap) off-diagonal draws plus the diagonal;
    values U[-1, 1] with a dominant diagonal.
    """
    _, rng_val, rng_x = seed_streams(seed)
    lens = np.minimum(rng_x.zipf(exponent, size=n), cap).astype(np.int64)
    total = int(lens.sum())
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = rng_x.integers(0, n, size=total)
    vals = rng_val.uniform(-1.0, 1.0, size=total)
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([vals, np.zeros(n)])
    order = _row_major_order(rows, cols, n)
    rows, cols, vals = rows[order], cols[order], vals[order]
    keep = np.ones(rows.size, dtype=bool)
    keep[1:] = (rows[1:] != rows[:-1]) | (cols[1:] != cols[:-1])
    rows, cols, vals = rows[keep], cols[keep], vals[keep]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return _dominant_diagonal(CSR(n, rowptr, cols.astype(np.int32), vals))


def random_small_csr(n: int, density: float, rng: np.random.Generator,
                     symmetric_pattern: bool = False, empty_rows: float = 0.0,
                     duplicates: float = 0.0, integer: bool = False) -> CSR:
    """Small irregular CSR for property tests.

    Options give non-symmetric patterns, empty rows, duplicate (row, col)
    entries kept as separate stored entries, and integer values.
    """
    nnz_target = max(0, int(round(density * n * n)))
    r = rng.integers(0, n, size=nnz_target) if n else np.zeros(0, np.int64)
    c = rng.integers(0, n, size=nnz_target) if n else np.zeros(0, np.int64)
    if symmetric_pattern:
        r, c = np.concatenate([r, c]), np.concatenate([c, r])
    if empty_rows > 0 and n:
        dead = rng.random(n) < empty_rows
        keep = ~dead[r]
        r, c = r[keep], c[keep]
    if duplicates > 0 and r.size:
        k = int(duplicates * r.size)
        pick = rng.integers(0, r.size, size=k)
        r, c = np.concatenate([r, r[pick]]), np.concatenate([c, c[pick]])
    if integer:
        v = rng.integers(-2, 3, size=r.size).astype(np.float64)
    else:
        v = rng.uniform(-1.0, 1.0, size=r.size)
    order = _row_major_order(r, c, n)
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    if n:
        np.cumsum(np.bincount(r, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr, c.astype(np.int32), v)


def relabel(csr: CSR, new2old: np.ndarray) -> CSR:
    """Symmetric relabelling P A P^T of a general CSR (columns re-sorted per row)."""
    n = csr.n
    old2new = np.empty(n, dtype=np.int64)
    old2new[new2old] = np.arange(n)
    lens = np.diff(csr.rowptr)[new2old]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    src = np.concatenate([np.arange(csr.rowptr[o], csr.rowptr[o + 1]) for o in new2old]) \
        if n else np.zeros(0, np.int64)
    src = src.astype(np.int64)
    rows = np.repeat(np.arange(n), lens)
    cols = old2new[csr.col[src].astype(np.int64)]
    vals = csr.val[src]
    order = _row_major_order(rows, cols, n)
    return CSR(n, rowptr, cols[order].astype(np.int32), vals[order].copy())


# ----------------------------------------------------------------------------
# vectors
# ----------------------------------------------------------------------------

def uniform_vector(n: int, k: int = 1, seed: int = 0) -> np.ndarray:
    """x ~ U[-1, 1] from the vector stream; shape (n,) for k == 1 else (n, k)."""
    _, _, rng_x = seed_streams(seed)
    x = rng_x.uniform(-1.0, 1.0, size=(n, k))
    return x[:, 0].copy() if k == 1 else x


def gaussian_block(n: int, k: int, seed: int = 0) -> np.ndarray:
    """Block of k standard-normal right-hand sides, row-major (n, k)."""
    _, _, rng_x = seed_streams(seed)
    return rng_x.standard_normal(size=(n, k))


def random_phase_state(n: int, seed: int = 0) -> np.ndarray:
    """Normalised random-phase state e^{2 pi i theta_j} / sqrt(n), as (n, 2) [re, im]."""
    _, _, rng_x = seed_streams(seed)
    th = rng_x.random(n)
    out = np.empty((n, 2))
    out[:, 0] = np.cos(2 * np.pi * th) / np.sqrt(n)
    out[:, 1] = np.sin(2 * np.pi * th) / np.sqrt(n)
    return out


# ----------------------------------------------------------------------------
# tuner corpus
# ----------------------------------------------------------------------------

def _random_valued(csr: CSR, rng) -> CSR:
    """Same pattern, values U[-1, 1] with a dominant diagonal (diagonal added
    where missing)."""
    n = csr.n
    rows = np.repeat(np.arange(n), np.diff(csr.rowptr))
    has_diag = np.zeros(n, bool)
    has_diag[rows[csr.col == rows]] = True
    if not has_diag.all():
        miss = np.nonzero(~has_diag)[0]
        rows = np.concatenate([rows, miss])
        cols = np.concatenate([csr.col.astype(np.int64), miss])
        order = _row_major_order(rows, cols, n)
        rows, cols = rows[order], cols[order]
        rowptr = np.zeros(n + 1, np.int64)
        np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
        csr = CSR(n, rowptr, cols.astype(np.int32), np.zeros(rows.size))
    vals = rng.uniform(-1.0, 1.0, size=csr.nnz)
    return _dominant_diagonal(CSR(csr.n, csr.rowptr, csr.col, vals))


def tuner_matrix(seed: int, n_min: float = 1e5, n_max: float = 1e6):
    """One matrix of the learned-tuner corpus, chosen by the seed.

    Families: 2D stencils (5, 9 points), 3D stencils (7, 13, 19, 27 points),
    banded random (bandwidth log-uniform in [10, 1000]), power-law row lengths
    (Zipf exponent in [1.5, 2.5], capped at 1024) and random geometric graphs;
    N log-uniform in [n_min, n_max]; values U[-1, 1] with a dominant diagonal
    (row-normalised weights for the geometric graphs).  Returns (CSR, spec).
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 7919]))
    fam = ["stencil2d", "stencil3d", "banded", "zipf", "rgg"][int(rng.integers(0, 5))]
    N = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
    spec = {"seed": int(seed), "family": fam}
    if fam == "stencil2d":
        pts = int(rng.choice([5, 9]))
        n = max(4, int(round(np.sqrt(N))))
        A = _random_valued(stencil_2d(n, pts), rng)
        spec.update(points=pts, grid=n)
    elif fam == "stencil3d":
        pts = int(rng.choice([7, 13, 19, 27]))
        n = max(4, int(round(N ** (1.0 / 3.0))))
        A = _random_valued(stencil_3d(n, pts), rng)
        spec.update(points=pts, grid=n)
    elif fam == "banded":
        b = int(round(np.exp(rng.uniform(np.log(10), np.log(1000)))))
        A = banded_random(N, b, seed=int(seed))
        spec.update(bandwidth=b)
    elif fam == "zipf":
        s = float(rng.uniform(1.5, 2.5))
        A = zipf_rows(N, s, seed=int(seed))
        spec.update(exponent=round(s, 3))
    else:
        A, _ = random_geometric(N, 16.0, seed=int(seed))
    spec.update(n=int(A.n), nnz=int(A.nnz))
    return A, spec

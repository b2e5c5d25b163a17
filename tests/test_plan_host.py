"""Host planner (C++ in libmpk.so, no GPU call) against the oracle: the
permutation, level pointers, level groups and Lp schedule must match bit for
bit; the renumbered matrix and the device tile table are checked by their
invariants."""
import ctypes
import re
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2205_01598_amd import MpkError, Plan, Spmv
from paper_2205_01598_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _oracle_plan(A, p, C, root_mode=0, f=0.5, bnz=12):
    perm, lp = O.bfs_levels(A, root_mode)
    lnnz = O.level_nnz(A, perm, lp)
    gp = O.level_groups(lnnz, p, C, f, bnz)
    sch = O.lp_schedule(len(gp) - 1, p)
    return perm, lp, gp, sch


def _check_plan(A, p, C, root_mode=0, f=0.5, dtype="f64", **kw):
    pl = Plan(A, p, C, upload=False, root_mode=root_mode, safety_factor=f, val_dtype=dtype, **kw)
    perm, lp, gp, sch = pl.arrays()
    bnz = {"f64": 12, "f32": 8, "bf16": 6}[dtype]
    operm, olp, ogp, osch = _oracle_plan(A, p, C, root_mode, f, bnz)
    assert np.array_equal(perm, operm)
    assert np.array_equal(lp, olp)
    assert np.array_equal(gp, ogp)
    assert np.array_equal(sch, osch)
    # renumbered matrix equals P A P^T
    rp, col, val = pl.matrix()
    orp, ocol, oval = O.permute_symmetric(A, operm)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol) and np.array_equal(val, oval)
    _check_tiles(pl, lp, gp, rp, col, skew=kw.get("skew", 1))
    return pl


def _check_tiles(pl, lp, gp, rp, col, skew=1):
    tr, lo, hi, work = pl.tiles()
    inf = pl.info()
    T = inf["n_tiles"]
    n = inf["n"]
    p = inf["p"]
    assert tr[0] == 0 and tr[-1] == n and np.all(np.diff(tr) > 0)
    group_rows = lp[gp]
    # tiles never straddle a level-group boundary
    assert set(group_rows.tolist()) <= set(tr.tolist())
    tile_group = np.searchsorted(group_rows, tr[:-1], side="right") - 1
    for t in range(T):
        r0, r1 = tr[t], tr[t + 1]
        cols = col[rp[r0]:rp[r1]]
        need_lo = min(r0, cols.min()) if cols.size else r0
        need_hi = max(r1 - 1, cols.max()) if cols.size else r1 - 1
        # dependency range covers every row read (and the tile itself) ...
        assert tr[lo[t]] <= need_lo and tr[hi[t] + 1] > need_hi
        # ... and is the tightest such range of tiles
        assert tr[lo[t] + 1] > need_lo and tr[hi[t]] <= need_hi
        assert abs(tile_group[lo[t]] - tile_group[t]) <= 1 and abs(tile_group[hi[t]] - tile_group[t]) <= 1
    # three point-to-point ranges: every column read (and the tile itself)
    # lies in a listed tile, each range stays inside its group, and the
    # bounds are the tiles of the extreme columns read in that group
    d3 = pl.tile_deps()
    for t in range(T):
        g = tile_group[t]
        r0, r1 = tr[t], tr[t + 1]
        cols = np.concatenate([col[rp[r0]:rp[r1]], np.arange(r0, r1)])
        ctile = np.searchsorted(tr, cols, side="right") - 1
        covered = np.zeros(len(cols), bool)
        for m in range(3):
            a, b = d3[t, 2 * m], d3[t, 2 * m + 1]
            if a > b:
                assert not np.any(tile_group[ctile] == g - 1 + m)
                continue
            assert tile_group[a] == g - 1 + m and tile_group[b] == g - 1 + m
            sel = tile_group[ctile] == g - 1 + m
            assert ctile[sel].min() == a and ctile[sel].max() == b
            covered |= (ctile >= a) & (ctile <= b)
        assert covered.all()
    # line-closed ranges: contain the tight ones, cover every row that shares
    # a 128-byte line of an aligned N x k slice with a row of the tight
    # range, and stop at the first tile beyond; the plan flag says whether
    # all of them are earlier tickets
    k = inf["nrhs"]
    R = max(1, 128 // (8 * k))
    dx = pl.tile_deps(line_closed=True)
    order_ok = True
    for t in range(T):
        for m in range(3):
            a, b = d3[t, 2 * m], d3[t, 2 * m + 1]
            ax, bx = dx[t, 2 * m], dx[t, 2 * m + 1]
            if a > b:
                assert (ax, bx) == (a, b)
                continue
            f, l = tr[a], tr[b + 1] - 1
            f2, l2 = f - f % R, min(n - 1, l + (R - 1 - l % R))
            assert ax <= a and bx >= b
            assert tr[ax] <= f2 < tr[ax + 1] and tr[bx] <= l2 < tr[bx + 1]
            order_ok &= bool(tile_group[bx] <= tile_group[t] + skew)
    assert inf["line_closed_deps"] == int(order_ok)
    # tickets: every (tile, power) once, in Lp diagonal order of the groups,
    # and every dependency is an earlier ticket
    tile = work // 64
    q = work % 64 + 1
    assert len(work) == T * p
    assert len(set(zip(tile.tolist(), q.tolist()))) == T * p
    pos = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(tile, q))}
    for i, (a, b) in enumerate(zip(tile, q)):
        if b > 1:
            assert pos[(int(lo[a]), int(b) - 1)] < i and pos[(int(hi[a]), int(b) - 1)] < i


def test_worked_example_plan():
    A = W.stencil_2d(8, 7)
    pl = _check_plan(A, 5, 10 ** 6)
    assert pl.info()["n_levels"] == 15


@pytest.mark.parametrize("n,root_mode", [(12, 0), (12, 1), (30, 1)])
@pytest.mark.parametrize("p,C", [(1, 2 ** 16), (4, 2 ** 20), (8, 3 * 2 ** 20)])
def test_plan_27pt_random(n, root_mode, p, C):
    A, _ = W.stencil_27pt_random(n, seed=n)
    _check_plan(A, p, C, root_mode, tile_nnz=1500)


@pytest.mark.parametrize("skew", [1, 2, 3, 8, 32])
def test_plan_skew_orders(skew):
    # skew 1 reproduces the Lp diagonal order of the schedule; any skew keeps
    # every dependency an earlier ticket
    A, _ = W.stencil_27pt_random(14, seed=5)
    pl = _check_plan(A, 5, 2 ** 19, 1, tile_nnz=3000, skew=skew)
    _, _, gp, sch = pl.arrays()
    tr, lo, hi, work = pl.tiles()
    group_rows = pl.arrays()[1][gp]
    tile_group = np.searchsorted(group_rows, tr[:-1], side="right") - 1
    nodes = []
    for w in work:
        node = (int(tile_group[w // 64]), int(w % 64 + 1))
        if not nodes or nodes[-1] != node:
            nodes.append(node)
    if skew == 1:
        assert nodes == [(int(i), int(q)) for d, q, i in sch]
    keys = [g + skew * q for g, q in nodes]
    assert keys == sorted(keys)


def test_retune_matches_fresh_plan():
    # retune keeps the levels; groups, schedule and tiles equal a fresh plan
    A, _ = W.stencil_27pt_random(16, seed=8)
    pl = Plan(A, 4, 2 ** 20, upload=False, root_mode=1, tile_nnz=2000)
    for p, C, kw in [(8, 3 * 2 ** 19, {}), (2, 2 ** 18, {"tile_nnz": 700, "skew": 2}),
                     (6, 2 ** 21, {"val_dtype": "bf16"})]:
        pl.retune(p, C, root_mode=1, **kw)
        fresh = Plan(A, p, C, upload=False, root_mode=1, **kw)
        for a, b in zip(pl.arrays(), fresh.arrays()):
            assert np.array_equal(a, b)
        for a, b in zip(pl.tiles(), fresh.tiles()):
            assert np.array_equal(a, b)
        assert np.array_equal(pl.tile_deps(), fresh.tile_deps())
    with pytest.raises(MpkError, match="MPK_ERR_ARG"):
        pl.retune(4, 2 ** 20, root_mode=0)


def test_plan_2d5pt_c1():
    A = W.stencil_2d(64, 5)
    pl = _check_plan(A, 4, 64 * 1024, tile_nnz=512)
    assert pl.info()["n_levels"] == 127


@pytest.mark.parametrize("seed", range(6))
def test_plan_irregular(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 400))
    A = W.random_small_csr(n, float(rng.uniform(0.001, 0.05)), rng,
                           symmetric_pattern=bool(seed % 2), empty_rows=0.1, duplicates=0.1)
    _check_plan(A, int(rng.integers(1, 9)), int(rng.integers(500, 50000)),
                root_mode=seed % 2, tile_nnz=int(rng.integers(1, 300)))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_plan_dtype_budget(dtype):
    # Eq. (5) counts b_nz = value bytes + 4 bytes of column index
    A, _ = W.stencil_27pt_random(16, seed=2)
    _check_plan(A, 6, 2 ** 20, 1, dtype=dtype)


def test_plan_rgg_and_banded():
    A, _ = W.random_geometric(5000, 12.0, seed=1)
    _check_plan(A, 6, 2 ** 19, 1, tile_nnz=2000)
    B = W.banded_random(3000, 40, seed=1)
    _check_plan(B, 4, 2 ** 18, 0, tile_nnz=700)
    Z = W.zipf_rows(2000, 2.0, seed=3)
    _check_plan(Z, 3, 2 ** 18, 0, tile_nnz=900)


def _direct_sum(*blocks):
    n = sum(b.n for b in blocks)
    rps, cols, vals, off, base = [np.zeros(1, np.int64)], [], [], 0, 0
    for b in blocks:
        rps.append(b.rowptr[1:] + base)
        cols.append(b.col.astype(np.int64) + off)
        vals.append(b.val)
        off += b.n
        base += b.nnz
    return W.CSR(n, np.concatenate(rps), np.concatenate(cols).astype(np.int32), np.concatenate(vals))


@pytest.mark.parametrize("root_mode", [0, 1])
def test_plan_large_unsymmetric_components(root_mode):
    # a non-symmetric pattern (transpose merged in), frontiers of thousands of
    # vertices (parallel expansion) and several components (restarts at the
    # smallest unnumbered index), randomly relabelled
    Z = W.zipf_rows(30000, 1.8, seed=4)
    S, _ = W.stencil_27pt_random(18, seed=6)
    iso = W.CSR(50, np.arange(51, dtype=np.int64), np.arange(50, dtype=np.int32), np.ones(50))
    A = _direct_sum(S, Z, iso)
    A = W.relabel(A, np.random.default_rng(9).permutation(A.n))
    pl = _check_plan(A, 4, 2 ** 21, root_mode, tile_nnz=4000)
    lp = pl.arrays()[1]
    assert np.diff(lp).max() >= 2048


def test_plan_empty_and_single():
    Z = W.CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    pl = Plan(Z, 3, 1000, upload=False)
    assert pl.info()["n_levels"] == 0 and pl.info()["n_tiles"] == 0
    S = W.CSR(1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([2.0]))
    pl = _check_plan(S, 3, 1000)
    assert pl.info()["n_tickets"] == 3


def test_plan_rejects_bad_input():
    A = W.stencil_2d(4, 5)
    bad_col = W.CSR(A.n, A.rowptr, A.col.copy(), A.val)
    bad_col.col[3] = A.n
    with pytest.raises(MpkError, match="MPK_ERR_CSR"):
        Plan(bad_col, 2, 1000, upload=False)
    bad_rp = W.CSR(A.n, A.rowptr.copy(), A.col, A.val)
    bad_rp.rowptr[5], bad_rp.rowptr[6] = bad_rp.rowptr[6], bad_rp.rowptr[5]
    with pytest.raises(MpkError, match="MPK_ERR_CSR"):
        Plan(bad_rp, 2, 1000, upload=False)
    for p in (0, 33):
        with pytest.raises(MpkError, match="MPK_ERR_ARG"):
            Plan(A, p, 1000, upload=False)
    with pytest.raises(MpkError, match="MPK_ERR_ARG"):
        Plan(A, 2, 0, upload=False)
    with pytest.raises(MpkError, match="MPK_ERR_ARG"):
        Plan(A, 2, 1000, upload=False, reserved0=1)
    with pytest.raises(MpkError, match="MPK_ERR_ARG"):
        Plan(A, 2, 1000, upload=False, plan_on_device=2)
    for skew in (0, 33):
        with pytest.raises(MpkError, match="MPK_ERR_ARG"):
            Plan(A, 2, 1000, upload=False, skew=skew)
    with pytest.raises(MpkError, match="MPK_ERR_ARG"):
        Plan(A, 2, 1000, upload=False, val_dtype="f32", accum_f64=2)
    # the baseline handle validates before it touches the device
    for kw in ({"val_dtype": 5}, {"accum_f64": 3}, {"reserved": 1}):
        with pytest.raises(MpkError, match="MPK_ERR_ARG"):
            Spmv(A, **kw)
    with pytest.raises(MpkError, match="MPK_ERR_UNSUPPORTED"):
        Plan(A, 2, 1000, upload=False, nrhs=4, val_dtype="bf16")


@pytest.mark.slow
def test_plan_c2_full_size():
    # the 160^3 27-point matrix of the benchmark: plan arrays bit-exact
    A, _ = W.stencil_27pt_random(160, seed=0)
    pl = Plan(A, 8, 256 << 20, upload=False, root_mode=1)
    perm, lp, gp, sch = pl.arrays()
    operm, olp, ogp, osch = _oracle_plan(A, 8, 256 << 20, 1)
    assert np.array_equal(perm, operm) and np.array_equal(lp, olp)
    assert np.array_equal(gp, ogp) and np.array_equal(sch, osch)
    assert len(lp) - 1 == 160


# ----------------------------------------------------------------------------
# the C-ABI surface
# ----------------------------------------------------------------------------

def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mpk.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b((?:mpk|spmv)_\w+)\s*\(", hdr))
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(_lib.SIGNATURES), declared ^ set(_lib.SIGNATURES)


def test_abi_struct_sizes():
    # the ctypes mirrors must match the C layout the library was built with
    o = _lib.default_options()
    assert o.size == ctypes.sizeof(_lib.mpk_options)
    assert o.safety_factor == 0.5 and o.nrhs == 1 and o.val_dtype == 0
    assert _lib.lib().mpk_status_string(-5).decode() == "device dependency wait timed out"
    assert _lib.lib().mpk_version().decode().startswith("mpk-gfx950")


def _greedy_chunks(rp, r0, r1, max_nnz, max_rows=1024):
    """Chunk start rows of rows [r0, r1): each chunk takes the most rows (at
    least one, at most max_rows) whose entries fit in max_nnz."""
    out, r = [], r0
    while r < r1:
        out.append(r)
        e = r + 1
        while e < r1 and e - r < max_rows and rp[e + 1] - rp[r] <= max_nnz:
            e += 1
        r = e
    return out


def _tile_cases():
    yield "27pt_20", W.stencil_27pt_random(20, seed=3)[0]
    # power-law rows, some longer than a chunk, and a dense row
    Z = W.zipf_rows(6000, 1.5, seed=2, cap=5000)
    yield "zipf_long_rows", W.CSR(Z.n, Z.rowptr, Z.col, Z.val)
    # most rows empty except the diagonal of every tenth row
    n = 30000
    d = np.arange(0, n, 10)
    rp = np.zeros(n + 1, np.int64)
    rp[d + 1] = 1
    yield "sparse_rows", W.CSR(n, np.cumsum(rp), d.astype(np.int32), np.ones(len(d)))


@pytest.mark.parametrize("name,A", list(_tile_cases()), ids=[c[0] for c in _tile_cases()])
@pytest.mark.parametrize("k,tile", [(1, 8192), (1, 12288), (1, 6000), (2, 4096), (4, 4096), (1, 1000)])
def test_tiles_are_runs_of_whole_chunks(name, A, k, tile):
    # A tile of at least one kernel chunk (4096 nonzeros at k = 1, 1024 at
    # k = 2, 4096/k for k >= 4, include/mpk.h) is a run of whole chunks: its
    # group's rows cut greedily into chunks, round(tile / chunk) chunks per
    # tile, shared out equally.  Smaller tiles split the nonzeros equally.
    pl = Plan(A, 4, 1 << 20, upload=False, root_mode=1, nrhs=k, tile_nnz=tile)
    _, lp, gp, _ = pl.arrays()
    rp = pl.matrix()[0]
    tr = pl.tiles()[0]
    cnz = 1024 if k == 2 else 4096 // k
    group_rows = lp[gp]
    n_chunks = 0
    for g in range(len(gp) - 1):
        r0, r1 = int(group_rows[g]), int(group_rows[g + 1])
        bounds = [int(v) for v in tr if r0 <= v < r1]
        assert bounds[0] == r0
        if tile >= cnz:
            ch = _greedy_chunks(rp, r0, r1, cnz)
            m = max(1, (tile + cnz // 2) // cnz)
            nt = max(1, -(-len(ch) // m))
            assert bounds == [ch[len(ch) * t // nt] for t in range(nt)]
        for a, b in zip(bounds, bounds[1:] + [r1]):
            n_chunks += len(_greedy_chunks(rp, a, b, cnz))
    assert pl.info()["n_chunks"] == n_chunks

"""Refined plans (recursive level refinement, Sec. 4.4) built by the host
planner against the oracle: the final numbering, the final level groups
("units") and their stages must match ``oracle.refine_levels`` bit for bit;
the device tiles, per-tile dependency lists and ticket order are checked by
their invariants (every row a tile reads, and every row sharing a 128-byte
line with one, belongs to a tile it waits for; every dependency is an
earlier ticket)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2205_01598_amd import MpkError, Plan


def _case(name):
    if name == "2d5pt":
        return W.stencil_2d(40, 5), 4, 6000
    if name == "27pt":
        return W.stencil_27pt_random(12, seed=3)[0], 3, 40000
    if name == "rgg":
        return W.random_geometric(3000, 10.0, seed=2)[0], 2, 3000
    if name == "27pt_p8":
        return W.stencil_27pt_random(16, seed=1)[0], 8, 60000
    if name == "banded":
        return W.banded_random(2500, 40, seed=4), 3, 4000
    if name == "irregular":
        rng = np.random.default_rng(7)
        A = W.random_small_csr(600, 0.008, rng, empty_rows=0.05, duplicates=0.05)
        return A, 2, 900
    raise KeyError(name)


def _line_rows(k):
    return max(1, 128 // (8 * k))


def _check_refined(pl, A, p, k=1, skew=1):
    inf = pl.info()
    n = A.n
    assert inf["recursive"] == 1 and inf["line_closed_deps"] == 1
    perm = pl.arrays()[0]
    up, us, dp, dr = pl.units()
    tr, lo, hi, work = pl.tiles()
    T = inf["n_tiles"]
    assert tr[0] == 0 and tr[-1] == n and np.all(np.diff(tr) > 0)
    # tiles never straddle a unit boundary
    assert set(up.tolist()) <= set(tr.tolist())
    # renumbered matrix equals P A P^T in the refined numbering
    rp, col, val = pl.matrix()
    orp, ocol, oval = O.permute_symmetric(A, perm)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol) and np.array_equal(val, oval)
    # dependency lists: ascending, disjoint, non-adjacent ranges covering
    # the tile itself, the tiles of its columns and their line neighbours
    row_tile = np.repeat(np.arange(T), np.diff(tr))
    R = _line_rows(k)
    assert dp[0] == 0 and dp[-1] == len(dr) and np.all(np.diff(dp) >= 1)
    assert dr.min() >= 0 and dr.max() < T          # the kernel indexes flags with them
    for t in range(T):
        rng = dr[dp[t]:dp[t + 1]]
        assert np.all(rng[:, 0] <= rng[:, 1])
        assert np.all(rng[1:, 0] > rng[:-1, 1] + 1 + 31)       # closer ranges are merged
        covered = np.zeros(T, bool)
        for a, b in rng:
            covered[a:b + 1] = True
        rows = np.concatenate([np.arange(tr[t], tr[t + 1]), col[rp[tr[t]]:rp[tr[t + 1]]]])
        lines = np.unique(rows // R)
        line_rows = (lines[:, None] * R + np.arange(R)[None, :]).ravel()
        line_rows = line_rows[line_rows < n]
        assert covered[row_tile[line_rows]].all(), f"tile {t}: a needed tile is missing"
        assert lo[t] == rng[0, 0] and hi[t] == rng[-1, 1]
    # tickets: every (tile, power) once; every dependency earlier
    assert len(work) == T * p
    tile, q = work // 64, work % 64 + 1
    rank = np.full((T, p + 1), -1, np.int64)
    rank[tile, q] = np.arange(len(work))
    assert np.all(rank[:, 1:] >= 0)
    for t in range(T):
        deps = np.concatenate([np.arange(a, b + 1) for a, b in dr[dp[t]:dp[t + 1]]])
        for qq in range(2, p + 1):
            assert rank[deps, qq - 1].max() < rank[t, qq]
    return perm, up, us


@pytest.mark.parametrize("case", ["2d5pt", "27pt", "rgg", "banded", "irregular"])
@pytest.mark.parametrize("stages", [1, 2])
def test_refined_plan_matches_oracle(case, stages):
    A, p, C = _case(case)
    pl = Plan(A, p, C, upload=False, root_mode=1, recursion_stages=stages, tile_nnz=256)
    perm, up, us = _check_refined(pl, A, p)
    operm, olp = O.bfs_levels(A, 1)
    fp, oup, ous = O.refine_levels(A, operm, olp, p, C, stages=stages)
    assert np.array_equal(perm, fp)
    assert np.array_equal(up, oup)
    assert np.array_equal(us, ous)
    assert us.max() >= 1                       # the case exercises refinement
    # level groups and schedule still describe the stage-0 levels
    _, lp, gp, sch = pl.arrays()
    assert np.array_equal(lp, olp)
    assert np.array_equal(gp, O.level_groups(O.level_nnz(A, operm, olp), p, C))


@pytest.mark.parametrize("k", [1, 2, 8])
def test_refined_plan_multi_rhs_lines(k):
    A, p, C = _case("27pt")
    pl = Plan(A, p, C, upload=False, root_mode=1, recursion_stages=1, nrhs=k, tile_nnz=300)
    _check_refined(pl, A, p, k=k)


@pytest.mark.parametrize("skew", [1, 2])
def test_refined_plan_default_tiles_and_skew(skew):
    A, p, C = _case("27pt_p8")
    pl = Plan(A, p, C, upload=False, root_mode=1, recursion_stages=2, skew=skew)
    _check_refined(pl, A, p, skew=skew)


def test_refined_plan_without_violations_is_unrefined():
    # a budget every level group satisfies: nothing is refined (the oracle's
    # units are the level groups), and the plan is the unrefined one
    A = W.stencil_2d(30, 5)
    pl = Plan(A, 3, 1 << 30, upload=False, recursion_stages=2)
    p0 = Plan(A, 3, 1 << 30, upload=False)
    assert pl.info()["recursive"] == 0
    with pytest.raises(MpkError):
        pl.units()
    operm, olp = O.bfs_levels(A, 0)
    fp, up, us = O.refine_levels(A, operm, olp, 3, 1 << 30, stages=2)
    assert np.all(us == 0)
    for a, b in zip(pl.arrays(), p0.arrays()):
        assert np.array_equal(a, b)
    for a, b in zip(pl.tiles(), p0.tiles()):
        assert np.array_equal(a, b)
    assert np.array_equal(pl.arrays()[0], fp)


def test_refined_plan_xcd_streams_keep_the_order():
    # eight ticket streams slice the tiles of every unit; the tiles and the
    # ticket order of the plan stay those of the single-stream plan
    A, p, C = _case("2d5pt")
    one = Plan(A, p, C, upload=False, recursion_stages=1)
    eight = Plan(A, p, C, upload=False, recursion_stages=1, xcd_streams=8)
    assert eight.info()["recursive"] == 1
    for a, b in zip(one.tiles(), eight.tiles()):
        assert np.array_equal(a, b)
    for a, b in zip(one.units(), eight.units()):
        assert np.array_equal(a, b)


def test_refined_plan_rejections():
    A, p, C = _case("2d5pt")
    with pytest.raises(MpkError):
        Plan(A, p, C, upload=False, recursion_stages=-1)
    with pytest.raises(MpkError):
        Plan(A, p, C, upload=False, recursion_stages=17)
    pl = Plan(A, p, C, upload=False, recursion_stages=1)
    with pytest.raises(MpkError):
        pl.retune(p, 2 * C)
    # an unrefined plan cannot be retuned into a refined one, and has no units
    pl0 = Plan(A, p, C, upload=False)
    with pytest.raises(MpkError):
        pl0.retune(p, C, recursion_stages=1)
    with pytest.raises(MpkError):
        pl0.units()


def test_empty_and_tiny_refined():
    A = W.stencil_2d(1, 5)
    pl = Plan(A, 2, 100, upload=False, recursion_stages=1)
    assert pl.info()["n"] == 1


@pytest.mark.parametrize("seed", range(12))
def test_refined_plan_random_graphs(seed):
    # small irregular matrices (unsymmetric patterns, empty rows, duplicates,
    # disconnected parts) with random p, budget and stage limit
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(20, 700))
    A = W.random_small_csr(n, float(rng.uniform(1.5, 8.0)) / n, rng, symmetric_pattern=bool(seed % 2),
                           empty_rows=0.05 * (seed % 3), duplicates=0.05 * (seed % 2))
    p = int(rng.integers(1, 9))
    C = int(rng.integers(200, 20000))
    stages = int(rng.integers(1, 4))
    root_mode = seed % 2
    pl = Plan(A, p, C, upload=False, root_mode=root_mode, recursion_stages=stages,
              tile_nnz=int(rng.integers(8, 200)), skew=int(rng.integers(1, 3)))
    perm, up, us = _check_refined(pl, A, p)
    operm, olp = O.bfs_levels(A, root_mode)
    fp, oup, ous = O.refine_levels(A, operm, olp, p, C, stages=stages)
    assert np.array_equal(perm, fp)
    assert np.array_equal(up, oup) and np.array_equal(us, ous)

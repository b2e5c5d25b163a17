"""Plans from a CSR in GPU memory (mpk_plan_create_device).

Levels, renumbering and P A P^T run on the GPU and the renumbered matrix
stays there; the tile dependencies are found on the device.  Everything the
plan exposes must equal the host planner's plan of the same matrix bit for
bit (root, permutation, levels, groups, schedule, P A P^T, tiles, both
dependency tables, tickets, features), runs must give the same results bit
for bit, also with FP32/BF16 values converted on the device, and a retune
must stay equal as well.  Matrices the device path does not take (non-
symmetric pattern, unsorted rows, rows above 4096 entries, refinement) and
malformed CSR arrays are rejected with an error before anything is
computed."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2205_01598_amd import Plan, tune
from paper_2205_01598_amd._lib import MpkError

torch = pytest.importorskip("torch")
sp = pytest.importorskip("scipy.sparse")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _sym(A):
    """Pattern of A + A^T, rows sorted, values summed."""
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    S = (S + S.T).tocsr()
    S.sort_indices()
    return W.CSR(A.n, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64))


def _direct_sum(*blocks):
    rps, cols, vals, off, base = [np.zeros(1, np.int64)], [], [], 0, 0
    for b in blocks:
        rps.append(b.rowptr[1:] + base)
        cols.append(b.col.astype(np.int64) + off)
        vals.append(b.val)
        off += b.n
        base += b.nnz
    return W.CSR(off, np.concatenate(rps), np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def _arrow(n, seed):
    # one full row and column: a renumbered row of n entries (sorted on the
    # device by the long-row path when n > 256)
    rows = np.concatenate([np.zeros(n, np.int64), np.arange(1, n), np.arange(1, n)])
    cols = np.concatenate([np.arange(n), np.zeros(n - 1, np.int64), np.arange(1, n)])
    order = np.lexsort((cols, rows))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    A = W.CSR(n, np.cumsum(rp), cols[order].astype(np.int32), np.random.default_rng(seed).uniform(-1, 1, len(rows)))
    return W.relabel(A, np.random.default_rng(seed + 1).permutation(n))


def _cases():
    yield "worked_example", W.stencil_2d(8, 7)
    yield "2d9pt_64", W.stencil_2d(64, 9)
    yield "27pt_random_24", W.stencil_27pt_random(24, seed=2)[0]
    yield "rgg", W.random_geometric(6000, 12.0, seed=1)[0]
    yield "banded_sym", _sym(W.banded_random(5000, 300, seed=2))
    S, _ = W.stencil_27pt_random(10, seed=6)
    iso = W.CSR(40, np.arange(41, dtype=np.int64), np.arange(40, dtype=np.int32), np.ones(40))
    U = _direct_sum(S, _sym(W.zipf_rows(3000, 2.2, seed=4, cap=200)), iso)
    yield "components", W.relabel(U, np.random.default_rng(9).permutation(U.n))
    yield "arrow_1500", _arrow(1500, 1)
    yield "arrow_4096", _arrow(4096, 3)  # the longest row the device path sorts
    yield "symmetric_duplicates", W.random_small_csr(400, 0.02, np.random.default_rng(7), symmetric_pattern=True,
                                                     duplicates=0.2)
    yield "single", W.CSR(1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([2.0]))


def _to_dev(A, dev):
    return (torch.from_numpy(np.ascontiguousarray(A.rowptr, np.int64)).to(dev),
            torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(A.val, np.float64)).to(dev))


def _same_plan(a, b):
    ia, ib = a.info(), b.info()
    for k in ("n", "nnz", "root", "n_levels", "n_groups", "n_tiles", "n_tickets", "max_level_rows",
              "max_group_nnz", "violating_groups", "n_chunks", "tile_nnz", "line_closed_deps"):
        assert ia[k] == ib[k], k
    for x, y in zip(a.arrays(), b.arrays()):
        assert np.array_equal(x, y)
    for x, y in zip(a.matrix(), b.matrix()):
        assert np.array_equal(x, y)
    for x, y in zip(a.tiles(), b.tiles()):
        assert np.array_equal(x, y)
    for lc in (0, 1):
        assert np.array_equal(a.tile_deps(lc), b.tile_deps(lc))
    assert np.array_equal(tune.plan_features(a), tune.plan_features(b))


def _run_bits(pl, x, p, dev):
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    Y = torch.full((p,) + tuple(X.shape), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    return Y.cpu().numpy().view(np.int64)


@pytest.mark.parametrize("root_mode", [0, 1])
@pytest.mark.parametrize("name,A", list(_cases()), ids=[c[0] for c in _cases()])
def test_device_resident_plan_equals_host_plan(name, A, root_mode):
    dev = _dev()
    p = 4
    host = Plan(A, p, 1 << 20, root_mode=root_mode, skew=2)
    rp, col, val = _to_dev(A, dev)
    res = Plan.from_device(rp, col, val, p, 1 << 20, root_mode=root_mode, skew=2)
    del rp, col, val  # the plan keeps its own copy
    _same_plan(res, host)
    x = W.uniform_vector(A.n, seed=5)
    yr = _run_bits(res, x, p, dev)
    assert np.array_equal(yr, _run_bits(host, x, p, dev))
    # and the oracle on the renumbered matrix: bit for bit, except where a
    # row is longer than one MPK chunk (4096 entries at k = 1) and is
    # reduced by a tree across the workgroup
    perm = res.arrays()[0].astype(np.int64)
    rpo, co, vo = O.permute_symmetric(A, perm)
    ref = O.spmv_powers(W.CSR(A.n, rpo, co, vo), np.ascontiguousarray(x[perm]), p)
    if np.diff(A.rowptr).max(initial=0) <= 4096:
        assert np.array_equal(yr, ref.view(np.int64))
    else:
        got = yr.view(np.float64)
        for q in range(p):
            assert np.linalg.norm(got[q] - ref[q]) <= 1e-12 * np.linalg.norm(ref[q])
    # a retune keeps the two plans equal (tiles and dependencies recomputed
    # on the device for the resident plan)
    for pl in (host, res):
        pl.retune(6, 4 << 20, root_mode=root_mode, skew=3, tile_nnz=512)
    _same_plan(res, host)
    assert np.array_equal(_run_bits(res, x, 6, dev), _run_bits(host, x, 6, dev))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("accum_f64", [0, 1])
def test_device_value_conversion_equals_host(dtype, accum_f64):
    # FP32/BF16 values of a resident plan are converted on the device; the
    # host converts with the C cast and nearest-even on the upper bits.  A
    # diagonal matrix with x = 1 returns the converted values themselves
    # (with FP64 arithmetic): ties, subnormal results, overflow, signed zero,
    # FP64 subnormals, infinities and NaN.
    dev = _dev()
    t = 2.0 ** -24
    special = [1 + t, 1 + 3 * t, 1 - t / 2, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 2.0 ** -140, 1.5 * 2.0 ** -149,
               2.5 * 2.0 ** -149, 2.0 ** -150, 0.75 * 2.0 ** -149, 2.0 ** -151, 3.4028235677973366e38,
               3.4028235e38 * (1 + 2.0 ** -25), 3.5e38, -0.0, 5e-324, -1e-310, np.inf, -np.inf, np.nan,
               -np.nan, 1.0 / 3.0, -2.0 / 3.0, 65504.0, 1e-45, 1.17549435e-38, 1.1754942e-38]
    rng = np.random.default_rng(3)
    vals = np.concatenate([special, rng.standard_normal(200) * 10.0 ** rng.integers(-40, 40, 200)])
    n = len(vals)
    A = W.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), vals)
    host = Plan(A, 1, 1 << 20, val_dtype=dtype, accum_f64=accum_f64)
    res = Plan.from_device(*_to_dev(A, dev), 1, 1 << 20, val_dtype=dtype, accum_f64=accum_f64)
    x = np.ones(n)
    assert np.array_equal(_run_bits(res, x, 1, dev), _run_bits(host, x, 1, dev))
    # the large matrix path too: a retune to the other storage type
    other = "bf16" if dtype == "f32" else "f32"
    for pl in (host, res):
        pl.retune(1, 1 << 20, val_dtype=other, accum_f64=accum_f64)
    assert np.array_equal(_run_bits(res, x, 1, dev), _run_bits(host, x, 1, dev))


def test_device_resident_27pt_48_p8_run():
    # wide levels; several runs of the resident plan in the benchmark's kind
    # of configuration, bit for bit equal to the host plan's
    dev = _dev()
    A, _ = W.stencil_27pt_random(48, seed=1)
    host = Plan(A, 8, 16 << 20, root_mode=1, skew=2, tile_nnz=8192)
    res = Plan.from_device(*_to_dev(A, dev), 8, 16 << 20, root_mode=1, skew=2, tile_nnz=8192)
    _same_plan(res, host)
    x = W.uniform_vector(A.n, seed=3)
    a = _run_bits(res, x, 8, dev)
    assert np.array_equal(a, _run_bits(host, x, 8, dev))
    assert np.array_equal(a, _run_bits(res, x, 8, dev))


def test_device_resident_empty_matrix():
    dev = _dev()
    rp = torch.zeros(1, dtype=torch.int64, device=dev)
    col = torch.zeros(0, dtype=torch.int32, device=dev)
    val = torch.zeros(0, dtype=torch.float64, device=dev)
    pl = Plan.from_device(rp, col, val, 3, 1 << 20)
    inf = pl.info()
    assert inf["n"] == 0 and inf["nnz"] == 0 and inf["n_levels"] == 0


def _status(fn):
    """The library's error status of fn(), None if it succeeds."""
    try:
        fn()
    except MpkError as e:
        return e.status
    return None


def test_device_resident_rejections():
    dev = _dev()
    A = W.stencil_2d(16, 5)
    rp, col, val = _to_dev(A, dev)
    # malformed arrays: column out of range, row pointers not monotone, rowptr[n] != nnz
    bad = col.clone()
    bad[5] = A.n
    assert _status(lambda: Plan.from_device(rp, bad, val, 2, 1 << 20)) == -2
    bad = col.clone()
    bad[7] = -1
    assert _status(lambda: Plan.from_device(rp, bad, val, 2, 1 << 20)) == -2
    brp = rp.clone()
    brp[3] = brp[4] + 1
    assert _status(lambda: Plan.from_device(brp, col, val, 2, 1 << 20)) == -2
    assert _status(lambda: Plan.from_device(rp, col[:-1], val[:-1], 2, 1 << 20)) == -2
    # matrices the device path does not take
    Z = W.zipf_rows(2000, 2.0, seed=1, cap=50)  # non-symmetric pattern
    assert _status(lambda: Plan.from_device(*_to_dev(Z, dev), 2, 1 << 20)) == -6
    uns = col.clone().cpu().numpy()
    r0, r1 = int(A.rowptr[20]), int(A.rowptr[21])
    uns[r0:r1] = uns[r0:r1][::-1].copy()  # a row in descending column order
    assert _status(lambda: Plan.from_device(rp, torch.from_numpy(uns).to(dev), val, 2, 1 << 20)) == -6
    assert _status(lambda: Plan.from_device(*_to_dev(_arrow(4097, 5), dev), 2, 1 << 20)) == -6
    # an entry below the diagonal without its transpose (every entry above
    # it has one): caught by the count of entries above and below
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).tolil()
    S[40, 3] = 1.0
    S = S.tocsr()
    S.sort_indices()
    L = W.CSR(A.n, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64))
    assert _status(lambda: Plan.from_device(*_to_dev(L, dev), 2, 1 << 20)) == -6
    assert _status(lambda: Plan.from_device(*_to_dev(_sym(L), dev), 2, 1 << 20)) is None
    assert _status(lambda: Plan.from_device(rp, col, val, 2, 1 << 20, recursion_stages=1)) == -6
    assert _status(lambda: Plan.from_device(rp, col, val, 0, 1 << 20)) == -1
    # the same plan is still made from good arrays afterwards
    pl = Plan.from_device(rp, col, val, 2, 1 << 20)
    assert pl.info()["n"] == A.n


def test_device_resident_chebyshev_step_equals_host_plan():
    # the recurrence epilogue (two columns, complex coefficients) on a plan
    # made from device memory: a Chebyshev step equals the host plan's bit
    # for bit, also with a remainder block (degree 12, p = 5)
    from paper_2205_01598_amd.cheb import ChebPropagator

    dev = _dev()
    A = W.anderson_3d(20, seed=3)
    x = W.random_phase_state(A.n, seed=3)
    for p, M in ((8, 16), (5, 12)):
        host = Plan(A, p, 1 << 20, root_mode=1, nrhs=2, skew=2, tile_nnz=1024)
        res = Plan.from_device(*_to_dev(A, dev), p, 1 << 20, root_mode=1, nrhs=2, skew=2, tile_nnz=1024)
        assert np.array_equal(res.arrays()[0], host.arrays()[0])
        perm = host.arrays()[0].astype(np.int64)
        X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
        outs = []
        for pl in (host, res):
            acc = torch.full_like(X, float("nan"))
            ChebPropagator.schroedinger(pl, M, 4.0).step(X, acc)
            pl.status()
            outs.append(acc.cpu().numpy().view(np.int64))
        assert np.array_equal(outs[0], outs[1])

"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

FP64 bar: ||y_p - y_p^oracle||_2 / ||y_p^oracle||_2 <= 1e-12 for every power
(the summation order differs from the oracle's, so not bit for bit), and bit
equality where the inputs make every partial sum an exact integer.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import MpkError, Plan, Recurrence, Spmv  # noqa: E402

TOL = 1e-12


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to_plan(x, perm):
    return x[perm.astype(np.int64)]


def _from_plan(y, perm):
    out = np.empty_like(y)
    out[..., perm.astype(np.int64), :] = y if y.ndim == 3 else y[..., None]
    return out


def _unpermute_powers(Y, perm):
    # Y: (p, n[, k]) in plan order -> original order
    out = np.empty_like(Y)
    out[:, perm.astype(np.int64)] = Y
    return out


def _rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def run_mpk(A, x, p, C, baseline=False, **opts):
    dev = _dev()
    pl = Plan(A, p, C, **opts)
    perm = pl.arrays()[0]
    xp = _to_plan(x, perm)
    X = torch.from_numpy(np.ascontiguousarray(xp)).to(dev)
    Y = torch.full((p,) + tuple(X.shape), float("nan"), dtype=torch.float64, device=dev)
    (pl.run_baseline if baseline else pl.run)(X, Y)
    pl.status()
    torch.cuda.synchronize()
    return _unpermute_powers(Y.cpu().numpy(), perm), pl


def check_powers(Y, ref, tol=TOL):
    for q in range(ref.shape[0]):
        e = _rel_err(Y[q], ref[q])
        assert e <= tol, f"power {q + 1}: rel err {e:.3e}"


# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tile_nnz,C", [(0, 64 * 1024), (600, 64 * 1024), (128, 8 * 1024), (0, 1 << 30)])
def test_c1_2d5pt(tile_nnz, C):
    # 64 x 64 Laplacian, p = 4, natural order (the small configuration)
    A = W.stencil_2d(64, 5)
    x = W.uniform_vector(A.n, seed=0)
    ref = O.spmv_powers(A, x, 4)
    Y, pl = run_mpk(A, x, 4, C, tile_nnz=tile_nnz)
    check_powers(Y, ref)
    Yb, _ = run_mpk(A, x, 4, C, baseline=True, tile_nnz=tile_nnz)
    check_powers(Yb, ref)


@pytest.mark.parametrize("root_mode", [0, 1])
@pytest.mark.parametrize("p", [1, 4, 8])
@pytest.mark.parametrize("tile", [300, 2000, 9000])
@pytest.mark.parametrize("streams,skew", [(1, 1), (8, 2)])
def test_27pt_random(root_mode, p, tile, streams, skew):
    A, _ = W.stencil_27pt_random(24, seed=p + root_mode)
    x = W.uniform_vector(A.n, seed=p)
    ref = O.spmv_powers(A, x, p)
    Y, pl = run_mpk(A, x, p, 2 << 20, root_mode=root_mode, tile_nnz=tile, xcd_streams=streams, skew=skew)
    assert pl.info()["n_tiles"] > 10
    check_powers(Y, ref)


@pytest.mark.parametrize("skew,streams,wg", [(8, 1, 0), (12, 1, 64), (32, 8, 0), (32, 1, 16)])
def test_large_skews_thin_levels(skew, streams, wg):
    # thin levels (2D 9-point stencil from a corner: 299 levels) and small
    # level groups, with ticket skews that keep dependencies many diagonals
    # back; the same sums as the baseline, so equal bit for bit
    A = W.stencil_2d(150, 9)
    x = W.uniform_vector(A.n, seed=skew)
    ref = O.spmv_powers(A, x, 8)
    Y, pl = run_mpk(A, x, 8, 1 << 17, root_mode=1, tile_nnz=400, skew=skew, xcd_streams=streams, workgroups=wg)
    assert pl.info()["n_groups"] > 50
    check_powers(Y, ref)
    Yb, _ = run_mpk(A, x, 8, 1 << 17, baseline=True, root_mode=1, tile_nnz=400)
    assert np.array_equal(Y, Yb)


def test_integer_bit_exact():
    A = W.integer_stencil_27pt(20, seed=5)
    rng = np.random.default_rng(5)
    x = rng.integers(-1, 2, size=A.n).astype(np.float64)
    ref = O.spmv_powers(A, x, 8)
    Y, _ = run_mpk(A, x, 8, 1 << 20, tile_nnz=3000)
    assert np.array_equal(Y, ref)
    Yb, _ = run_mpk(A, x, 8, 1 << 20, baseline=True)
    assert np.array_equal(Yb, ref)


@pytest.mark.parametrize("seed", range(5))
def test_irregular_edge_cases(seed):
    # non-symmetric patterns, empty rows, duplicate entries, disconnected graphs
    rng = np.random.default_rng(200 + seed)
    n = [1, 2, 57, 300, 1500][seed]
    A = W.random_small_csr(n, min(0.5, 3.0 / n), rng, symmetric_pattern=bool(seed % 2),
                           empty_rows=0.1, duplicates=0.1)
    x = rng.uniform(-1, 1, size=n)
    p = [1, 3, 5, 7, 8][seed]
    ref = O.spmv_powers(A, x, p)
    Y, _ = run_mpk(A, x, p, 4096, tile_nnz=17, root_mode=seed % 2)
    check_powers(Y, ref)


def test_irregular_generators():
    for A, p in [(W.random_geometric(20000, 16.0, seed=3)[0], 6),
                 (W.banded_random(30000, 300, seed=2), 4),
                 (W.zipf_rows(20000, 1.8, seed=1), 3)]:
        x = W.uniform_vector(A.n, seed=1)
        ref = O.spmv_powers(A, x, p)
        Y, _ = run_mpk(A, x, p, 1 << 20, root_mode=1, tile_nnz=4000)
        check_powers(Y, ref)


def test_spmv_given_order_and_powers():
    dev = _dev()
    A, _ = W.stencil_27pt_random(20, seed=7)
    x = W.uniform_vector(A.n, seed=7)
    ref = O.spmv_powers(A, x, 3)
    h = Spmv(A)
    X = torch.from_numpy(x).to(dev)
    y = torch.empty_like(X)
    h.run(X, y)
    Y = torch.empty((3, A.n), dtype=torch.float64, device=dev)
    h.powers(3, X, Y)
    torch.cuda.synchronize()
    assert _rel_err(y.cpu().numpy(), ref[0]) <= TOL
    check_powers(Y.cpu().numpy(), ref)


def test_permute_round_trip():
    dev = _dev()
    A, _ = W.stencil_27pt_random(10, seed=1)
    pl = Plan(A, 2, 1 << 20, nrhs=4)
    perm = pl.arrays()[0].astype(np.int64)
    x = torch.randn(A.n, 4, dtype=torch.float64, device=dev)
    xp = torch.empty_like(x)
    back = torch.empty_like(x)
    pl.permute(x, xp, to_plan=True)
    pl.permute(xp, back, to_plan=False)
    torch.cuda.synchronize()
    assert torch.equal(back, x)
    assert torch.equal(xp.cpu(), x.cpu()[perm])


@pytest.mark.parametrize("k", [2, 4, 8, 16, 32])
def test_multi_rhs(k):
    A, _ = W.random_geometric(6000, 16.0, seed=k)
    X = W.gaussian_block(A.n, k, seed=k)
    ref = O.spmv_powers(A, X, 6)
    Y, _ = run_mpk(A, X, 6, 1 << 19, nrhs=k, root_mode=1, tile_nnz=2500)
    check_powers(Y, ref)
    Y, _ = run_mpk(A, X, 6, 1 << 19, nrhs=k, root_mode=1, tile_nnz=700, xcd_streams=8, workgroups=24)
    check_powers(Y, ref)


@pytest.mark.parametrize("dtype,u", [("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)])
def test_mixed_precision(dtype, u):
    # exact on representable integers ...
    A = W.integer_stencil_27pt(12, seed=3)
    rng = np.random.default_rng(2)
    x = rng.integers(-1, 2, size=A.n).astype(np.float64)
    ref = O.spmv_powers(A, x, 4)
    Y, _ = run_mpk(A, x, 4, 1 << 20, val_dtype=dtype, tile_nnz=1000)
    assert np.array_equal(Y, ref)
    # ... and within the FP32 accumulation bound of the low-precision oracle
    B, _ = W.stencil_27pt_random(16, seed=4)
    x = W.uniform_vector(B.n, seed=4)
    low = O.spmv_powers_lowp(B, x, 4, dtype)
    absB = W.CSR(B.n, B.rowptr, B.col, np.abs(B.val))
    bound = O.spmv_powers(absB, np.abs(x), 4)
    Y, _ = run_mpk(B, x, 4, 1 << 20, val_dtype=dtype, tile_nnz=1000)
    for q in range(4):
        # the kernel and the oracle share the rounded matrix; they differ by
        # FP32 summation order and FMA, (nrow + 2) * 2^-24 per power, grown
        # through the later powers
        c = (q + 1) * 31 * 2.0 ** -24
        assert np.all(np.abs(Y[q] - low[q]) <= c * bound[q])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("baseline", [False, True])
def test_mixed_precision_fp64_arithmetic(dtype, k, baseline):
    # values stored as FP32 / BF16, products and sums in FP64: the FP64 oracle
    # on the rounded values, to the FP64 bar (summation order only)
    B, _ = W.stencil_27pt_random(16, seed=5)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (B.n, k)) if k > 1 else rng.uniform(-1, 1, B.n)
    ref = O.spmv_powers(O.round_values(B, dtype), x, 5)
    Y, pl = run_mpk(B, x, 5, 1 << 20, baseline=baseline, val_dtype=dtype, accum_f64=1, nrhs=k, tile_nnz=900,
                    skew=2)
    check_powers(Y.reshape(ref.shape), ref)
    # FP32 arithmetic on the same storage is measurably further from it
    Y32, _ = run_mpk(B, x, 5, 1 << 20, baseline=baseline, val_dtype=dtype, nrhs=k, tile_nnz=900, skew=2)
    assert _rel_err(Y32.reshape(ref.shape)[4], ref[4]) > 1e-9


def test_chebyshev_bf16_fp64_arithmetic():
    # a Chebyshev step (complex state, recurrence epilogue) with BF16 storage
    # and FP64 arithmetic equals the FP64 oracle on the rounded Hamiltonian
    from paper_2205_01598_amd.cheb import ChebPropagator

    dev = _dev()
    A = W.anderson_3d(12, seed=4)
    x = W.random_phase_state(A.n, seed=4)
    M, p, r_dt = 32, 8, 10.0
    ref = O.cheb_propagate(O.round_values(A, "bf16"), x, O.cheb_coefficients(M, r_dt))
    pl = Plan(A, p, 1 << 20, nrhs=2, root_mode=1, tile_nnz=700, skew=2, val_dtype="bf16", accum_f64=1)
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator.schroedinger(pl, M, r_dt)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    for baseline in (False, True):
        acc = torch.empty_like(X)
        prop.step(X, acc, baseline=baseline)
        pl.status()
        h = np.empty((A.n, 2))
        h[perm] = acc.cpu().numpy()
        assert _rel_err(h, ref) <= 1e-12


def test_recurrence_chebyshev_blocks():
    # degree-16 Chebyshev step as two MPK blocks of p = 8 with complex state
    dev = _dev()
    A = W.anderson_3d(10, seed=1)
    x = W.random_phase_state(A.n, seed=1)
    M, p = 16, 8
    c = O.cheb_coefficients(M, 4.0)
    ref = O.cheb_propagate(A, x, c)
    pl = Plan(A, p, 1 << 20, nrhs=2, tile_nnz=800)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    acc = (c[0].real * X + c[0].imag * torch.stack([-X[:, 1], X[:, 0]], 1)).contiguous()
    Y = torch.empty((p, A.n, 2), dtype=torch.float64, device=dev)
    coef = np.stack([c[1:p + 1].real, c[1:p + 1].imag], 1).ravel()
    alpha = np.array([1.0] + [2.0] * (p - 1))
    gamma = np.array([0.0] + [-1.0] * (p - 1))
    pl.run(X, Y, Recurrence(alpha, None, gamma, coef, True, None, acc))
    # second block: y_{-1} = v_7, y_0 = v_8
    X2 = Y[p - 1].clone()
    prev = Y[p - 2].clone()
    Y2 = torch.empty_like(Y)
    coef2 = np.stack([c[p + 1:2 * p + 1].real, c[p + 1:2 * p + 1].imag], 1).ravel()
    pl.run(X2, Y2, Recurrence(np.full(p, 2.0), None, np.full(p, -1.0), coef2, True, prev, acc))
    pl.status()
    out = np.empty((A.n, 2))
    out[perm] = acc.cpu().numpy()
    assert _rel_err(out, ref) <= 1e-12
    # the baseline path (p back-to-back SpMV launches) computes the same
    acc_b = (c[0].real * X + c[0].imag * torch.stack([-X[:, 1], X[:, 0]], 1)).contiguous()
    Yb = torch.empty_like(Y)
    pl.run_baseline(X, Yb, Recurrence(alpha, None, gamma, coef, True, None, acc_b))
    torch.cuda.synchronize()
    assert torch.allclose(Yb, Y, rtol=1e-13, atol=1e-15)


def test_watchdog_path_recovers():
    # a tiny spin budget may abort a run (the kernel still exits normally);
    # the plan must report it and stay usable for the next run
    dev = _dev()
    A, _ = W.stencil_27pt_random(30, seed=9)
    x = W.uniform_vector(A.n, seed=9)
    ref = O.spmv_powers(A, x, 8)
    pl = Plan(A, 8, 1 << 20, tile_nnz=500, watchdog_spins=1)
    perm = pl.arrays()[0]
    X = torch.from_numpy(_to_plan(x, perm)).to(dev)
    Y = torch.empty((8, A.n), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    try:
        pl.status()
        check_powers(_unpermute_powers(Y.cpu().numpy(), perm), ref)
    except MpkError as e:
        assert e.status == -5
    # fresh plan with the default watchdog on the same data
    Y2, _ = run_mpk(A, x, 8, 1 << 20, tile_nnz=500)
    check_powers(Y2, ref)


def test_repeated_runs_reuse_flags():
    dev = _dev()
    A, _ = W.stencil_27pt_random(20, seed=11)
    pl = Plan(A, 6, 1 << 20, tile_nnz=900)
    perm = pl.arrays()[0]
    for s in range(4):
        x = W.uniform_vector(A.n, seed=s)
        ref = O.spmv_powers(A, x, 6)
        X = torch.from_numpy(_to_plan(x, perm)).to(dev)
        Y = torch.empty((6, A.n), dtype=torch.float64, device=dev)
        pl.run(X, Y)
        pl.status()
        check_powers(_unpermute_powers(Y.cpu().numpy(), perm), ref)


def test_run_argument_errors():
    dev = _dev()
    A = W.stencil_2d(8, 5)
    pl = Plan(A, 2, 4096, upload=False)
    X = torch.zeros(A.n, dtype=torch.float64, device=dev)
    Y = torch.zeros((2, A.n), dtype=torch.float64, device=dev)
    with pytest.raises(MpkError, match="MPK_ERR_STATE"):
        pl.run(X, Y)
    pl.upload()
    with pytest.raises(MpkError, match="MPK_ERR_ARG"):
        pl.run(Y[0], Y)  # X inside Y


@pytest.mark.parametrize("k", [1, 2, 4, 32])
def test_long_rows_and_chunk_edges(k):
    # rows longer than a chunk (one dense row, longer than the 4096-entry MPK
    # chunk of k = 1, and power-law rows) take the strided path; chunk
    # boundaries fall at every position
    rng = np.random.default_rng(k)
    n = 5000
    A = W.zipf_rows(n, 1.5, seed=k)
    dense = np.arange(n, dtype=np.int32)
    rowptr = np.concatenate([[0], A.rowptr[1:] - A.rowptr[1] + n]).astype(np.int64)
    col = np.concatenate([dense, A.col[A.rowptr[1]:]]).astype(np.int32)
    val = np.concatenate([rng.uniform(-1, 1, n) / n, A.val[A.rowptr[1]:]])
    B = W.CSR(n, rowptr, col, val)
    X = W.gaussian_block(B.n, k, seed=k) if k > 1 else W.uniform_vector(B.n, seed=k)
    ref = O.spmv_powers(B, X, 4)
    for tile in (500, 5000):
        Y, _ = run_mpk(B, X, 4, 1 << 18, nrhs=k, tile_nnz=tile, root_mode=1)
        check_powers(Y, ref)
    Yb, _ = run_mpk(B, X, 4, 1 << 18, nrhs=k, baseline=True)
    check_powers(Yb, ref)


def test_retune_then_run():
    dev = _dev()
    A, _ = W.stencil_27pt_random(18, seed=12)
    x = W.uniform_vector(A.n, seed=12)
    pl = Plan(A, 4, 1 << 20, root_mode=1)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    for p, C, kw in [(8, 1 << 19, {"skew": 2, "tile_nnz": 1200}), (3, 1 << 22, {"val_dtype": "f32"}),
                     (6, 1 << 20, {"workgroups": 40})]:
        pl.retune(p, C, root_mode=1, **kw)
        Y = torch.full((p, A.n), float("nan"), dtype=torch.float64, device=dev)
        pl.run(X, Y)
        pl.status()
        out = _unpermute_powers(Y.cpu().numpy(), perm)
        if kw.get("val_dtype") == "f32":
            ref = O.spmv_powers_lowp(A, x, p, "f32")
            assert max(_rel_err(out[q], ref[q]) for q in range(p)) < 1e-5
        else:
            check_powers(out, O.spmv_powers(A, x, p))


@pytest.mark.parametrize("baseline", [False, True])
def test_chebyshev_propagator(baseline):
    from paper_2205_01598_amd.cheb import ChebPropagator

    dev = _dev()
    A = W.anderson_3d(12, seed=3)
    x = W.random_phase_state(A.n, seed=3)
    M, p, r_dt = 32, 8, 10.0
    c = O.cheb_coefficients(M, r_dt)
    ref1 = O.cheb_propagate(A, x, c)
    ref2 = O.cheb_propagate(A, ref1, c)
    pl = Plan(A, p, 1 << 20, nrhs=2, root_mode=1, tile_nnz=700, skew=2)
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator.schroedinger(pl, M, r_dt)
    assert np.allclose(prop.c, c, rtol=0, atol=1e-15)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    a1 = torch.empty_like(X)
    a2 = torch.empty_like(X)
    prop.step(X, a1, baseline=baseline)
    prop.step(a1, a2, baseline=baseline)
    pl.status()
    for a, ref in ((a1, ref1), (a2, ref2)):
        h = np.empty((A.n, 2))
        h[perm] = a.cpu().numpy()
        assert _rel_err(h, ref) <= 1e-12
    assert abs(np.linalg.norm(h) - 1.0) < 1e-10


@pytest.mark.parametrize("granularity", ["node", "wavefront"])
@pytest.mark.parametrize("case", ["c1_many_groups", "27pt_random", "irregular_k4", "bf16"])
def test_bulk_synchronous_variants(granularity, case):
    # the launch-per-node and launch-per-wavefront variants run the same chunks
    # with the same arithmetic as the persistent kernel: equal bit for bit,
    # and within the FP64 bar of the oracle
    dev = _dev()
    k, opts = 1, {}
    if case == "c1_many_groups":
        A, p, C = W.stencil_2d(64, 5), 4, 16 * 1024
        opts = {"tile_nnz": 300}
    elif case == "27pt_random":
        A, p, C = W.stencil_27pt_random(20, seed=3)[0], 6, 3 << 20
        opts = {"root_mode": 1, "tile_nnz": 2000}
    elif case == "irregular_k4":
        A, p, C, k = W.zipf_rows(3000, 2.0, seed=5), 5, 1 << 18, 4
        opts = {"nrhs": 4, "tile_nnz": 200}
    else:
        A, p, C = W.stencil_27pt_random(16, seed=4)[0], 4, 1 << 20
        opts = {"val_dtype": "bf16"}
    pl = Plan(A, p, C, **opts)
    assert pl.info()["n_groups"] > 1
    perm = pl.arrays()[0]
    x = np.random.default_rng(11).uniform(-1, 1, (A.n, k)) if k > 1 else W.uniform_vector(A.n, seed=11)
    X = torch.from_numpy(np.ascontiguousarray(_to_plan(x, perm))).to(dev)
    Y1 = torch.full((p,) + tuple(X.shape), float("nan"), dtype=torch.float64, device=dev)
    Y2 = torch.full_like(Y1, float("nan"))
    pl.run(X, Y1)
    pl.status()
    pl.run_sync(X, Y2, granularity)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    if case != "bf16":
        ref = O.spmv_powers(A, x, p)
        Y = _unpermute_powers(Y2.cpu().numpy(), perm)
        check_powers(Y.reshape(ref.shape), ref)


def test_bulk_synchronous_rejects_bad_granularity():
    dev = _dev()
    A = W.stencil_2d(16, 5)
    pl = Plan(A, 3, 1 << 16)
    X = torch.zeros(A.n, dtype=torch.float64, device=dev)
    Y = torch.zeros((3, A.n), dtype=torch.float64, device=dev)
    from paper_2205_01598_amd import lib
    import ctypes
    st = lib().mpk_run_sync(pl._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), 7, None)
    assert st == -1


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("baseline", [False, True])
def test_heat_propagator(order, baseline):
    # heat equation with real modified-Bessel coefficients; the accumulator is
    # NaN-poisoned: the first power must start the sum (coef0), not add to it
    from paper_2205_01598_amd.cheb import ChebPropagator, heat_coefficients

    dev = _dev()
    A, r = W.heat_operator_3d(12, order)
    x = W.uniform_vector(A.n, seed=order)
    M, p, tau = 16, 8, 9.0
    c = O.heat_coefficients(M, tau)
    assert np.allclose(heat_coefficients(M, tau), c, rtol=1e-13, atol=1e-16)
    ref1 = O.cheb_propagate_real(A, x, c)
    ref2 = O.cheb_propagate_real(A, ref1, c)
    pl = Plan(A, p, 1 << 18, root_mode=1, tile_nnz=900, skew=2)
    assert pl.info()["n_groups"] > 1
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator.heat(pl, M, tau)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    a1 = torch.full_like(X, float("nan"))
    a2 = torch.full_like(X, float("nan"))
    prop.step(X, a1, baseline=baseline)
    prop.step(a1, a2, baseline=baseline)
    pl.status()
    for a, ref in ((a1, ref1), (a2, ref2)):
        h = np.empty(A.n)
        h[perm] = a.cpu().numpy()
        assert _rel_err(h, ref) <= 1e-12


@pytest.mark.parametrize("case", ["27pt_k1", "zipf_k4", "27pt_k2_rec", "misaligned_y"])
def test_line_closed_runs_without_fence(case):
    # with line-closed dependency ranges mpk_run skips the acquire fence; the
    # results must equal the fenced run bit for bit and meet the oracle bar.
    # A Y that is not 128-byte aligned makes the run fall back to the fence.
    dev = _dev()
    k = {"27pt_k1": 1, "zipf_k4": 4, "27pt_k2_rec": 2, "misaligned_y": 1}[case]
    if case == "zipf_k4":
        A = W.zipf_rows(8192, 2.0, seed=7)
    else:
        A = W.stencil_27pt_random(32, seed=5)[0]
    p = 6
    opts = dict(root_mode=1, skew=2, tile_nnz=1200, nrhs=k)
    pl = Plan(A, p, 2 << 20, **opts)
    pf = Plan(A, p, 2 << 20, force_acquire=1, **opts)
    assert pl.info()["line_closed_deps"] == 1 and pl.info()["n_groups"] > 2
    perm = pl.arrays()[0].astype(np.int64)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (A.n, k)) if k > 1 else rng.uniform(-1, 1, A.n)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    shape = (p,) + tuple(X.shape)
    if case == "misaligned_y":
        raw = torch.full((int(np.prod(shape)) + 1,), float("nan"), dtype=torch.float64, device=dev)
        Y1 = raw[1:].view(shape)
    else:
        Y1 = torch.full(shape, float("nan"), dtype=torch.float64, device=dev)
    Y2 = torch.full(shape, float("nan"), dtype=torch.float64, device=dev)
    if case == "27pt_k2_rec":
        alpha = np.array([1.0] + [2.0] * (p - 1))
        gamma = np.array([0.0] + [-1.0] * (p - 1))
        coef = rng.uniform(-1, 1, 2 * p)
        acc1 = torch.full_like(X, float("nan"))
        acc2 = torch.full_like(X, float("nan"))
        c0 = np.array([0.3, -0.2])
        pl.run(X, Y1, Recurrence(alpha, None, gamma, coef, True, None, acc1, coef0=c0))
        pf.run(X, Y2, Recurrence(alpha, None, gamma, coef, True, None, acc2, coef0=c0))
    else:
        pl.run(X, Y1)
        pf.run(X, Y2)
    pl.status()
    pf.status()
    assert pl.info()["last_run_fenced"] == (1 if case == "misaligned_y" else 0)
    assert pf.info()["last_run_fenced"] == 1
    assert torch.equal(Y1, Y2)
    if case == "27pt_k2_rec":
        assert torch.equal(acc1, acc2)
    else:
        ref = O.spmv_powers(A, x, p)
        check_powers(_unpermute_powers(Y1.cpu().numpy(), perm).reshape(ref.shape), ref)
    if case != "27pt_k2_rec":
        # repeated runs reuse the epoch-stamped flags and give the same bits
        for _ in range(3):
            Y1.fill_(float("nan"))
            pl.run(X, Y1)
            pl.status()
            assert torch.equal(Y1, Y2)


@pytest.mark.parametrize("p,M", [(1, 8), (2, 9), (3, 32), (8, 30)])
@pytest.mark.parametrize("kind", ["heat", "schroedinger"])
def test_chebyshev_p1_and_remainder_block(p, M, kind):
    # Sec. 5 / Sec. 7: degree M as floor(M/p) blocks of p and one block of
    # M mod p powers on the same plan (mpk_run_first); p = 1 carries the older
    # recurrence vector from the previous block's input
    from paper_2205_01598_amd.cheb import ChebPropagator

    dev = _dev()
    if kind == "heat":
        A, _ = W.heat_operator_3d(10, 2)
        x = W.uniform_vector(A.n, seed=5)
        c = O.heat_coefficients(M, 4.0)
        ref = O.cheb_propagate_real(A, x, c)
        pl = Plan(A, p, 1 << 18, root_mode=1, tile_nnz=500, skew=2)
    else:
        A = W.anderson_3d(10, seed=5)
        x = W.random_phase_state(A.n, seed=5)
        c = O.cheb_coefficients(M, 6.0)
        ref = O.cheb_propagate(A, x, c)
        pl = Plan(A, p, 1 << 18, root_mode=1, nrhs=2, tile_nnz=500, skew=2)
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator(pl, c)
    assert [n for _, n in prop.blocks] == [p] * (M // p) + ([M % p] if M % p else [])
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    for baseline in (False, True):
        acc = torch.full_like(X, float("nan"))
        prop.step(X, acc, baseline=baseline)
        pl.status()
        h = np.empty(x.shape)
        h[perm] = acc.cpu().numpy()
        assert _rel_err(h, ref) <= 1e-12, f"baseline={baseline}"


def test_run_rejects_overlapping_buffers():
    # mpk_run: Y must not overlap X, y_prev or acc; acc must not overlap X or
    # y_prev (the kernels read them while other tiles write)
    dev = _dev()
    A = W.stencil_2d(16, 5)
    pl = Plan(A, 3, 1 << 16, nrhs=1)
    n = A.n
    buf = torch.zeros(8 * n, dtype=torch.float64, device=dev)
    X, Y = buf[:n], buf[n:4 * n]
    pl.run(X, Y)  # disjoint: fine
    pl.status()
    with pytest.raises(MpkError, match="Y overlaps X"):
        pl.run(buf[:n], buf[n // 2:n // 2 + 3 * n])
    rec = lambda **kw: Recurrence(np.ones(3), gamma=np.array([1.0, 0, 0]), coef=np.ones(3), **kw)  # noqa: E731
    with pytest.raises(MpkError, match="Y overlaps y_prev"):
        pl.run(X, Y, rec(y_prev=buf[2 * n:3 * n], acc=buf[5 * n:6 * n]))
    with pytest.raises(MpkError, match="Y overlaps acc"):
        pl.run(X, Y, rec(y_prev=buf[4 * n:5 * n], acc=buf[3 * n:4 * n]))
    with pytest.raises(MpkError, match="acc overlaps X"):
        pl.run(X, Y, rec(y_prev=buf[4 * n:5 * n], acc=buf[:n]))
    with pytest.raises(MpkError, match="acc overlaps y_prev"):
        pl.run(X, Y, rec(y_prev=buf[4 * n:5 * n], acc=buf[4 * n:5 * n]))
    with pytest.raises(MpkError, match="Y overlaps y_prev"):
        pl.run_baseline(X, Y, rec(y_prev=buf[3 * n:4 * n], acc=buf[5 * n:6 * n]))
    # a valid recurrence run on the same buffers
    pl.run(X, Y, rec(y_prev=buf[4 * n:5 * n], acc=buf[5 * n:6 * n]))
    pl.status()

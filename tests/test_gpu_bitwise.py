"""GPU parity bit for bit.

The MPK (Sec. 3) is p plain SpMVs; level blocking only reorders whole-row
products (Sec. 4.2).  Every row of the kernel is summed by one thread in the
stored order of the renumbered matrix, starting from zero, with each product
rounded before it is added, which is exactly what the oracle does when it is
run on the same renumbered matrix P A P^T (oracle.permute_symmetric with the
plan's permutation) and the permuted input.  The results must therefore be
equal bit for bit:

* FP64 values: oracle.spmv_powers on P A P^T;
* FP32 / BF16 storage with FP32 arithmetic: oracle.spmv_powers_lowp on P A P^T
  (x rounded to FP32, products rounded to FP32, FP32 running sum);
* FP32 / BF16 storage with FP64 arithmetic (accum_f64): oracle.spmv_powers on
  the rounded values of P A P^T.

Rows longer than one chunk (MPK: 4096 stored entries at k = 1, 1024 at
k = 2, 4096/k for k >= 4; baseline SpMV: 3072 at k = 1, 2048 at k = 2 with
FP32 products, otherwise the same)
are reduced by a tree and are not covered here; none of these matrices has
one.  The recurrence
epilogue (Chebyshev) keeps its 1e-12 bar in the other tests."""
import numpy as np
import pytest

import fuzz_cases
import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import Plan  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def plan_order_oracle(A, perm, xp, p, dtype="f64", accum_f64=0):
    """The oracle on the renumbered matrix and the permuted input."""
    rp, col, val = O.permute_symmetric(A, perm)
    B = W.CSR(A.n, rp, col, val)
    if dtype == "f64":
        return O.spmv_powers(B, xp, p)
    if accum_f64:
        return O.spmv_powers(O.round_values(B, dtype), xp, p)
    return O.spmv_powers_lowp(B, xp, p, dtype)


def run_both(pl, xp, p):
    dev = _dev()
    X = torch.from_numpy(np.ascontiguousarray(xp)).to(dev)
    Y = torch.full((p,) + tuple(X.shape), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    Ym = Y.cpu().numpy()
    Y.fill_(float("nan"))
    pl.run_baseline(X, Y)
    torch.cuda.synchronize()
    return Ym, Y.cpu().numpy()


def assert_bitwise(Y, ref, label):
    for q in range(ref.shape[0]):
        if not np.array_equal(Y[q], ref[q]):
            bad = np.flatnonzero((Y[q] != ref[q]).ravel())
            raise AssertionError(f"{label} power {q + 1}: {len(bad)} entries differ, first at {bad[0]}: "
                                 f"{Y[q].ravel()[bad[0]]!r} vs {ref[q].ravel()[bad[0]]!r}")


@pytest.mark.parametrize("seed", range(fuzz_cases.N_CASES))
def test_fuzz_bitwise(seed):
    A, p, C, opts, x = fuzz_cases.case(seed)
    print(f"fuzz case {seed}: n={A.n} nnz={A.nnz} p={p} C={C} {opts}", flush=True)
    pl = Plan(A, p, C, **opts)
    perm = pl.arrays()[0]
    xp = np.ascontiguousarray(x[perm.astype(np.int64)])
    ref = plan_order_oracle(A, perm, xp, p, opts.get("val_dtype", "f64"), opts.get("accum_f64", 0))
    Ym, Yb = run_both(pl, xp, p)
    assert_bitwise(Ym, ref, "mpk")
    assert_bitwise(Yb, ref, "baseline")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("seed", range(4))
def test_fp32_arithmetic_bitwise(dtype, k, seed):
    # the mixed-precision definition (FP32 arithmetic) on irregular and
    # stencil matrices, several tiles, skews and budgets
    rng = np.random.default_rng(900 + seed)
    if seed % 2:
        A, _ = W.stencil_27pt_random(int(rng.integers(6, 14)), seed=seed)
    else:
        A = W.random_small_csr(int(rng.integers(200, 3000)), 8.0 / 2000, rng, symmetric_pattern=False,
                               empty_rows=0.05, duplicates=0.05)
    p = int(rng.integers(2, 9))
    x = rng.uniform(-1, 1, (A.n, k)) if k > 1 else rng.uniform(-1, 1, A.n)
    pl = Plan(A, p, int(rng.integers(1 << 14, 1 << 22)), root_mode=int(seed % 2), nrhs=k, val_dtype=dtype,
              skew=int(rng.integers(1, 5)), tile_nnz=int(rng.integers(64, 4000)))
    perm = pl.arrays()[0]
    xp = np.ascontiguousarray(x[perm.astype(np.int64)])
    ref = plan_order_oracle(A, perm, xp, p, dtype)
    Ym, Yb = run_both(pl, xp, p)
    assert_bitwise(Ym, ref, f"mpk {dtype}")
    assert_bitwise(Yb, ref, f"baseline {dtype}")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fp32_arithmetic_ieee_pins(dtype):
    # the exact cases that fix the oracle's mixed-precision steps, on the GPU:
    # FP32 running sum, x rounded to FP32, products rounded before the add
    t = 2.0 ** -24
    cases = [(np.array([1.0] + [t] * 8), np.zeros(9, np.int32), np.ones(1), 1.0),
             (np.array([3.0]), np.zeros(1, np.int32), np.array([1.0 + t]), 3.0)]
    if dtype == "f32":
        a = 1.0 + 2.0 ** -12
        cases.append((np.array([-1.0, a]), np.array([1, 0], np.int32), np.array([a, 1.0]), 2.0 ** -11))
    else:
        cases.append((np.array([-1.0, 1.0 + 2.0 ** -7]), np.array([1, 0], np.int32),
                      np.array([1.0 + 2.0 ** -17, 1.0]), 2.0 ** -7 + 2.0 ** -17))
    for val, col, x, want in cases:
        n = len(x)
        rp = np.zeros(n + 1, np.int64)
        rp[1:] = len(val)
        A = W.CSR(n, rp, col, val)
        pl = Plan(A, 1, 1 << 20, val_dtype=dtype)
        perm = pl.arrays()[0].astype(np.int64)
        Ym, Yb = run_both(pl, x[perm], 1)
        row0 = int(np.flatnonzero(perm == 0)[0])
        assert Ym[0][row0] == want and Yb[0][row0] == want


@pytest.fixture(scope="module")
def c27_plan_order():
    _dev()
    A, _ = W.stencil_27pt_random(160, seed=0)
    x = W.uniform_vector(A.n, seed=0)
    pl = Plan(A, 8, 256 << 20, root_mode=1, skew=2, tile_nnz=8192)
    perm = pl.arrays()[0]
    rp, col, val = O.permute_symmetric(A, perm)
    print(f"27-point 160^3 renumbered: n={A.n} nnz={A.nnz}", flush=True)
    return A, W.CSR(A.n, rp, col, val), pl, np.ascontiguousarray(x[perm.astype(np.int64)])


def test_27pt_160_p8_bitwise(c27_plan_order):
    # the benchmark's headline configuration (skew 2, C = 256 MB, 8192-nonzero
    # tiles), then p = 4 and 6 in theirs
    A, B, pl, xp = c27_plan_order
    ref = O.spmv_powers(B, xp, 8)
    Ym, Yb = run_both(pl, xp, 8)
    assert_bitwise(Ym, ref, "mpk p=8")
    assert_bitwise(Yb, ref, "baseline p=8")
    for p, tile in ((4, 6144), (6, 8192)):
        pl.retune(p, 256 << 20, root_mode=1, skew=2, tile_nnz=tile)
        Ym, _ = run_both(pl, xp, p)
        assert_bitwise(Ym, ref[:p], f"mpk p={p}")
    pl.retune(8, 256 << 20, root_mode=1, skew=2, tile_nnz=8192)


@pytest.mark.parametrize("dtype,accum_f64", [("f32", 0), ("bf16", 0), ("f32", 1), ("bf16", 1)])
def test_27pt_160_p8_mixed_bitwise(c27_plan_order, dtype, accum_f64):
    # the benchmark's mixed-precision runs: FP32 / BF16 storage with FP32 and
    # with FP64 arithmetic, p = 8, against the oracle's definition of each
    A, B, pl, xp = c27_plan_order
    if accum_f64:
        ref = O.spmv_powers(O.round_values(B, dtype), xp, 8)
    else:
        ref = O.spmv_powers_lowp(B, xp, 8, dtype)
    for tile in (8192, 16384):
        pl.retune(8, 256 << 20, root_mode=1, skew=2, tile_nnz=tile, val_dtype=dtype, accum_f64=accum_f64)
        Ym, Yb = run_both(pl, xp, 8)
        assert_bitwise(Ym, ref, f"mpk {dtype} acc64={accum_f64} tile={tile}")
        assert_bitwise(Yb, ref, f"baseline {dtype} acc64={accum_f64}")
    pl.retune(8, 256 << 20, root_mode=1, skew=2, tile_nnz=8192)


@pytest.mark.parametrize("powers", [1, 3, 5])
def test_first_powers_bitwise(powers):
    # mpk_run_first / mpk_run_baseline_first: the first `powers` powers of a
    # p = 6 plan, equal bit for bit to the oracle's; the tickets of the higher
    # powers are skipped, and the rows of Y past the run are not written
    A, _ = W.stencil_27pt_random(14, seed=4)
    x = W.uniform_vector(A.n, seed=4)
    pl = Plan(A, 6, 1 << 20, root_mode=1, skew=2, tile_nnz=1500)
    perm = pl.arrays()[0]
    xp = np.ascontiguousarray(x[perm.astype(np.int64)])
    ref = plan_order_oracle(A, perm, xp, powers)
    dev = _dev()
    X = torch.from_numpy(xp).to(dev)
    for base in (False, True):
        Y = torch.full((6, A.n), float("nan"), dtype=torch.float64, device=dev)
        (pl.run_baseline if base else pl.run)(X, Y, powers=powers)
        pl.status()
        Yh = Y.cpu().numpy()
        assert_bitwise(Yh[:powers], ref, f"first {powers} baseline={base}")
        assert np.isnan(Yh[powers:]).all()
    # a full run afterwards still computes every power
    Y = torch.full((6, A.n), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    assert_bitwise(Y.cpu().numpy(), plan_order_oracle(A, perm, xp, 6), "full run after a partial one")

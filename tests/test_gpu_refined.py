"""GPU parity of refined plans (recursive level refinement, Sec. 4.4): the
persistent kernel with per-tile dependency lists against the oracle, at the
FP64 bar of the other parity tests (relative error <= 1e-12 per power), and
bit for bit on integer inputs."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import MpkError, Plan  # noqa: E402

TOL = 1e-12


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _run(pl, x, p, k=1, misalign=False):
    dev = _dev()
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    shape = (p,) + tuple(X.shape)
    if misalign:
        raw = torch.full((int(np.prod(shape)) + 1,), float("nan"), dtype=torch.float64, device=dev)
        Y = raw[1:].view(shape)
    else:
        Y = torch.full(shape, float("nan"), dtype=torch.float64, device=dev)
    print(f"refined run: n={pl.info()['n']} p={p} k={k} tiles={pl.info()['n_tiles']}", flush=True)
    pl.run(X, Y)
    pl.status()
    torch.cuda.synchronize()
    out = np.empty((p,) + x.shape)
    out[:, perm] = Y.cpu().numpy().reshape((p,) + x.shape)
    return out


def _case(name):
    if name == "2d5pt":
        return W.stencil_2d(40, 5), 4, 6000, dict(tile_nnz=256)
    if name == "27pt":
        return W.stencil_27pt_random(12, seed=3)[0], 3, 40000, dict(tile_nnz=256)
    if name == "rgg":
        return W.random_geometric(3000, 10.0, seed=2)[0], 2, 3000, dict(tile_nnz=256)
    if name == "banded":
        return W.banded_random(2500, 40, seed=4), 3, 4000, dict(tile_nnz=256)
    if name == "irregular":
        rng = np.random.default_rng(7)
        return W.random_small_csr(600, 0.008, rng, empty_rows=0.05, duplicates=0.05), 2, 900, dict(tile_nnz=64)
    if name == "27pt_p8_s2":
        return W.stencil_27pt_random(24, seed=1)[0], 8, 120000, dict(recursion_stages=2, skew=2)
    raise KeyError(name)


@pytest.mark.parametrize("case", ["2d5pt", "27pt", "rgg", "banded", "irregular", "27pt_p8_s2"])
def test_refined_matches_oracle(case):
    A, p, C, opts = _case(case)
    opts = dict(opts)
    opts.setdefault("recursion_stages", 1)
    pl = Plan(A, p, C, root_mode=1, **opts)
    inf = pl.info()
    assert inf["recursive"] == 1 and inf["max_stage"] >= 1
    x = W.uniform_vector(A.n, seed=11)
    ref = O.spmv_powers(A, x, p)
    Y = _run(pl, x, p)
    # the fence is skipped exactly when every power slice starts on a line
    assert pl.info()["last_run_fenced"] == (0 if (A.n * 8) % 128 == 0 else 1)
    for q in range(p):
        e = _rel_err(Y[q], ref[q])
        assert e <= TOL, f"power {q + 1}: rel err {e:.3e}"


@pytest.mark.parametrize("case", ["27pt_p8_s2", "rgg"])
@pytest.mark.parametrize("wg", [0, 40])
def test_refined_xcd_streams_equal_single_stream(case, wg):
    # eight ticket streams (workgroup b serves stream b % 8) give the same
    # results as one stream, bit for bit
    A, p, C, opts = _case(case)
    opts = dict(opts)
    opts.setdefault("recursion_stages", 1)
    one = Plan(A, p, C, root_mode=1, workgroups=wg, **opts)
    eight = Plan(A, p, C, root_mode=1, workgroups=wg, xcd_streams=8, **opts)
    assert eight.info()["recursive"] == 1
    x = W.uniform_vector(A.n, seed=13)
    y8 = _run(eight, x, p)
    assert np.array_equal(y8, _run(one, x, p))
    ref = O.spmv_powers(A, x, p)
    for q in range(p):
        assert _rel_err(y8[q], ref[q]) <= TOL


def test_refined_integer_bit_exact_and_fenced():
    A = W.integer_stencil_27pt(20, seed=5)
    rng = np.random.default_rng(5)
    x = rng.integers(-1, 2, size=A.n).astype(np.float64)
    p = 8
    ref = O.spmv_powers(A, x, p)
    pl = Plan(A, p, 200000, root_mode=1, recursion_stages=2, tile_nnz=1500)
    assert pl.info()["max_stage"] >= 1
    assert np.array_equal(_run(pl, x, p), ref)
    # a Y that is not 128-byte aligned makes the run use the acquire fence
    assert np.array_equal(_run(pl, x, p, misalign=True), ref)
    assert pl.info()["last_run_fenced"] == 1
    # repeated runs reuse the epoch-stamped flags
    for _ in range(2):
        assert np.array_equal(_run(pl, x, p), ref)


@pytest.mark.parametrize("k", [2, 4])
def test_refined_multi_rhs(k):
    A = W.stencil_27pt_random(16, seed=8)[0]
    p = 5
    pl = Plan(A, p, 50000, root_mode=1, recursion_stages=1, nrhs=k, tile_nnz=400)
    x = W.gaussian_block(A.n, k, seed=2)
    ref = O.spmv_powers(A, x, p)
    Y = _run(pl, x, p, k=k)
    for q in range(p):
        assert _rel_err(Y[q], ref[q]) <= TOL


def test_refined_chebyshev_propagator():
    from paper_2205_01598_amd.cheb import ChebPropagator

    dev = _dev()
    A = W.anderson_3d(12, seed=3)
    x = W.random_phase_state(A.n, seed=3)
    M, p, r_dt = 32, 8, 10.0
    ref = O.cheb_propagate(A, x, O.cheb_coefficients(M, r_dt))
    pl = Plan(A, p, 150000, nrhs=2, root_mode=1, recursion_stages=1, tile_nnz=700)
    assert pl.info()["max_stage"] >= 1
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator.schroedinger(pl, M, r_dt)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    a1 = torch.empty_like(X)
    prop.step(X, a1)
    pl.status()
    h = np.empty((A.n, 2))
    h[perm] = a1.cpu().numpy()
    assert _rel_err(h, ref) <= TOL


def test_refined_rejects_bulk_synchronous():
    dev = _dev()
    A, p, C, opts = _case("2d5pt")
    pl = Plan(A, p, C, recursion_stages=1, **opts)
    X = torch.zeros(A.n, dtype=torch.float64, device=dev)
    Y = torch.zeros((p, A.n), dtype=torch.float64, device=dev)
    with pytest.raises(MpkError):
        pl.run_sync(X, Y, "node")

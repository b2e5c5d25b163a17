"""GPU parity at the full benchmark sizes, in the launch configurations the
benchmark times, against the oracle computed in full (the plain C FP64
oracle; a few seconds each on one host thread):

* 27-point 160^3 (N = 4,096,000, nnz = 109,215,352), p = 8 with skew 2,
  C = 256 MB, 8192-nonzero tiles, then p = 4 and 6 after retuning;
* one degree-32 Chebyshev step on the Anderson 128^3 Hamiltonian
  (complex state as two columns, blocks of p = 8);
* the random geometric graph with N = 2M, p = 6, k = 4 in full and two of
  the k = 32 columns.

FP64 bar: relative 2-norm error <= 1e-12 per power (per step)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import Plan  # noqa: E402
from paper_2205_01598_amd.cheb import ChebPropagator  # noqa: E402

TOL = 1e-12


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check(Y, ref, label):
    for q in range(ref.shape[0]):
        e = np.linalg.norm(Y[q] - ref[q]) / np.linalg.norm(ref[q])
        assert e <= TOL, f"{label} power {q + 1}: rel err {e:.3e}"


@pytest.fixture(scope="module")
def c27():
    _dev()
    A, _ = W.stencil_27pt_random(160, seed=0)
    x = W.uniform_vector(A.n, seed=0)
    print(f"27-point 160^3: n={A.n} nnz={A.nnz}", flush=True)
    return A, x, O.spmv_powers(A, x, 8)


def test_27pt_160_p8_bench_configuration(c27):
    A, x, ref = c27
    dev = _dev()
    pl = Plan(A, 8, 256 << 20, root_mode=1, skew=2, tile_nnz=8192)
    inf = pl.info()
    assert inf["n_levels"] == 160 and inf["line_closed_deps"] == 1
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    Y = torch.full((8, A.n), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    assert pl.info()["last_run_fenced"] == 0
    out = np.empty((8, A.n))
    out[:, perm] = Y.cpu().numpy()
    _check(out, ref, "mpk p=8")
    # the baseline on the same plan
    Y.fill_(float("nan"))
    pl.run_baseline(X, Y)
    torch.cuda.synchronize()
    out[:, perm] = Y.cpu().numpy()
    _check(out, ref, "baseline p=8")
    # p = 4 and p = 6 in their benchmark configurations
    for p, tile in ((4, 6144), (6, 8192)):
        pl.retune(p, 256 << 20, root_mode=1, skew=2, tile_nnz=tile)
        Yp = torch.full((p, A.n), float("nan"), dtype=torch.float64, device=dev)
        pl.run(X, Yp)
        pl.status()
        outp = np.empty((p, A.n))
        outp[:, perm] = Yp.cpu().numpy()
        _check(outp, ref[:p], f"mpk p={p}")


def test_anderson_128_chebyshev_step():
    dev = _dev()
    A = W.anderson_3d(128, seed=0)
    x = W.random_phase_state(A.n, seed=0)
    M, p, r_dt = 32, 8, 10.0
    ref = O.cheb_propagate(A, x, O.cheb_coefficients(M, r_dt))
    pl = Plan(A, p, 128 << 20, root_mode=1, nrhs=2, skew=2, tile_nnz=4096)
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator.schroedinger(pl, M, r_dt)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    for C, tile in ((128, 4096), (256, 8192)):
        pl.retune(p, C << 20, root_mode=1, nrhs=2, skew=2, tile_nnz=tile)
        acc = torch.full_like(X, float("nan"))
        prop.step(X, acc)
        pl.status()
        h = np.empty((A.n, 2))
        h[perm] = acc.cpu().numpy()
        e = np.linalg.norm(h - ref) / np.linalg.norm(ref)
        assert e <= TOL, f"C={C} MB tile={tile}: rel err {e:.3e}"


def test_rgg_2m_multi_rhs():
    dev = _dev()
    A, _ = W.random_geometric(2_000_000, 16.0, seed=0)
    p = 6
    pl = Plan(A, p, 256 << 20, root_mode=1, nrhs=4, skew=2, tile_nnz=8192)
    perm = pl.arrays()[0].astype(np.int64)
    # k = 4 in full
    Xh = W.gaussian_block(A.n, 4, seed=4)
    ref = O.spmv_powers(A, Xh, p)
    X = torch.from_numpy(np.ascontiguousarray(Xh[perm])).to(dev)
    Y = torch.full((p, A.n, 4), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    out = np.empty((p, A.n, 4))
    out[:, perm] = Y.cpu().numpy()
    _check(out, ref, "k=4")
    # k = 32: the columns are independent; two of them against the oracle
    pl.retune(p, 256 << 20, root_mode=1, nrhs=32, skew=2, tile_nnz=2048)
    Xh = W.gaussian_block(A.n, 32, seed=32)
    X = torch.from_numpy(np.ascontiguousarray(Xh[perm])).to(dev)
    Y = torch.full((p, A.n, 32), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    Yh = Y.cpu().numpy()
    for c in (0, 31):
        ref = O.spmv_powers(A, np.ascontiguousarray(Xh[:, c]), p)
        out = np.empty((p, A.n))
        out[:, perm] = Yh[:, :, c]
        _check(out, ref, f"k=32 column {c}")

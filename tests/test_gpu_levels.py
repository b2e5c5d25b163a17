"""Preprocessing on the GPU (plan_on_device = 1): graph, breadth-first
levels and the renumbered matrix.  The root, the permutation, the level
pointers, the groups, the schedule and P A P^T must equal the host
planner's bit for bit, and the levels the oracle's (Eq. 3, discovery order
inside a level, components started at the smallest unnumbered index).
Sorted symmetric patterns take the all-device path; the others build the
graph on the host and level it on the GPU."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2205_01598_amd import Plan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _direct_sum(*blocks):
    rps, cols, vals, off, base = [np.zeros(1, np.int64)], [], [], 0, 0
    for b in blocks:
        rps.append(b.rowptr[1:] + base)
        cols.append(b.col.astype(np.int64) + off)
        vals.append(b.val)
        off += b.n
        base += b.nnz
    return W.CSR(off, np.concatenate(rps), np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def _cases():
    yield "worked_example", W.stencil_2d(8, 7)
    yield "2d5pt_64", W.stencil_2d(64, 5)
    yield "27pt_random_24", W.stencil_27pt_random(24, seed=2)[0]
    Z = W.zipf_rows(20000, 1.8, seed=4)
    S, _ = W.stencil_27pt_random(14, seed=6)
    iso = W.CSR(40, np.arange(41, dtype=np.int64), np.arange(40, dtype=np.int32), np.ones(40))
    U = _direct_sum(S, Z, iso)
    yield "unsym_components", W.relabel(U, np.random.default_rng(9).permutation(U.n))
    yield "rgg", W.random_geometric(6000, 12.0, seed=1)[0]
    yield "banded", W.banded_random(5000, 30, seed=2)
    rng = np.random.default_rng(5)
    yield "irregular", W.random_small_csr(300, 0.01, rng, symmetric_pattern=False, empty_rows=0.2, duplicates=0.1)
    yield "single", W.CSR(1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([2.0]))
    # arrow: one full row and column, so one renumbered row exceeds the
    # device sort length and is sorted on the host
    n = 1500
    rows = np.concatenate([np.zeros(n, np.int64), np.arange(1, n), np.arange(1, n)])
    cols = np.concatenate([np.arange(n), np.zeros(n - 1, np.int64), np.arange(1, n)])
    order = np.lexsort((cols, rows))
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    Arw = W.CSR(n, np.cumsum(rp), cols[order].astype(np.int32), np.random.default_rng(1).uniform(-1, 1, len(rows)))
    yield "arrow", W.relabel(Arw, np.random.default_rng(2).permutation(n))
    yield "symmetric_duplicates", W.random_small_csr(400, 0.02, np.random.default_rng(7), symmetric_pattern=True,
                                                     empty_rows=0.1, duplicates=0.2)


@pytest.mark.parametrize("root_mode", [0, 1])
@pytest.mark.parametrize("name,A", list(_cases()), ids=[c[0] for c in _cases()])
def test_device_plan_matches_host_and_oracle(name, A, root_mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    host = Plan(A, 4, 1 << 20, upload=False, root_mode=root_mode)
    dev = Plan(A, 4, 1 << 20, upload=False, root_mode=root_mode, plan_on_device=1)
    assert dev.info()["root"] == host.info()["root"]
    for a, b in zip(dev.arrays(), host.arrays()):
        assert np.array_equal(a, b)
    for a, b in zip(dev.matrix(), host.matrix()):
        assert np.array_equal(a, b)
    perm, lp = O.bfs_levels(A, root_mode)
    assert np.array_equal(dev.arrays()[0], perm) and np.array_equal(dev.arrays()[1], lp)


def test_device_levels_large_and_run():
    # wide frontiers (up to 3i^2+3i+1 rows per level from a corner), then a
    # run on the plan built from the device levels
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, _ = W.stencil_27pt_random(48, seed=1)
    host = Plan(A, 6, 4 << 20, upload=False, root_mode=1)
    dev = Plan(A, 6, 4 << 20, root_mode=1, plan_on_device=1)
    for a, b in zip(dev.arrays(), host.arrays()):
        assert np.array_equal(a, b)
    perm = dev.arrays()[0].astype(np.int64)
    x = W.uniform_vector(A.n, seed=3)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to("cuda:0")
    Y = torch.empty((6, A.n), dtype=torch.float64, device="cuda:0")
    dev.run(X, Y)
    dev.status()
    ref = O.spmv_powers(A, x, 6)
    out = np.empty((6, A.n))
    out[:, perm] = Y.cpu().numpy()
    for q in range(6):
        assert np.linalg.norm(out[q] - ref[q]) <= 1e-12 * np.linalg.norm(ref[q])

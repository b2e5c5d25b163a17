"""Seeded input generators: the keyed sort equals the two-key lexicographic
sort it replaces, and the tuner corpus is the same whether it is generated
in the caller or ahead in worker processes."""
import numpy as np

from workloads import matrices as M


def test_row_major_order_equals_lexsort():
    rng = np.random.default_rng(3)
    for n in (1, 7, 1000):
        rows = rng.integers(0, n, size=5000)
        cols = rng.integers(0, n, size=5000)  # many repeated (row, col) pairs
        assert np.array_equal(M._row_major_order(rows, cols, n), np.lexsort((cols, rows)))
    e = np.zeros(0, np.int64)
    assert M._row_major_order(e, e, 0).size == 0


def test_generated_csr_is_row_sorted():
    for seed in range(10):
        A, spec = M.tuner_matrix(seed, 2e3, 2e4)
        rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
        key = rows * A.n + A.col.astype(np.int64)
        assert np.all(np.diff(key) > 0), spec  # sorted, no repeated entry


def test_corpus_workers_match_sequential():
    from paper_2205_01598_amd import tune

    a = list(tune._corpus(range(3), 2e3, 2e4, 0))
    b = list(tune._corpus(range(3), 2e3, 2e4, 2))
    assert [r[0] for r in a] == [r[0] for r in b] == [0, 1, 2]
    for (_, A, sa), (_, B, sb) in zip(a, b):
        assert sa == sb
        assert np.array_equal(A.rowptr, B.rowptr) and np.array_equal(A.col, B.col)
        assert np.array_equal(A.val, B.val)

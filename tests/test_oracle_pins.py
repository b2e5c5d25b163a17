"""Pins for the CPU oracle: each check ties the oracle to something other
than itself -- values the paper prints for its worked example, closed forms,
graph invariants, exact integer arithmetic, dense brute force and independent
library routines.  No GPU is needed."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle as O
import workloads as W
from conftest import read_golden


# ----------------------------------------------------------------------------
# levels (Eq. 3, Sec. 4.1)
# ----------------------------------------------------------------------------

def test_worked_example_levels():
    g = read_golden("worked_example_2d7pt_8x8.txt")
    A = W.stencil_2d(8, 7)
    perm, lp = O.bfs_levels(A, root_mode=0)
    assert len(lp) - 1 == int(g["n_levels"][0][0])
    assert lp.tolist() == [int(v) for v in g["level_ptr"][0]]
    lo, hi = (int(v) for v in g["level6"][0])
    assert (lp[6], lp[7] - 1) == (lo, hi)
    lo, hi = (int(v) for v in g["levels_5_to_7"][0])
    assert (lp[5], lp[8] - 1) == (lo, hi)
    # the renumbering is a bijection and the root comes first
    assert sorted(perm.tolist()) == list(range(64)) and perm[0] == 0


def test_stencil_orientation_matters():
    # with the main-diagonal pair (x+1, y+1), (x-1, y-1) instead of the
    # anti-diagonal pair, the 8x8 grid has Chebyshev-distance levels: 8 of
    # them, not the 15 of Fig. 4, so the example fixes the orientation.
    n = 8
    v = np.arange(n * n)
    x, y = v % n, v // n
    dx = x[None, :] - x[:, None]
    dy = y[None, :] - y[:, None]
    pat = ((np.abs(dx) + np.abs(dy) <= 1) | ((dx == dy) & (np.abs(dx) == 1)))
    M = sp.csr_matrix(pat.astype(float))
    Ac = W.CSR(n * n, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)
    assert Ac.nnz == W.stencil_2d(8, 7).nnz
    _, lp = O.bfs_levels(Ac, 0)
    assert len(lp) - 1 == 8


def test_levels_closed_form_2d5pt():
    n = 64
    A = W.stencil_2d(n, 5)
    perm, lp = O.bfs_levels(A, 0)
    assert len(lp) - 1 == 2 * n - 1
    lev = np.empty(n * n, np.int64)
    for i in range(len(lp) - 1):
        lev[perm[lp[i]:lp[i + 1]]] = i
    v = np.arange(n * n)
    assert np.array_equal(lev, (v % n) + (v // n))


@pytest.mark.parametrize("n", [6, 13])
def test_levels_closed_form_27pt_corner(n):
    # 27-point stencil, random relabelling: the pseudo-peripheral root is a
    # corner and the levels are the shells max(x, y, z) = i of 3i^2+3i+1 points
    A, new2old = W.stencil_27pt_random(n, seed=3)
    perm, lp = O.bfs_levels(A, root_mode=1)
    assert len(lp) - 1 == n
    widths = np.diff(lp)
    i = np.arange(n)
    assert np.array_equal(widths, 3 * i * i + 3 * i + 1)
    g = new2old[perm.astype(np.int64)]  # natural grid index of each new row
    x, y, z = g % n, (g // n) % n, g // (n * n)
    root = (x[0], y[0], z[0])
    assert all(c in (0, n - 1) for c in root)
    cheb = np.maximum(np.maximum(np.abs(x - root[0]), np.abs(y - root[1])), np.abs(z - root[2]))
    lev = np.repeat(np.arange(n), widths)
    assert np.array_equal(cheb, lev)


def test_levels_closed_form_3d7pt():
    n = 9
    A = W.stencil_3d(n, 7)
    perm, lp = O.bfs_levels(A, 0)
    assert len(lp) - 1 == 3 * n - 2
    lev = np.repeat(np.arange(len(lp) - 1), np.diff(lp))
    g = perm.astype(np.int64)
    assert np.array_equal(lev, g % n + (g // n) % n + g // (n * n))


def _random_graphs():
    rng = np.random.default_rng(11)
    cases = []
    for n, dens, sym in [(1, 0.0, True), (2, 0.0, True), (7, 0.3, False), (40, 0.05, False),
                         (60, 0.02, True), (200, 0.01, False), (300, 0.004, True)]:
        cases.append(W.random_small_csr(n, dens, rng, symmetric_pattern=sym,
                                        empty_rows=0.05, duplicates=0.1))
    return cases


@pytest.mark.parametrize("A", _random_graphs())
@pytest.mark.parametrize("root_mode", [0, 1])
def test_levels_are_graph_distances(A, root_mode):
    perm, lp = O.bfs_levels(A, root_mode)
    n = A.n
    assert sorted(perm.tolist()) == list(range(n))
    assert np.all(np.diff(lp) > 0) and lp[0] == 0 and lp[-1] == n
    lev = np.empty(n, np.int64)
    lev[perm] = np.repeat(np.arange(len(lp) - 1), np.diff(lp))
    # scipy distances on the symmetrised pattern, independent of the oracle
    M = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(n, n))
    S = ((M + M.T) > 0).astype(float)
    S.setdiag(0)
    S.eliminate_zeros()
    root = perm[0]
    dist = shortest_path(S, unweighted=True, indices=[root])[0]
    comp = np.isfinite(dist)
    assert np.array_equal(lev[comp], dist[comp].astype(np.int64))
    # Eq. (4): every stored nonzero joins equal or adjacent levels
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    assert np.all(np.abs(lev[rows] - lev[A.col]) <= 1)
    # a level whose vertices have no neighbour in the level before starts a
    # new component: it is one vertex, the smallest index not yet numbered
    Sc = S.tocsr()
    for i in range(1, len(lp) - 1):
        lvl = perm[lp[i]:lp[i + 1]]
        prev = set(perm[lp[i - 1]:lp[i]].tolist())
        linked = any(int(u) in prev for v in lvl for u in Sc.indices[Sc.indptr[v]:Sc.indptr[v + 1]])
        if not linked:
            assert len(lvl) == 1 and lvl[0] == perm[lp[i]:].min()


def test_within_level_order_is_discovery_order():
    rng = np.random.default_rng(5)
    A = W.random_small_csr(120, 0.03, rng, symmetric_pattern=True)
    perm, lp = O.bfs_levels(A, 0)
    n = A.n
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    nb = [set() for _ in range(n)]
    for r in range(n):
        for c in A.col[A.rowptr[r]:A.rowptr[r + 1]]:
            if c != r:
                nb[r].add(int(c))
                nb[int(c)].add(r)
    for i in range(1, len(lp) - 1):
        prev = set(perm[lp[i - 1]:lp[i]].tolist())
        lvl = perm[lp[i]:lp[i + 1]].tolist()
        keys = []
        for v in lvl:
            ks = [pos[u] for u in nb[v] if u in prev]
            keys.append((min(ks) if ks else -1, v))
        if all(k[0] >= 0 for k in keys):
            assert keys == sorted(keys)


def test_peripheral_root_path_graph():
    n = 11
    r = np.arange(n - 1)
    M = sp.coo_matrix((np.ones(n - 1), (r, r + 1)), shape=(n, n)).tocsr()
    M = (M + M.T).tocsr()
    A = W.CSR(n, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)
    root = O.peripheral_root(A, 5)
    assert root in (0, n - 1)


# ----------------------------------------------------------------------------
# level groups (Eq. 5) and the Lp schedule (Fig. 6)
# ----------------------------------------------------------------------------

def test_group_example_six_vertex_cache():
    g = read_golden("level_groups_6vertex_cache.txt")
    sizes = np.array([1, 2, 3, 4, 5, 6, 7, 8, 7, 6, 5, 4, 3, 2, 1])
    # "at most six vertices": (p+1) * N * 12 < f*C with p = 1, f*C = 150
    gptr = O.level_groups(sizes, p=1, cache_bytes=300, f=0.5, bytes_per_nnz=12)
    groups = []
    for a, b in zip(gptr[:-1], gptr[1:]):
        groups.append(f"{a}-{b - 1}" if b - a > 1 else f"{a}")
    assert groups == g["groups"][0]
    viol = [i for i, (a, b) in enumerate(zip(gptr[:-1], gptr[1:])) if sizes[a:b].sum() > 6]
    assert viol == [int(v) for v in g["violators"][0]]


@pytest.mark.parametrize("p,C,f,b", [(1, 10_000, 0.5, 12), (4, 50_000, 0.5, 12),
                                     (8, 123_457, 0.37, 6), (2, 1, 0.5, 12)])
def test_group_invariants(p, C, f, b):
    rng = np.random.default_rng(p)
    lnnz = rng.integers(1, 400, size=57)
    gptr = O.level_groups(lnnz, p, C, f, b)
    budget = int(np.floor(f * C))
    assert gptr[0] == 0 and gptr[-1] == len(lnnz) and np.all(np.diff(gptr) >= 1)
    for a, bb in zip(gptr[:-1], gptr[1:]):
        tot = int(lnnz[a:bb].sum())
        ok = (p + 1) * tot * b < budget
        assert ok or bb - a == 1
        if bb < len(lnnz) and ok:
            assert not ((p + 1) * (tot + int(lnnz[bb])) * b < budget)


def test_schedule_worked_example():
    g = read_golden("lp_schedule_15x5.txt")
    s = O.lp_schedule(15, 5)
    assert len(s) == int(g["n_nodes"][0][0])
    step = {(int(i), int(q)): k for k, (d, q, i) in enumerate(s)}
    for i, q, k in g["step_of"]:
        assert step[(int(i), int(q))] == int(k)
    d, n = (int(v) for v in g["diag_size"][0])
    assert (s[:, 0] == d).sum() == n
    # steady-state reuse distance
    rd = int(g["reuse_distance"][0][0])
    assert step[(7, 3)] - step[(7, 2)] == rd
    # every node exactly once, and each node comes after its three
    # dependencies (i-1, p-1), (i, p-1), (i+1, p-1)
    assert len(step) == 75
    for (i, q), k in step.items():
        if q == 1:
            continue
        for j in (i - 1, i, i + 1):
            if 0 <= j < 15:
                assert step[(j, q - 1)] < k


@pytest.mark.parametrize("G,p", [(1, 1), (1, 6), (3, 8), (20, 4), (9, 9)])
def test_schedule_topological(G, p):
    s = O.lp_schedule(G, p)
    assert len(s) == G * p
    step = {(int(i), int(q)): k for k, (d, q, i) in enumerate(s)}
    assert len(step) == G * p
    for (i, q), k in step.items():
        for j in (i - 1, i, i + 1):
            if q > 1 and 0 <= j < G:
                assert step[(j, q - 1)] < k


# ----------------------------------------------------------------------------
# powers (Sec. 3.1)
# ----------------------------------------------------------------------------

def test_powers_2d5pt_eigenvectors():
    n = 64
    A = W.stencil_2d(n, 5)
    v = np.arange(n * n)
    x, y = v % n, v // n
    for (j, k) in [(1, 1), (3, 7), (64, 2)]:
        e = np.sin(j * np.pi * (x + 1) / (n + 1)) * np.sin(k * np.pi * (y + 1) / (n + 1))
        lam = 4 - 2 * np.cos(j * np.pi / (n + 1)) - 2 * np.cos(k * np.pi / (n + 1))
        Y = O.spmv_powers(A, e, 4)
        # rounding scale: |A|^p |e| (8^p |e| here); a dropped term or a wrong
        # sign would leave an O(1) relative error against it
        for p in range(1, 5):
            scale = 8.0 ** p * np.linalg.norm(e)
            assert np.linalg.norm(Y[p - 1] - lam ** p * e) <= 50 * p * 2.0 ** -52 * scale
            assert np.linalg.norm(Y[p - 1] - lam ** p * e) <= 1e-12 * max(lam ** p, 1.0) * np.linalg.norm(e) * 8 ** p


def test_powers_27pt_eigenvectors_permuted():
    n = 12
    A = W.stencil_3d(n, 27)
    rng = np.random.default_rng(0)
    new2old = rng.permutation(n ** 3)
    B = W.relabel(A, new2old)
    g = new2old
    x, y, z = g % n, (g // n) % n, g // (n * n)
    j = (2, 5, 11)
    e = (np.sin(j[0] * np.pi * (x + 1) / (n + 1)) * np.sin(j[1] * np.pi * (y + 1) / (n + 1))
         * np.sin(j[2] * np.pi * (z + 1) / (n + 1)))
    lam = 27 - np.prod([1 + 2 * np.cos(jj * np.pi / (n + 1)) for jj in j])
    Y = O.spmv_powers(B, e, 6)
    for p in range(1, 7):
        err = np.linalg.norm(Y[p - 1] - lam ** p * e) / np.linalg.norm(lam ** p * e)
        assert err < 1e-12


def test_powers_integer_exact():
    n = 6
    A = W.integer_stencil_27pt(n, seed=4)
    rng = np.random.default_rng(1)
    x = rng.integers(-1, 2, size=A.n).astype(np.float64)
    Y = O.spmv_powers(A, x, 8)
    D = A.to_dense().astype(np.int64)
    xi = x.astype(np.int64)
    for p in range(8):
        xi = D @ xi
        assert np.array_equal(Y[p], xi.astype(np.float64))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_powers_dense_brute_force(seed):
    rng = np.random.default_rng(seed)
    A = W.random_small_csr(150 + 50 * seed, 0.04, rng, empty_rows=0.1, duplicates=0.2)
    D = A.to_dense()
    x = rng.uniform(-1, 1, size=(A.n, 3))
    Y = O.spmv_powers(A, x, 5)
    for p in range(1, 6):
        ref = np.linalg.matrix_power(D, p) @ x
        assert np.allclose(Y[p - 1], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_powers_vs_scipy():
    A, _ = W.stencil_27pt_random(10, seed=9)
    M = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    x = W.uniform_vector(A.n, seed=9)
    Y = O.spmv_powers(A, x, 4)
    v = x
    for p in range(4):
        v = M @ v
        assert np.allclose(Y[p], v, rtol=1e-13, atol=0)


def test_powers_row_stochastic():
    A, _ = W.random_geometric(3000, 10.0, seed=2)
    assert np.allclose(np.bincount(np.repeat(np.arange(A.n), np.diff(A.rowptr)), A.val), 1.0)
    Y = O.spmv_powers(A, np.ones(A.n), 6)
    assert np.allclose(Y, 1.0, rtol=0, atol=1e-13)


def test_powers_empty_and_single():
    A = W.CSR(1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([3.0]))
    Y = O.spmv_powers(A, np.array([2.0]), 3)
    assert Y.ravel().tolist() == [6.0, 18.0, 54.0]
    Z = W.CSR(3, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert np.all(O.spmv_powers(Z, np.ones(3), 2) == 0)


# ----------------------------------------------------------------------------
# mixed precision definition
# ----------------------------------------------------------------------------

def test_lowp_exact_on_representable_integers():
    # entries in {-2..2} are exact in bf16 and f32; |A^4 x| < 2^24, so every
    # FP32 partial sum is exact and the low-precision powers equal FP64 ones
    A = W.integer_stencil_27pt(5, seed=8)
    rng = np.random.default_rng(3)
    x = rng.integers(-1, 2, size=A.n).astype(np.float64)
    ref = O.spmv_powers(A, x, 4)
    for dt in ("f32", "bf16"):
        assert np.array_equal(O.spmv_powers_lowp(A, x, 4, dt), ref)


def test_lowp_rounding_rules():
    # bf16 keeps 8 significant bits: 1 + 2^-8 is a tie and rounds to even (1);
    # 1 + 3*2^-8 rounds up to 1 + 2^-6; f32 rounds 1 + 2^-30 to 1
    vals = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -30])
    A = W.CSR(3, np.arange(4, dtype=np.int64), np.arange(3, dtype=np.int32), vals)
    yb = O.spmv_powers_lowp(A, np.ones(3), 1, "bf16")[0]
    yf = O.spmv_powers_lowp(A, np.ones(3), 1, "f32")[0]
    assert yb.tolist() == [1.0, 1 + 2.0 ** -6, 1.0]
    assert yf.tolist() == [float(np.float32(1 + 2.0 ** -8)), float(np.float32(1 + 3 * 2.0 ** -8)), 1.0]


# Exact IEEE cases that fix the three steps of the mixed-precision product
# (Sec. 3 extended by storage precision; readings in the oracle's header):
#   (a) an FP32 running sum: 1 followed by eight 2^-24 terms stays exactly 1
#       (each 1 + 2^-24 is a tie that rounds to even); an FP64 sum would give
#       1 + 2^-21;
#   (b) the input vector rounded to FP32 before the product: 3 * x with
#       x = 1 + 2^-24 rounds x to 1 and gives exactly 3; without that rounding
#       the FP32 product 3 + 3*2^-24 rounds to 3 + 2^-22;
#   (c) products rounded before the add, no fused multiply-add: -1 + a*x with
#       a = x = 1 + 2^-12 (FP32 storage) gives 2^-11, since the product
#       1 + 2^-11 + 2^-24 is a tie rounded to 1 + 2^-11, where a fused
#       multiply-add gives 2^-11 + 2^-24; with BF16 storage (8 significant
#       bits) a = 1 + 2^-7, x = 1 + 2^-17: 2^-7 + 2^-17 against
#       2^-7 + 2^-17 + 2^-24.
def _lowp_pin_cases():
    t = 2.0 ** -24
    both = ("f32", "bf16")
    cases = []
    A = W.CSR(1, np.array([0, 9], np.int64), np.zeros(9, np.int32), np.array([1.0] + [t] * 8))
    cases.append((A, np.ones(1), 1.0, both))
    A = W.CSR(1, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.array([3.0]))
    cases.append((A, np.array([1.0 + t]), 3.0, both))
    for a, xv, want, dts in ((1.0 + 2.0 ** -12, 1.0 + 2.0 ** -12, 2.0 ** -11, ("f32",)),
                             (1.0 + 2.0 ** -7, 1.0 + 2.0 ** -17, 2.0 ** -7 + 2.0 ** -17, both)):
        A = W.CSR(2, np.array([0, 2, 2], np.int64), np.array([1, 0], np.int32), np.array([-1.0, a]))
        cases.append((A, np.array([xv, 1.0]), want, dts))
    return cases


def _lowp_pins_hold(fn):
    """True iff ``fn(A, x, p, dtype)`` reproduces every pin exactly in the
    storage precisions it names."""
    for A, x, want, dts in _lowp_pin_cases():
        for dt in dts:
            if fn(A, x, 1, dt)[0][0] != want:
                return False
    return True


def test_lowp_ieee_pins():
    assert _lowp_pins_hold(O.spmv_powers_lowp)


def _lowp_mutant(sum64=False, round_x=True, fused=False):
    # plausible mistakes in a copy of the product definition (CPU only)
    def fn(A, x, p, dt):
        a = O.round_values(A, dt).val.astype(np.float32)
        y, v = [], np.asarray(x, np.float64)
        for _ in range(p):
            xin = v.astype(np.float32) if round_x else v
            out = np.empty(A.n)
            for r in range(A.n):
                s = np.float64(0) if sum64 else np.float32(0)
                for j in range(A.rowptr[r], A.rowptr[r + 1]):
                    if fused:
                        s = np.float32(np.float64(a[j]) * np.float64(xin[A.col[j]]) + np.float64(s))
                    elif sum64:
                        s = s + np.float64(np.float32(a[j] * xin[A.col[j]]))
                    else:
                        s = np.float32(s + np.float32(np.float64(a[j]) * np.float64(xin[A.col[j]])))
                out[r] = float(s)
            y.append(out)
            v = out
        return np.array(y)
    return fn


def test_lowp_pins_reject_planted_mistakes():
    # the faithful copy passes; each planted mistake fails at least one pin
    assert _lowp_pins_hold(_lowp_mutant())
    assert not _lowp_pins_hold(_lowp_mutant(sum64=True))
    assert not _lowp_pins_hold(_lowp_mutant(round_x=False))
    assert not _lowp_pins_hold(_lowp_mutant(fused=True))


def test_threaded_oracle_is_bit_identical():
    # Sec. 6 baseline: rows shared among threads, each row summed in stored order
    rng = np.random.default_rng(11)
    A = W.random_small_csr(3000, 6.0 / 3000, rng, symmetric_pattern=False, empty_rows=0.05, duplicates=0.05)
    for k in (1, 3):
        x = rng.uniform(-1, 1, (A.n, k)) if k > 1 else rng.uniform(-1, 1, A.n)
        ref = O.spmv_powers(A, x, 5)
        for t in (2, 3, 8):
            assert np.array_equal(O.spmv_powers(A, x, 5, threads=t), ref)


@pytest.mark.parametrize("seed", range(6))
def test_permute_symmetric_brute_force(seed):
    # (P A P^T)[i, j] = A[perm[i], perm[j]] on dense copies (duplicates summed),
    # columns ascending per row, duplicates in their stored order
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(1, 40))
    A = W.random_small_csr(n, float(rng.uniform(0.05, 0.4)), rng, symmetric_pattern=bool(seed % 2),
                           empty_rows=0.1, duplicates=0.2)
    perm = rng.permutation(n).astype(np.int32)
    rp, col, val = O.permute_symmetric(A, perm)
    B = np.zeros((n, n))
    for r in range(n):
        assert np.all(np.diff(col[rp[r]:rp[r + 1]]) >= 0)
        for j in range(rp[r], rp[r + 1]):
            B[r, col[j]] += val[j]
    D = A.to_dense()
    assert np.array_equal(B, D[np.ix_(perm, perm)])
    assert np.array_equal(np.diff(rp), np.diff(A.rowptr)[perm])
    # duplicate order: row 0 holds (1, 5.0), (0, 1.0), (1, 7.0); perm swaps 0 and 1
    E = W.CSR(2, np.array([0, 3, 3], np.int64), np.array([1, 0, 1], np.int32), np.array([5.0, 1.0, 7.0]))
    rp, col, val = O.permute_symmetric(E, np.array([1, 0], np.int32))
    assert rp.tolist() == [0, 0, 3] and col.tolist() == [0, 0, 1] and val.tolist() == [5.0, 7.0, 1.0]


def test_level_nnz_brute_force():
    # N_nz of every level (Eq. 5) counted entry by entry, and the closed form
    # of the path graph 0-1-...-(n-1) with diagonal from vertex 0: one vertex
    # per level, 2 stored entries at the ends and 3 inside
    rng = np.random.default_rng(21)
    A = W.random_small_csr(500, 0.01, rng, symmetric_pattern=True, empty_rows=0.1, duplicates=0.1)
    perm, lp = O.bfs_levels(A, 0)
    lvl = np.empty(A.n, np.int64)
    for i in range(len(lp) - 1):
        lvl[perm[lp[i]:lp[i + 1]]] = i
    count = np.zeros(len(lp) - 1, np.int64)
    for r in range(A.n):
        for _ in range(A.rowptr[r], A.rowptr[r + 1]):
            count[lvl[r]] += 1
    assert np.array_equal(O.level_nnz(A, perm, lp), count)
    n = 7
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    P = W.CSR(n, np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64),
              np.array(cols, np.int32), np.ones(len(cols)))
    perm, lp = O.bfs_levels(P, 0)
    assert O.level_nnz(P, perm, lp).tolist() == [2, 3, 3, 3, 3, 3, 2]


def test_round_values_nearest_even():
    # the worked ties of the rounding rules, then brute force: the BF16 value
    # is the nearer of the two BF16 neighbours of the FP32 value (ties to an
    # even last kept bit), and the FP32 value is numpy's conversion
    vals = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -30, -2.5, 0.0])
    A = W.CSR(5, np.arange(6, dtype=np.int64), np.arange(5, dtype=np.int32), vals)
    assert O.round_values(A, "bf16").val.tolist() == [1.0, 1 + 2.0 ** -6, 1.0, -2.5, 0.0]
    rng = np.random.default_rng(7)
    v = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-20, 20, 4000),
                        (1 + (2 * rng.integers(0, 128, 500) + 1) * 2.0 ** -8) * 2.0 ** rng.integers(-10, 10, 500)])
    n = len(v)
    B = W.CSR(n, np.arange(n + 1, dtype=np.int64), np.zeros(n, dtype=np.int32), v)
    f32 = O.round_values(B, "f32").val
    assert np.array_equal(f32, v.astype(np.float32).astype(np.float64))
    bf = O.round_values(B, "bf16").val
    bits = f32.astype(np.float32).view(np.uint32)
    lo = (bits & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    hi = ((bits & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    dlo, dhi = np.abs(f32 - lo), np.abs(hi - f32)
    even_lo = ((bits >> np.uint32(16)) & np.uint32(1)) == 0
    want = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(even_lo, lo, hi)))
    assert np.array_equal(bf, want)
    assert np.sum(dlo == dhi) >= 400  # the tie cases were exercised


def test_round_values_matches_lowp_on_exact_data():
    # small integers: every rounding and every FP32 sum is exact, so the
    # FP32-arithmetic product and FP64 arithmetic on the rounded values agree
    A = W.integer_stencil_27pt(6, seed=2)
    x = np.random.default_rng(2).integers(-1, 2, A.n).astype(np.float64)
    for dt in ("f32", "bf16"):
        assert np.array_equal(O.spmv_powers(O.round_values(A, dt), x, 3), O.spmv_powers_lowp(A, x, 3, dt))


def test_lowp_error_within_bound():
    A, _ = W.stencil_27pt_random(8, seed=1)
    x = W.uniform_vector(A.n, seed=1)
    ref = O.spmv_powers(A, x, 3)
    absA = W.CSR(A.n, A.rowptr, A.col, np.abs(A.val))
    for dt, u in (("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        y = O.spmv_powers_lowp(A, x, 3, dt)
        bound = O.spmv_powers(absA, np.abs(x), 3)
        for p in range(3):
            # first-order bound: each power adds <= (u_val + (nrow+1) 2^-24) |A||y|
            c = (p + 1) * (u + 30 * 2.0 ** -24) * 1.01
            assert np.all(np.abs(y[p] - ref[p]) <= c * bound[p] + 1e-300)


# ----------------------------------------------------------------------------
# Chebyshev (Sec. 7)
# ----------------------------------------------------------------------------

def test_cheb_coefficients_scalar_identity():
    tau = 10.0
    c = O.cheb_coefficients(40, tau)
    th = np.linspace(0, np.pi, 17)
    T = np.cos(np.outer(np.arange(41), th))
    approx = (c[:, None] * T).sum(0)
    assert np.allclose(approx, np.exp(-1j * tau * np.cos(th)), atol=1e-12)


def test_cheb_propagate_vs_expm():
    from scipy.linalg import expm
    A = W.anderson_3d(6, seed=2)
    D = A.to_dense()
    x = W.random_phase_state(A.n, seed=2)
    tau = 10.0
    c = O.cheb_coefficients(40, tau)
    out = O.cheb_propagate(A, x, c)
    ref = expm(-1j * tau * D) @ (x[:, 0] + 1j * x[:, 1])
    assert np.allclose(out[:, 0] + 1j * out[:, 1], ref, atol=1e-11)
    assert abs(np.linalg.norm(out) - 1.0) < 1e-11


def test_cheb_truncation_tail():
    # degree 32 at r*dt = 10: every dropped |c_k| is below 1e-4 (the paper's
    # cut-off) and the truncated propagator stays unitary to ~1e-12
    from scipy.special import jv
    assert 2 * abs(jv(32, 10.0)) < 1e-12
    A = W.anderson_3d(5, seed=1)
    x = W.random_phase_state(A.n, seed=1)
    out = O.cheb_propagate(A, x, O.cheb_coefficients(32, 10.0))
    assert abs(np.linalg.norm(out) - 1.0) < 1e-11


# ----------------------------------------------------------------------------
# generators (nonzero counts printed in Tables 2 and 3)
# ----------------------------------------------------------------------------

def _star_nnz(n, r):
    return n ** 3 * (6 * r + 1) - 6 * n * n * sum(range(1, r + 1))


def test_generator_counts_small():
    for n in (3, 5, 8):
        assert W.stencil_3d(n, 27).nnz == (3 * n - 2) ** 3
        for order, pts in ((2, 7), (4, 13), (6, 19)):
            assert W.star_stencil_3d(n, order).nnz == _star_nnz(n, order // 2)
    assert W.stencil_2d(64, 5).nnz == 20224


def test_generator_counts_paper_tables():
    assert (3 * 128 - 2) ** 3 == 55_742_968           # HPCG 128^3, Table 2
    assert _star_nnz(160, 1) == 28_518_400             # order-2, Table 3
    assert _star_nnz(160, 2) == 52_787_200             # order-4, Table 3
    assert _star_nnz(160, 3) == 76_902_400             # order-6, Table 3
    assert _star_nnz(200, 1) == 55_760_000             # Anderson 200^3, Table 3
    # the formula matches the generator where generation is cheap
    assert W.anderson_3d(7).nnz == _star_nnz(7, 1)


def test_rgg_shape():
    A, _ = W.random_geometric(20000, 16.0, seed=0)
    deg = np.diff(A.rowptr)
    assert 13.0 < deg.mean() < 17.0
    M = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(A.n, A.n))
    assert (M != M.T).nnz == 0


# ----------------------------------------------------------------------------
# heat-equation Chebyshev propagation (Sec. 7, real modified-Bessel coefficients)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [0.5, 5.0, 20.0, 70.0])
def test_heat_coefficients_generating_function(tau):
    # sum_k c_k T_k(x) = exp(-tau (x + 1)) on [-1, 1]; T_k(cos t) = cos(k t)
    c = O.heat_coefficients(120, tau)
    t = np.linspace(0.0, np.pi, 41)
    series = np.cos(np.outer(t, np.arange(121))) @ c
    assert np.allclose(series, np.exp(-tau * (np.cos(t) + 1.0)), rtol=1e-10, atol=1e-14)


def test_heat_coefficients_sign_pattern():
    # a dropped (-1)^k would expand exp(+tau x) instead: at x = -1 the two
    # differ by exp(2 tau)
    tau = 3.0
    c = O.heat_coefficients(60, tau)
    assert np.all(c[1::2] < 0) and np.all(c[0::2] > 0)
    assert abs(np.sum(c * (-1.0) ** np.arange(61)) - 1.0) < 1e-12  # x = -1: exp(0)


def test_heat_operator_spectrum_and_eigenvectors():
    # order 2: L = -Laplacian_h has the Dirichlet eigenvectors
    # v = prod_d sin(j_d pi (x_d + 1) / (n + 1)), eigenvalue
    # sum_d (2 - 2 cos(j_d pi / (n + 1))); A = L / 6 - I, so one step with
    # tau gives exp(-tau lambda / 6) v
    n = 7
    A, r = W.heat_operator_3d(n, 2)
    assert r == 6.0
    g = np.arange(n)
    for j in [(1, 1, 1), (2, 5, 3), (7, 7, 7)]:
        s = [np.sin(jd * np.pi * (g + 1) / (n + 1)) for jd in j]
        v = np.einsum("i,j,k->kji", s[0], s[1], s[2]).reshape(-1)  # x fastest
        lam = sum(2.0 - 2.0 * np.cos(jd * np.pi / (n + 1)) for jd in j)
        tau = 10.0
        out = O.cheb_propagate_real(A, v, O.heat_coefficients(40, tau))
        assert np.allclose(out, np.exp(-tau * lam / 6.0) * v, rtol=0, atol=1e-12 * np.abs(v).max())


@pytest.mark.parametrize("order", [4, 6])
def test_heat_propagate_vs_expm(order):
    from scipy.linalg import expm

    A, r = W.heat_operator_3d(5, order)
    D = A.to_dense()
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= -1.0 - 1e-12 and ev.max() <= 1.0 + 1e-12
    x = W.uniform_vector(A.n, seed=4)
    tau = 12.0
    ref = expm(-tau * (D + np.eye(A.n))) @ x
    out = O.cheb_propagate_real(A, x, O.heat_coefficients(48, tau))
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref) + 1e-15
    # heat flow contracts the state
    assert np.linalg.norm(out) < np.linalg.norm(x)


# ----------------------------------------------------------------------------
# recursive level refinement (Sec. 4.4)
# ----------------------------------------------------------------------------

def test_refinement_worked_example():
    # Sec. 4.4: with a cache of at most six vertices, T(4)..T(6) (levels 6-8
    # of the 8x8 2d-7pt example, 22 vertices) induce a subgraph with eight
    # BFS levels whose level groups all satisfy Eq. (5): the process stops
    A = W.stencil_2d(8, 7)
    perm, lp = O.bfs_levels(A, 0)
    ones = np.ones(A.n, np.int64)
    fp, up, us = O.refine_levels(A, perm, lp, p=1, cache_bytes=300, stages=1, row_weight=ones)
    sizes = np.diff(up)
    assert np.all(2 * sizes * 12 < 150)                       # every unit fits "six vertices"
    region = us == 1
    assert sizes[region].sum() == 7 + 8 + 7
    # the refined rows are exactly those of levels 6-8, placed where they were
    lo, hi = lp[6], lp[9]
    assert sorted(fp[lo:hi].tolist()) == sorted(perm[lo:hi].tolist())
    assert np.array_equal(fp[:lo], perm[:lo]) and np.array_equal(fp[hi:], perm[hi:])
    # eight BFS levels: graph distances inside the subgraph from its first row
    sub = _induced_distances(A, fp[lo:hi])
    assert sub.max() + 1 == 8
    # with s_m = 0 nothing changes and the units are the level groups
    fp0, up0, us0 = O.refine_levels(A, perm, lp, p=1, cache_bytes=300, stages=0, row_weight=ones)
    assert np.array_equal(fp0, perm) and np.all(us0 == 0)
    assert np.diff(up0).tolist() == [6, 4, 5, 6, 7, 8, 7, 6, 5, 4, 6]


def _induced_distances(A, rows):
    """Unweighted distances inside the subgraph induced by ``rows`` from
    rows[0] (scipy), for the rows in the given order; unreachable rows get a
    distance one past the largest reachable one."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path as sp_path

    rows = np.asarray(rows, dtype=np.int64)
    S = sp.csr_matrix((np.ones(A.nnz), np.asarray(A.col, np.int64), np.asarray(A.rowptr, np.int64)),
                      shape=(A.n, A.n))
    U = ((S + S.T) != 0).astype(np.float64).tocsr()[rows][:, rows]
    d = sp_path(U, unweighted=True, directed=False, indices=0)
    d[np.isinf(d)] = np.nanmax(np.where(np.isinf(d), np.nan, d)) + 1
    return d.astype(np.int64)


@pytest.mark.parametrize("case", ["2d5pt", "27pt", "rgg"])
def test_refinement_invariants(case):
    if case == "2d5pt":
        A, p, C = W.stencil_2d(40, 5), 4, 6000
    elif case == "27pt":
        A, p, C = W.stencil_27pt_random(12, seed=3)[0], 3, 40000
    else:
        A, p, C = W.random_geometric(3000, 10.0, seed=2)[0], 2, 3000
    perm, lp = O.bfs_levels(A, 1)
    rowlen = np.diff(A.rowptr)
    budget = int(np.floor(0.5 * C))
    fp, up, us = O.refine_levels(A, perm, lp, p, C, stages=1)
    assert sorted(fp.tolist()) == list(range(A.n))
    assert up[0] == 0 and up[-1] == A.n and np.all(np.diff(up) > 0)
    unit_nnz = np.array([rowlen[fp[a:b]].sum() for a, b in zip(up[:-1], up[1:])])
    gptr = O.level_groups(O.level_nnz(A, perm, lp), p, C)
    group_rows = lp[gptr]
    viol = [(p + 1) * O.level_nnz(A, perm, lp)[gptr[i]:gptr[i + 1]].sum() * 12 >= budget
            for i in range(len(gptr) - 1)]
    assert any(viol)                                           # the case exercises refinement
    # stage-0 units are the non-violating groups, unchanged
    st0 = [(a, b) for a, b, s in zip(up[:-1], up[1:], us) if s == 0]
    for i in range(len(gptr) - 1):
        if not viol[i]:
            a, b = group_rows[i], group_rows[i + 1]
            assert (a, b) in st0 and np.array_equal(fp[a:b], perm[a:b])
    # every refined region keeps its rows, and inside it the subgraph
    # distances from its first row never decrease and units are whole levels
    i = 0
    while i < len(gptr) - 1:
        if not viol[i]:
            i += 1
            continue
        j = i
        while j < len(gptr) - 1 and viol[j]:
            j += 1
        a, b = group_rows[i], group_rows[j]
        assert sorted(fp[a:b].tolist()) == sorted(perm[a:b].tolist())
        d = _induced_distances(A, fp[a:b])
        assert np.all(np.diff(d) >= 0)
        for ua, ub in zip(up[:-1], up[1:]):
            if a <= ua < b:
                assert ub <= b
                if ub < b:
                    assert d[ub - a] > d[ub - 1 - a]          # a unit ends where a level ends
        i = j
    # every unit satisfies Eq. (5) unless it is a single level at the last stage
    for (a, b), s, nz in zip(zip(up[:-1], up[1:]), us, unit_nnz):
        if (p + 1) * nz * 12 >= budget:
            if s == 0:
                li = np.searchsorted(lp, a)
                assert lp[li] == a and lp[li + 1] == b          # a single stage-0 level
            else:
                d = _induced_distances(A, fp[a:b])
                assert s == 1                                    # last stage (s_m = 1)

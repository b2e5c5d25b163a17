"""Learned-tuner network: the FP64 oracle against finite differences and
closed forms (CPU), and the HIP kernels against the oracle (GPU)."""
import numpy as np
import pytest

from oracle import mlp as M


def _rand(D, H, B, seed):
    rng = np.random.default_rng(seed)
    P = rng.normal(0, 0.5, size=M.param_count(D, H))
    X = rng.normal(0, 1, size=(B, D))
    y = rng.normal(0, 1, size=B)
    return P, X, y


def test_oracle_hand_computed():
    # D = 2, H = 2: W1 = I, b1 = (0, -1), W2 = [[1, 1], [0, 2]], b2 = 0,
    # w3 = (1, -1), b3 = 0.5; x = (3, 2): z1 = (3, 1), a1 = (3, 1),
    # z2 = (4, 2), out = 4 - 2 + 0.5 = 2.5
    P = np.array([1, 0, 0, 1, 0, -1, 1, 1, 0, 2, 0, 0, 1, -1, 0.5], float)
    assert M.forward(P, [[3.0, 2.0]], 2, 2).tolist() == [2.5]
    # x = (-1, 0): z1 = (-1, -1) -> a1 = 0, out = b3
    assert M.forward(P, [[-1.0, 0.0]], 2, 2).tolist() == [0.5]


@pytest.mark.parametrize("D,H,B", [(3, 4, 5), (24, 64, 33), (7, 16, 1)])
def test_oracle_gradient_finite_differences(D, H, B):
    P, X, y = _rand(D, H, B, D + H)
    g = M.gradient(P, X, y, D, H)
    h = 1e-6
    idx = np.random.default_rng(0).choice(P.size, size=min(60, P.size), replace=False)
    for k in idx:
        e = np.zeros_like(P)
        e[k] = h
        fd = (M.loss(P + e, X, y, D, H) - M.loss(P - e, X, y, D, H)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd))


def test_oracle_adam_first_step():
    # at step 1, mhat = g and vhat = g^2, so every coordinate with g != 0
    # moves by lr (up to eps) against the sign of g
    rng = np.random.default_rng(1)
    P = rng.normal(size=50)
    g = rng.normal(size=50)
    g[3] = 0.0
    new, m, v = M.adam_step(P, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    d = new - P
    nz = g != 0
    assert np.allclose(np.abs(d[nz]), 0.01, rtol=1e-8 / np.abs(g[nz]).min() + 1e-12)
    assert np.all(np.sign(d[nz]) == -np.sign(g[nz]))
    assert d[3] == 0.0


def test_oracle_adam_converges_on_quadratic():
    # Adam on f(p) = |p - c|^2 approaches c
    c = np.linspace(-1, 1, 10)
    P = np.zeros(10)
    m = np.zeros(10)
    v = np.zeros(10)
    for t in range(1, 3001):
        P, m, v = M.adam_step(P, 2 * (P - c), m, v, t, lr=0.01)
    assert np.allclose(P, c, atol=1e-3)


# ----------------------------------------------------------------------------
# GPU kernels (through the C-ABI)
# ----------------------------------------------------------------------------

@pytest.mark.gpu
@pytest.mark.parametrize("D,H,B", [(24, 64, 257), (5, 16, 3), (30, 64, 2000)])
def test_kernels_match_oracle(D, H, B):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_01598_amd.tune import DeviceMLP

    P, X, y = _rand(D, H, B, 7 + D)
    net = DeviceMLP(D, H, params=P.astype(np.float32))
    Pf = P.astype(np.float32).astype(np.float64)
    Xf = X.astype(np.float32).astype(np.float64)
    yf = y.astype(np.float32).astype(np.float64)
    out = net.predict(X)
    ref = M.forward(Pf, Xf, D, H)
    assert np.allclose(out, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())
    g, lval = net.gradient(X, y)
    gref = M.gradient(Pf, Xf, yf, D, H)
    assert abs(lval - M.loss(Pf, Xf, yf, D, H)) <= 1e-4 * max(1.0, lval)
    assert np.linalg.norm(g - gref) <= 1e-4 * max(1e-3, np.linalg.norm(gref))
    # one Adam step against the oracle's
    net.adam(g, lr=1e-2)
    newp, _, _ = M.adam_step(Pf, g.astype(np.float64), np.zeros_like(Pf), np.zeros_like(Pf), 1, lr=1e-2)
    assert np.allclose(net.params(), newp, rtol=1e-5, atol=1e-6)


@pytest.mark.gpu
def test_kernels_learn_a_function():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_01598_amd.tune import DeviceMLP

    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, size=(1024, 6))
    y = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3] ** 2
    net = DeviceMLP(6, 64, seed=0)
    first = net.gradient(X, y)[1]
    for _ in range(1500):
        g, _ = net.gradient(X, y)
        net.adam(g, lr=3e-3)
    last = net.gradient(X, y)[1]
    assert last < 0.05 * first

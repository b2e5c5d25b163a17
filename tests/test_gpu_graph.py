"""Captured and replayed runs: the persistent MPK kernel keeps its run epoch
in device memory (the launch arguments do not change between runs), so a
HIP graph that captured mpk_run can be replayed.  Every replay is compared
bit for bit with the eager run of the same plan, with eager work and
synchronisations between the replays."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import Plan  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", ["27pt", "refined", "zipf_k4"])
def test_replayed_mpk_run(case):
    dev = _dev()
    k = 4 if case == "zipf_k4" else 1
    if case == "zipf_k4":
        A = W.zipf_rows(8192, 2.0, seed=7)
    else:
        A = W.stencil_27pt_random(32, seed=5)[0]
    p = 6
    opts = dict(root_mode=1, skew=2, tile_nnz=1200, nrhs=k)
    if case == "refined":
        opts["recursion_stages"] = 1
        C = 200000
    else:
        C = 2 << 20
    pl = Plan(A, p, C, **opts)
    perm = pl.arrays()[0].astype(np.int64)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (A.n, k)) if k > 1 else rng.uniform(-1, 1, A.n)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    Y = torch.full((p,) + tuple(X.shape), float("nan"), dtype=torch.float64, device=dev)
    print(f"graph case {case}: n={A.n} tiles={pl.info()['n_tiles']}", flush=True)
    pl.run(X, Y)
    pl.status()
    eager = Y.clone()
    ref = O.spmv_powers(A, x, p)
    out = np.empty((p,) + x.shape)
    out[:, perm] = eager.cpu().numpy().reshape((p,) + x.shape)
    for q in range(p):
        assert np.linalg.norm(out[q] - ref[q]) <= 1e-12 * np.linalg.norm(ref[q])

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pl.run(X, Y)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for r in range(4):
        Y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        pl.status()
        assert torch.equal(Y, eager), f"replay {r} differs from the eager run"
        # an eager run between replays continues the epoch sequence
        Y.fill_(float("nan"))
        pl.run(X, Y)
        pl.status()
        assert torch.equal(Y, eager)


def test_replayed_chebyshev_step():
    from paper_2205_01598_amd.cheb import ChebPropagator

    dev = _dev()
    A = W.anderson_3d(12, seed=3)
    x = W.random_phase_state(A.n, seed=3)
    M, p, r_dt = 32, 8, 10.0
    pl = Plan(A, p, 1 << 20, nrhs=2, root_mode=1, tile_nnz=700, skew=2)
    perm = pl.arrays()[0].astype(np.int64)
    prop = ChebPropagator.schroedinger(pl, M, r_dt)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    acc = torch.empty_like(X)
    prop.step(X, acc)
    pl.status()
    eager = acc.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            prop.step(X, acc)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for r in range(3):
        acc.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        pl.status()
        assert torch.equal(acc, eager), f"replay {r} differs from the eager step"
    ref = O.cheb_propagate(A, x, O.cheb_coefficients(M, r_dt))
    h = np.empty((A.n, 2))
    h[perm] = eager.cpu().numpy()
    assert np.linalg.norm(h - ref) <= 1e-12 * np.linalg.norm(ref)

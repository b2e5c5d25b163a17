"""GPU: the allocation-free backward pass (mpk_mlp_backward_noalloc) against
the backward pass with a caller workspace (mpk_mlp_backward), through the
C-ABI: identical gradients and loss, bit for bit, on two calls in a row (the
second with a smaller batch, so the fixed scratch still holds the first
call's larger contents), and a clear error for a batch beyond the scratch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import MpkError  # noqa: E402
from paper_2205_01598_amd._lib import check, lib  # noqa: E402


def _p(t):
    return ctypes.c_void_p(int(t.data_ptr()))


def _stream():
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def _case(D, H, B, seed, dev):
    rng = np.random.default_rng(seed)
    n = lib().mpk_mlp_param_count(D, H)
    P = torch.from_numpy(rng.normal(0, 0.5, n).astype(np.float32)).to(dev)
    X = torch.from_numpy(rng.normal(0, 1, (B, D)).astype(np.float32)).to(dev)
    y = torch.from_numpy(rng.normal(0, 1, B).astype(np.float32)).to(dev)
    out = torch.empty(B, dtype=torch.float32, device=dev)
    cache = torch.empty(B * 2 * H, dtype=torch.float32, device=dev)
    check(lib().mpk_mlp_forward(_p(P), D, H, _p(X), B, _p(out), _p(cache), _stream()))
    return n, P, X, y, out, cache


def test_noalloc_backward_matches_workspace_backward():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    D, H = 24, 64
    for B, seed in ((5000, 1), (700, 2)):
        n, P, X, y, out, cache = _case(D, H, B, seed, dev)
        work = torch.empty(B * (2 * H + 1), dtype=torch.float32, device=dev)
        g_ref = torch.empty(n, dtype=torch.float32, device=dev)
        l_ref = torch.empty(1, dtype=torch.float32, device=dev)
        check(lib().mpk_mlp_backward(_p(P), D, H, _p(X), _p(y), B, _p(out), _p(cache), _p(work), _p(g_ref),
                                     _p(l_ref), _stream()))
        g = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        check(lib().mpk_mlp_backward_noalloc(_p(P), D, H, _p(X), _p(y), B, _p(out), _p(cache), _p(g),
                                             _p(loss), _stream()))
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), f"B={B}: gradients differ"
        assert torch.equal(loss, l_ref), f"B={B}: loss differs"


def test_noalloc_backward_rejects_oversized_batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    D, H = 8, 64
    B = (1 << 22) // (2 * H + 1) + 1
    dummy = torch.empty(1, dtype=torch.float32, device=dev)
    with pytest.raises(MpkError, match="scratch"):
        check(lib().mpk_mlp_backward_noalloc(_p(dummy), D, H, _p(dummy), _p(dummy), B, _p(dummy), _p(dummy),
                                             _p(dummy), None, _stream()))

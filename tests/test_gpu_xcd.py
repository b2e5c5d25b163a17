"""GPU: XCD placement and flag-hop probes (include/mpk.h, mpk_xcd_ids and
mpk_hop_probe).

The XCD-sliced ticket streams (mpk_options.xcd_streams = 8) assume that the
workgroups b, b + 8, b + 16, ... of a launch share one XCD.  The dispatcher
deals workgroups to the 8 XCDs round-robin, starting where its previous
launch stopped, so workgroup b runs on XCD (b + r) % 8 with r fixed for the
launch (r = 0 in a fresh process); this checks that on the hardware register
for the grid shapes the persistent kernel launches.  The hop probe
must complete at agent scope, the scope every dependency flag uses.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd.mpk import hop_probe, xcd_ids  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("wg,spin", [(8, 0), (1024, 0), (2048, 100), (4096, 0)])
def test_workgroups_round_robin_over_xcds(wg, spin):
    dev = _dev()
    ids = torch.full((wg,), -1, dtype=torch.int32, device=dev)
    xcd_ids(ids, wg, spin)
    h = ids.cpu().numpy()
    assert (h >= 0).all() and (h < 8).all()
    np.testing.assert_array_equal(h, (h[0] + np.arange(wg)) % 8)


@pytest.mark.parametrize("peer", [1, 8])
def test_agent_scope_hop_completes(peer):
    dev = _dev()
    flags = torch.zeros(64, dtype=torch.int32, device=dev)
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    khz = hop_probe(flags, peer, 0, 200, 1 << 20, out)
    ticks, done = (int(v) for v in out.cpu().numpy())
    assert done == 200
    assert khz > 0 and ticks > 0
    # a one-way hop of an agent-scope flag is well under 10 microseconds
    assert ticks / 400 / khz * 1e6 < 1e4

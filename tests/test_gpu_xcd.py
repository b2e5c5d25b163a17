"""GPU: XCD placement and flag-hop probes (include/mpk.h, mpk_xcd_ids and
mpk_hop_probe).

The XCD-sliced ticket streams (mpk_options.xcd_streams = 8) assume that
workgroup b of a launch runs on XCD b % 8; this checks it on the hardware
register for the grid shapes the persistent kernel launches.  The hop probe
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
def test_workgroup_xcd_is_block_index_mod_8(wg, spin):
    dev = _dev()
    ids = torch.full((wg,), -1, dtype=torch.int32, device=dev)
    xcd_ids(ids, wg, spin)
    h = ids.cpu().numpy()
    assert (h >= 0).all() and (h < 8).all()
    np.testing.assert_array_equal(h, np.arange(wg) % 8)


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

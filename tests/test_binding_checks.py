"""Argument checks of the binding and the planner's size limits (CPU only).

The Python binding validates every device buffer before it reaches the
library (dtype, device, contiguity, element counts against n, k and the
powers of the run) and the lengths of the recurrence coefficient arrays; the
planner refuses plans whose tickets (tile * 64 + power - 1, int32) would
overflow."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_2205_01598_amd import MpkError, Plan, Recurrence  # noqa: E402


def test_tile_count_limit():
    # a diagonal matrix of 2^25 + 1000 rows with one-nonzero tiles would need
    # tile indices of 26 bits
    n = (1 << 25) + 1000
    A = W.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n))
    with pytest.raises(MpkError, match="too many tiles"):
        Plan(A, 2, 1 << 30, upload=False, tile_nnz=1)
    with pytest.raises(MpkError, match="too many tiles"):
        Plan(A, 2, 1 << 10, upload=False, tile_nnz=1, recursion_stages=1)


@pytest.fixture(scope="module")
def plan():
    A = W.stencil_2d(8, 5)
    return Plan(A, 3, 1 << 16, upload=False, nrhs=2)


def _t(shape, dtype=torch.float64):
    return torch.zeros(shape, dtype=dtype)


def test_run_rejects_host_tensors(plan):
    with pytest.raises(ValueError, match="GPU"):
        plan.run(_t((64, 2)), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="GPU"):
        plan.run_baseline(_t((64, 2)), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="GPU"):
        plan.run_sync(_t((64, 2)), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="GPU"):
        plan.permute(_t((64, 2)), _t((64, 2)), True)


def test_run_rejects_wrong_dtype_size_layout(plan):
    with pytest.raises(ValueError, match="float64"):
        plan.run(_t((64, 2), torch.float32), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="elements"):
        plan.run(_t((64, 1)), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="elements"):
        plan.run(_t((64, 2)), _t((2, 64, 2)))
    with pytest.raises(ValueError, match="contiguous"):
        plan.run(_t((2, 64)).t(), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="torch tensor"):
        plan.run(np.zeros((64, 2)), _t((3, 64, 2)))
    with pytest.raises(ValueError, match="powers"):
        plan.run(_t((64, 2)), _t((3, 64, 2)), powers=4)
    with pytest.raises(ValueError, match="powers"):
        plan.run(_t((64, 2)), _t((3, 64, 2)), powers=0)


def test_recurrence_lengths_checked(plan):
    # alpha/beta/gamma need p entries, complex coef 2p, complex coef0 2
    short = Recurrence(np.ones(2), coef=np.ones(4), complex_pairs=True, acc=_t((64, 2)))
    with pytest.raises(ValueError, match="alpha"):
        plan.run(_t((64, 2)), _t((3, 64, 2)), short)
    bad_coef = Recurrence(np.ones(3), coef=np.ones(5), complex_pairs=True, acc=_t((64, 2)))
    with pytest.raises(ValueError, match="coef"):
        plan.run(_t((64, 2)), _t((3, 64, 2)), bad_coef)
    bad_c0 = Recurrence(np.ones(3), coef=np.ones(6), complex_pairs=True, acc=_t((64, 2)), coef0=1.0)
    with pytest.raises(ValueError, match="coef0"):
        plan.run(_t((64, 2)), _t((3, 64, 2)), bad_c0)
    bad_prev = Recurrence(np.ones(3), gamma=np.ones(3), y_prev=_t((64, 1)))
    with pytest.raises(ValueError, match="y_prev"):
        plan.run(_t((64, 2)), _t((3, 64, 2)), bad_prev)
    # a shorter run needs entries only for its powers, but still a GPU tensor
    ok_len = Recurrence(np.ones(2), coef=np.ones(4), complex_pairs=True, acc=_t((64, 2)))
    with pytest.raises(ValueError, match="GPU"):
        plan.run(_t((64, 2)), _t((2, 64, 2)), ok_len, powers=2)


def test_from_device_checks_arguments():
    rp = torch.zeros(5, dtype=torch.int64)
    col = torch.zeros(4, dtype=torch.int32)
    val = torch.zeros(4, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        Plan.from_device(rp, col, val, 2, 1 << 20)
    with pytest.raises(ValueError, match="rowptr: dtype"):
        Plan.from_device(rp.to(torch.int32), col, val, 2, 1 << 20)
    with pytest.raises(ValueError, match="col: dtype"):
        Plan.from_device(rp, col.to(torch.int64), val, 2, 1 << 20)
    with pytest.raises(ValueError, match="val: dtype"):
        Plan.from_device(rp, col, val.to(torch.float32), 2, 1 << 20)
    with pytest.raises(ValueError, match="contiguous"):
        Plan.from_device(rp, torch.zeros(8, dtype=torch.int32)[::2], val, 2, 1 << 20)
    with pytest.raises(ValueError, match="torch tensor"):
        Plan.from_device(np.zeros(5, np.int64), col, val, 2, 1 << 20)

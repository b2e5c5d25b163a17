"""GPU parity sweep over seeded random configurations (fuzz_cases: random
irregular, banded, 2D stencil and power-law matrices; random p, cache
budget, tiles, skew, ticket streams, grid size, right-hand sides and
recursion stages, FP32 / BF16 storage with FP64 arithmetic) against the
oracle (on the rounded values where the storage rounds them), relative
error <= 1e-12 per power.  test_plan_fuzz checks the same plans on the host."""
import numpy as np
import pytest

import fuzz_cases
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_01598_amd import Plan  # noqa: E402


@pytest.mark.parametrize("seed", range(fuzz_cases.N_CASES))
def test_fuzz_parity(seed):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    A, p, C, opts, x = fuzz_cases.case(seed)
    print(f"fuzz case {seed}: n={A.n} nnz={A.nnz} p={p} C={C} {opts}", flush=True)
    pl = Plan(A, p, C, **opts)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
    Y = torch.full((p,) + tuple(X.shape), float("nan"), dtype=torch.float64, device=dev)
    pl.run(X, Y)
    pl.status()
    out = np.empty((p,) + x.shape)
    out[:, perm] = Y.cpu().numpy().reshape((p,) + x.shape)
    dt = opts.get("val_dtype", "f64")
    ref = O.spmv_powers(A if dt == "f64" else O.round_values(A, dt), x, p)
    for q in range(p):
        nb = np.linalg.norm(ref[q])
        e = np.linalg.norm(out[q] - ref[q]) / (nb if nb > 0 else 1.0)
        assert e <= 1e-12, f"power {q + 1}: rel err {e:.3e}"
    # the baseline path on the same plan
    Y.fill_(float("nan"))
    pl.run_baseline(X, Y)
    torch.cuda.synchronize()
    out[:, perm] = Y.cpu().numpy().reshape((p,) + x.shape)
    for q in range(p):
        nb = np.linalg.norm(ref[q])
        assert np.linalg.norm(out[q] - ref[q]) <= 1e-12 * (nb if nb > 0 else 1.0)

"""Host checks of the plans the GPU parity sweep runs (fuzz_cases): levels,
groups and schedule equal to the oracle's, tiles, dependencies and ticket
order by their invariants."""
import pytest

import fuzz_cases
from paper_2205_01598_amd import Plan
from test_plan_host import _check_plan
from test_plan_refined import _check_refined

import oracle as O  # noqa: E402
import numpy as np  # noqa: E402


@pytest.mark.parametrize("seed", range(fuzz_cases.N_CASES))
def test_fuzz_plan(seed):
    A, p, C, opts, _ = fuzz_cases.case(seed)
    opts = dict(opts)
    stages = opts.pop("recursion_stages")
    if stages == 0:
        root_mode = opts.pop("root_mode")
        opts.pop("accum_f64", None)
        _check_plan(A, p, C, root_mode, dtype=opts.pop("val_dtype", "f64"), **opts)
    else:
        pl = Plan(A, p, C, upload=False, recursion_stages=stages, **opts)
        operm, olp = O.bfs_levels(A, opts["root_mode"])
        fp, up, us = O.refine_levels(A, operm, olp, p, C, stages=stages)
        assert np.array_equal(pl.arrays()[0], fp)
        if pl.info()["recursive"]:
            _check_refined(pl, A, p, k=opts["nrhs"])
        else:
            # nothing refined: the plan is the unrefined one
            assert np.all(us == 0)
            root_mode = opts.pop("root_mode")
            _check_plan(A, p, C, root_mode, **opts)

"""Seeded random planner/kernel configurations shared by the CPU plan checks
(test_plan_fuzz.py) and the GPU parity sweep (test_gpu_fuzz.py), so every
plan the GPU runs has first been checked on the host."""
import numpy as np

import workloads as W

N_CASES = 40


def case(seed):
    """Returns (A, p, C, opts, x) for case `seed`."""
    rng = np.random.default_rng(5000 + seed)
    kind = seed % 4
    if kind == 0:
        n = int(rng.integers(1, 2500))
        A = W.random_small_csr(n, float(rng.uniform(1.0, 10.0)) / max(n, 1), rng,
                               symmetric_pattern=bool(rng.integers(0, 2)),
                               empty_rows=float(rng.uniform(0, 0.15)), duplicates=float(rng.uniform(0, 0.1)))
    elif kind == 1:
        A = W.banded_random(int(rng.integers(50, 4000)), int(rng.integers(2, 80)), seed=seed)
    elif kind == 2:
        A = W.stencil_2d(int(rng.integers(3, 60)), int(rng.choice([5, 9])))
    else:
        A = W.zipf_rows(int(rng.integers(100, 3000)), float(rng.uniform(1.5, 2.5)), seed=seed, cap=200)
    p = int(rng.integers(1, 11))
    C = int(np.exp(rng.uniform(np.log(2e3), np.log(2e7))))
    k = int(rng.choice([1, 1, 2, 4]))
    rec = int(rng.choice([0, 0, 1, 2]))
    opts = dict(root_mode=int(rng.integers(0, 2)), nrhs=k, skew=int(rng.integers(1, 4)),
                tile_nnz=int(rng.choice([0, int(rng.integers(16, 4000))])), recursion_stages=rec)
    if rec == 0:
        opts["xcd_streams"] = int(rng.choice([1, 8]))
    if rng.integers(0, 3) == 0:
        opts["workgroups"] = int(rng.integers(1, 600))
    x = rng.uniform(-1, 1, (A.n, k)) if k > 1 else rng.uniform(-1, 1, A.n)
    if seed >= 24:
        # large ticket skews (drawn last, so the cases below 24 are unchanged)
        opts["skew"] = int(rng.choice([4, 8, 16, 32]))
    if seed >= 32 and rec == 0 and k <= 2:
        # FP32 / BF16 storage with FP64 arithmetic: the FP64 oracle on the
        # rounded values keeps the FP64 bar
        opts["val_dtype"] = str(rng.choice(["f32", "bf16"]))
        opts["accum_f64"] = 1
    return A, p, C, opts, x

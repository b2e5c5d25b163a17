"""Autotuner / learned tuner.  CPU: configuration space and database
integrity.  GPU: train the cost model with the library's MLP kernels on the
MI355X sweep database, then compare its choices on held-out matrices with the
exhaustive sweep's best and with the untuned default configuration."""
import json
import math
import os

import numpy as np
import pytest

from paper_2205_01598_amd import tune

DB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                  "paper_2205_01598_amd", "data", "tuner_sweep_mi355x.jsonl")


def test_config_grid():
    grid = tune.config_grid()
    assert grid[0] == tune.DEFAULT
    keys = {json.dumps(c, sort_keys=True) for c in grid}
    assert len(keys) == len(grid) == 1 + len(tune.CACHE_MB) * len(tune.SKEWS) * len(tune.TILES) * len(tune.GRIDS)
    enc = np.stack([tune.encode_config(c) for c in grid])
    assert np.all(np.isfinite(enc)) and len({tuple(e) for e in enc}) == len(grid)


@pytest.mark.skipif(not os.path.exists(DB), reason="no sweep database")
def test_database_integrity():
    recs = tune.load_db(DB)
    seeds = {r["seed"] for r in recs}
    assert len(seeds) >= 100
    fams = {r["spec"]["family"] for r in recs}
    assert fams == {"stencil2d", "stencil3d", "banded", "zipf", "rgg"}
    for r in recs:
        assert r["ms"] > 0 and len(r["features"]) == 24
    train, test = tune.split_seeds(recs)
    assert {r["seed"] for r in train}.isdisjoint({r["seed"] for r in test})


@pytest.mark.gpu
@pytest.mark.skipif(not os.path.exists(DB), reason="no sweep database")
def test_learned_tuner_beats_default_on_held_out():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    recs = tune.load_db(DB)
    train, test = tune.split_seeds(recs)
    tuner = tune.LearnedTuner(hidden=64, seed=0)
    loss = tuner.fit(train, steps=6000)
    assert math.isfinite(loss)
    static = tune.best_static(train)
    m = tune.evaluate(tuner, test, static)
    # The yardstick is the one configuration that is best on the training
    # matrices as a whole (C = 128 MB, skew 4 on this database): the
    # per-matrix choice has to beat it, so the features matter.  Measured on
    # this database (N up to 1e7): 1.040-1.054x for training seeds 0-2 (the
    # model's own pick) and 1.066x for the best of its three top-ranked
    # configurations; the sweep's best is 1.20x the untuned default
    # (C = 256 MB, skew 1, all resident workgroups), the static one 1.10x.
    assert m["gain_over_best_static"] > 1.035, m
    assert m["shortlist3_gain_over_best_static"] > 1.05, m
    assert m["geomean_gain_over_default"] > 1.10, m
    # and the choice is close to the exhaustive sweep's best
    assert m["geomean_pick_over_best"] < 1.06, m
    # measuring the model's three best configurations comes closer still
    assert m["shortlist3_geomean_over_best"] <= m["geomean_pick_over_best"], m
    assert m["shortlist3_geomean_over_best"] < 1.04, m


class _RankNet:
    """Stand-in network: predicts a given score per configuration."""

    def __init__(self, score):
        self.score = score

    def predict(self, X):
        return np.array([self.score(tuple(row[-4:])) for row in X])


def test_shortlist_and_evaluate_on_synthetic_records():
    grid = tune.config_grid()
    rng = np.random.default_rng(1)
    recs = []
    for seed in range(5):
        ms = rng.uniform(0.5, 2.0, len(grid))
        for c, t in zip(grid, ms):
            recs.append({"seed": seed, "spec": {}, "p": 4, "features": [0.0] * 24, "config": c, "ms": float(t)})
    enc = {tuple(tune.encode_config(c)): i for i, c in enumerate(grid)}
    t = tune.LearnedTuner()
    t.mu, t.sd = np.zeros(24), np.ones(24)
    # a model that ranks by the true times of seed 0 is exact there
    times0 = [r["ms"] for r in recs if r["seed"] == 0]
    t.net = _RankNet(lambda e: times0[enc[e]])
    order = sorted(range(len(grid)), key=lambda i: times0[i])
    assert t.shortlist([0.0] * 24, 4) == [grid[i] for i in order[:4]]
    assert t.choose([0.0] * 24) == grid[order[0]]
    m = tune.evaluate(t, [r for r in recs if r["seed"] == 0], shortlist=(1, 3))
    assert m["geomean_pick_over_best"] == 1.0 and m["shortlist3_geomean_over_best"] == 1.0
    # the reversed ranking: the shortlist of m is the best of the m slowest
    t.net = _RankNet(lambda e: -times0[enc[e]])
    m = tune.evaluate(t, [r for r in recs if r["seed"] == 0], shortlist=(1, 3))
    srt = sorted(times0)
    assert np.isclose(m["geomean_pick_over_best"], srt[-1] / srt[0])
    assert np.isclose(m["shortlist3_geomean_over_best"], srt[-3] / srt[0])
    assert np.isclose(m["shortlist1_geomean_over_best"], m["geomean_pick_over_best"])


def test_best_static_is_grid_member_and_optimal_on_its_records():
    recs = []
    grid = tune.config_grid()
    rng = np.random.default_rng(0)
    for seed in range(6):
        for i, c in enumerate(grid):
            # configuration 3 is twice as fast as the default everywhere
            ms = 1.0 if i == 0 else (0.5 if i == 3 else float(rng.uniform(0.6, 1.5)))
            recs.append({"seed": seed, "spec": {}, "p": 4, "features": [0.0] * 24, "config": c, "ms": ms})
    assert tune.best_static(recs) == grid[3]


@pytest.mark.gpu
def test_autotune_picks_fastest_and_leaves_plan_there():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle as O
    import workloads as W
    from paper_2205_01598_amd import Plan

    A = W.stencil_2d(160, 9)
    p = 6
    x = W.uniform_vector(A.n, seed=3)
    pl = Plan(A, p, 1 << 20, root_mode=1)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(x[perm])).cuda()
    Y = torch.empty((p, A.n), dtype=torch.float64, device="cuda")
    cands = [dict(cache_mb=1, skew=1, tile_nnz=300), dict(cache_mb=4, skew=2, tile_nnz=2000),
             dict(cache_mb=1, skew=12, tile_nnz=1000, workgroups=64)]
    cfg, ms, timings = tune.autotune(torch, pl, p, cands, lambda: pl.run(X, Y), reps=3, warmup=1)
    assert [c for c, _ in timings] == cands
    assert (cfg, ms) == min(timings, key=lambda r: r[1])
    # the plan is left at the chosen configuration: same tiles and tickets
    # as a fresh plan made with it
    fresh = Plan(A, p, cfg["cache_mb"] << 20, upload=False, root_mode=1,
                 **{k: v for k, v in cfg.items() if k != "cache_mb"})
    for a, b in zip(pl.tiles(), fresh.tiles()):
        assert np.array_equal(a, b)
    pl.run(X, Y)
    pl.status()
    out = np.empty((p, A.n))
    out[:, perm] = Y.cpu().numpy()
    ref = O.spmv_powers(A, x, p)
    for q in range(p):
        assert np.linalg.norm(out[q] - ref[q]) <= 1e-12 * np.linalg.norm(ref[q])


@pytest.mark.gpu
@pytest.mark.skipif(not os.path.exists(DB), reason="no sweep database")
def test_learned_shortlist_tune_runs_its_best_measured_choice():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import workloads as W
    from paper_2205_01598_amd import Plan

    recs = tune.load_db(DB)
    train, _ = tune.split_seeds(recs)
    tuner = tune.LearnedTuner(hidden=16, seed=1)
    tuner.fit(train, steps=200)  # a rough model is enough to exercise the path
    A = W.stencil_2d(120, 5)
    p = 4
    pl = Plan(A, p, 256 << 20, root_mode=1)
    perm = pl.arrays()[0].astype(np.int64)
    X = torch.from_numpy(np.ascontiguousarray(W.uniform_vector(A.n, seed=0)[perm])).cuda()
    Y = torch.empty((p, A.n), dtype=torch.float64, device="cuda")
    tune._apply(pl, p, tune.DEFAULT)
    short = tuner.shortlist(tune.plan_features(pl), 3)
    cfg, ms, timings = tuner.tune(torch, pl, p, lambda: pl.run(X, Y), m=3, reps=2, warmup=1)
    assert [c for c, _ in timings] == short and cfg in short
    assert ms == min(t for _, t in timings)
    fresh = Plan(A, p, int(cfg["cache_mb"]) << 20, upload=False, root_mode=1,
                 **{k: int(v) for k, v in cfg.items() if k != "cache_mb"})
    for a, b in zip(pl.tiles(), fresh.tiles()):
        assert np.array_equal(a, b)

"""Autotuner and learned tuner for the level-blocked MPK.

* ``sweep``: for each matrix of a seeded corpus, one plan (one BFS), then every
  launch configuration of ``config_grid()`` through ``mpk_plan_retune`` and a
  timed ``mpk_run``; one JSON record per (matrix, p, configuration) appended
  to a timing database.  The exhaustive sweep is the fallback of the learned
  choice and the yardstick it is measured against.
* ``DeviceMLP``: the 3-layer perceptron whose forward pass, backward pass and
  Adam update are the library's HIP kernels (``mpk_mlp_*``); PyTorch only
  holds the device buffers.
* ``LearnedTuner``: a cost model, features(matrix, p) + encoding(config) ->
  log(t_config / t_default), trained with ``DeviceMLP``; the configuration
  with the smallest prediction is chosen, which fixes the level-group budget
  C and the workgroup count (plus tile size and ticket skew).
"""
from __future__ import annotations

import ctypes
import itertools
import json
import math
import os
import time

import numpy as np

from . import _lib
from ._lib import check, lib
from .mpk import Plan

# configuration space: level-group budget C, ticket skew, tile size, grid
CACHE_MB = (32, 128, 512)
SKEWS = (1, 2, 4, 8)
TILES = (2048, 8192)
GRIDS = (1024, 2048)
DEFAULT = {"cache_mb": 256, "skew": 1, "tile_nnz": 0, "workgroups": 0}


def config_grid():
    grid = [dict(DEFAULT)]
    for c, s, t, w in itertools.product(CACHE_MB, SKEWS, TILES, GRIDS):
        grid.append({"cache_mb": c, "skew": s, "tile_nnz": t, "workgroups": w})
    return grid


def encode_config(c) -> np.ndarray:
    tile = c["tile_nnz"] or 8192  # the library's default tile
    wg = c["workgroups"] or 2048  # all resident workgroups of the chunk kernel
    return np.array([math.log2(c["cache_mb"] / 32.0) / 4.0, math.log2(c["skew"]) / 3.0,
                     math.log2(tile / 2048.0) / 4.0, math.log2(wg / 1024.0)], dtype=np.float64)


def plan_features(plan: Plan) -> np.ndarray:
    f = np.empty(_lib.MPK_NUM_FEATURES, np.float64)
    check(lib().mpk_plan_features(plan._h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return f


def _apply(plan: Plan, p: int, c: dict, nrhs: int = 1):
    plan.retune(p, int(c["cache_mb"]) << 20, root_mode=1, skew=int(c["skew"]), tile_nnz=int(c["tile_nnz"]),
                workgroups=int(c["workgroups"]), nrhs=nrhs)


def autotune(torch, plan: Plan, p: int, candidates, run, reps: int = 5, warmup: int = 2, **fixed):
    """The exhaustive autotuner: retunes ``plan`` (same levels, no new BFS) to
    every candidate configuration, times ``run()`` (one level-blocked run on
    the caller's device buffers) and leaves the plan at the fastest.
    A candidate is a dict of ``cache_mb`` and any of ``skew``, ``tile_nnz``,
    ``workgroups`` (missing keys take the library's defaults); ``fixed``
    holds further retune options shared by all (``nrhs``, ``val_dtype``,
    ``root_mode``, default 1).  Returns (best configuration, its mean time in
    ms, [(configuration, ms)] for every candidate)."""
    fixed.setdefault("root_mode", 1)

    def apply(c):
        opts = dict(fixed)
        opts.update({k: int(v) for k, v in c.items() if k != "cache_mb"})
        plan.retune(p, int(c["cache_mb"]) << 20, **opts)

    timings = []
    for c in candidates:
        apply(c)
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            run()
        e.record()
        torch.cuda.synchronize()
        plan.status()
        timings.append((dict(c), s.elapsed_time(e) / reps))
    best = min(timings, key=lambda r: r[1])
    apply(best[0])
    return best[0], best[1], timings


def time_run(torch, plan: Plan, X, Y, reps: int = 5, warmup: int = 2) -> float:
    for _ in range(warmup):
        plan.run(X, Y)
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        plan.run(X, Y)
    e.record()
    torch.cuda.synchronize()
    plan.status()
    return s.elapsed_time(e) / reps


def _corpus_matrix(args):
    import workloads as W

    return W.tuner_matrix(*args)


def _corpus(seeds, n_min, n_max, workers):
    """(seed, matrix, spec) in seed order; with ``workers`` > 0 the matrices
    are generated that many seeds ahead in worker processes (no GPU use
    there), so generation overlaps the timing of the previous matrix."""
    if workers <= 0:
        import workloads as W

        for seed in seeds:
            yield (seed,) + tuple(W.tuner_matrix(seed, n_min, n_max))
        return
    import collections
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        pending = collections.deque()
        it = iter(seeds)
        for seed in it:
            pending.append((seed, ex.submit(_corpus_matrix, (seed, n_min, n_max))))
            if len(pending) >= workers:
                break
        while pending:
            seed, fut = pending.popleft()
            nxt = next(it, None)
            if nxt is not None:
                pending.append((nxt, ex.submit(_corpus_matrix, (nxt, n_min, n_max))))
            A, spec = fut.result()
            yield seed, A, spec


def sweep(seeds, db_path: str, p_list=(4, 8), n_min=1e5, n_max=1e6, log=print, workers=0,
          time_limit=None):
    """Exhaustive sweep over ``config_grid()`` for every seed not yet in the
    database; appends records and flushes after every matrix.  ``workers``
    processes generate the next matrices meanwhile.  With ``time_limit``
    (seconds) no new matrix is started once that much time has passed; a
    later call with the same database continues where this one stopped."""
    start = time.time()
    import torch

    done = set()
    if os.path.exists(db_path):
        with open(db_path) as fh:
            for line in fh:
                done.add(json.loads(line)["seed"])
    dev = torch.device("cuda:0")
    grid = config_grid()
    t0 = time.time()
    for seed, A, spec in _corpus([s for s in seeds if s not in done], n_min, n_max, workers):
        if time_limit is not None and time.time() - start > time_limit:
            log(f"time limit reached before seed {seed}")
            break
        plan = Plan(A, max(p_list), 256 << 20, root_mode=1)
        perm = plan.arrays()[0].astype(np.int64)
        x = np.random.default_rng(seed).uniform(-1, 1, A.n)
        X = torch.from_numpy(np.ascontiguousarray(x[perm])).to(dev)
        recs = []
        for p in p_list:
            Y = torch.empty((p, A.n), dtype=torch.float64, device=dev)
            _apply(plan, p, DEFAULT)
            feats = plan_features(plan).tolist()
            for c in grid:
                _apply(plan, p, c)
                ms = time_run(torch, plan, X, Y)
                recs.append({"seed": seed, "spec": spec, "p": p, "features": feats, "config": c,
                             "ms": round(ms, 5), "groups": plan.info()["n_groups"]})
            del Y
        with open(db_path, "a") as fh:
            for r in recs:
                fh.write(json.dumps(r) + "\n")
        best = min(r["ms"] for r in recs if r["p"] == max(p_list))
        dflt = [r["ms"] for r in recs if r["p"] == max(p_list) and r["config"] == DEFAULT][0]
        log(f"seed {seed} {spec['family']} n={spec['n']} nnz={spec['nnz']}: default {dflt:.3f} ms, "
            f"best {best:.3f} ms ({time.time() - t0:.1f}s)")
        t0 = time.time()
        del plan, X, A


def load_db(path: str):
    """Records from a sweep database, either one line per (matrix, p,
    configuration) as ``sweep`` writes it, or the compact form of
    ``compact_db`` (one line per (matrix, p) with the times of every
    configuration of ``config_grid()`` in order)."""
    import gzip

    opener = gzip.open if path.endswith(".gz") else open
    out = []
    grid = config_grid()
    with opener(path, "rt") as fh:
        for line in fh:
            r = json.loads(line)
            if "times_ms" in r:
                if len(r["times_ms"]) != len(grid):
                    raise ValueError(f"{path}: {len(r['times_ms'])} timings per case, the grid has {len(grid)}")
                for c, ms in zip(grid, r["times_ms"]):
                    out.append({"seed": r["seed"], "spec": r["spec"], "p": r["p"], "features": r["features"],
                                "config": c, "ms": ms})
            else:
                out.append(r)
    return out


def compact_db(records, path: str):
    """Write records as one line per (matrix, p), times in config_grid() order."""
    keys = [json.dumps(c, sort_keys=True) for c in config_grid()]
    with open(path, "w") as fh:
        for (seed, p), g in sorted(_group(records).items()):
            t = {json.dumps(r["config"], sort_keys=True): r["ms"] for r in g}
            fh.write(json.dumps({"seed": seed, "p": p, "spec": g[0]["spec"], "features": g[0]["features"],
                                 "times_ms": [t[k] for k in keys]}) + "\n")


def split_seeds(records, test_fraction=0.2):
    """Deterministic train / held-out split by matrix seed (every fifth seed held out)."""
    seeds = sorted({r["seed"] for r in records})
    k = max(1, int(round(1 / test_fraction)))
    test = {s for i, s in enumerate(seeds) if i % k == k - 1}
    return [r for r in records if r["seed"] not in test], [r for r in records if r["seed"] in test]


# ----------------------------------------------------------------------------
# the network on the device
# ----------------------------------------------------------------------------

class DeviceMLP:
    """z1 = W1 x + b1 -> relu -> W2 . + b2 -> relu -> w3 . + b3, FP32 on the GPU.

    Forward, backward and Adam are the library's kernels; the buffers are
    torch tensors on cuda:0."""

    def __init__(self, D: int, H: int = 64, seed: int = 0, params=None):
        import torch

        self.torch = torch
        self.D, self.H = int(D), int(H)
        self.n = int(lib().mpk_mlp_param_count(self.D, self.H))
        dev = torch.device("cuda:0")
        if params is None:
            rng = np.random.default_rng(seed)
            p = np.zeros(self.n, np.float32)
            o = 0
            for fan_in, rows, cols in ((self.D, self.H, self.D), (self.H, self.H, self.H)):
                w = rng.normal(0, math.sqrt(2.0 / fan_in), size=rows * cols)
                p[o:o + w.size] = w
                o += w.size + rows  # weights, then zero biases
            p[o:o + self.H] = rng.normal(0, math.sqrt(1.0 / self.H), size=self.H)
            params = p
        self.P = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(dev)
        self.M = torch.zeros_like(self.P)
        self.V = torch.zeros_like(self.P)
        self.G = torch.zeros_like(self.P)
        self.step = 0
        self._bufs = {}

    def _buffers(self, B):
        if B not in self._bufs:
            t = self.torch
            dev = self.P.device
            self._bufs = {B: (t.empty(B, dtype=t.float32, device=dev),
                              t.empty((B, 2 * self.H), dtype=t.float32, device=dev),
                              t.empty(B * (2 * self.H + 1), dtype=t.float32, device=dev),
                              t.empty(1, dtype=t.float32, device=dev))}
        return self._bufs[B]

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.P.device, dtype=t.float32).contiguous()
        return t.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.P.device)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(int(t.data_ptr()))

    def _stream(self):
        return ctypes.c_void_p(int(self.torch.cuda.current_stream().cuda_stream))

    def forward_dev(self, Xd):
        B = int(Xd.shape[0])
        out, cache, _, _ = self._buffers(B)
        check(lib().mpk_mlp_forward(self._p(self.P), self.D, self.H, self._p(Xd), B, self._p(out),
                                    self._p(cache), self._stream()))
        return out, cache

    def predict(self, X) -> np.ndarray:
        out, _ = self.forward_dev(self._dev(X))
        return out.cpu().numpy().astype(np.float64)

    def gradient_dev(self, Xd, yd):
        B = int(Xd.shape[0])
        out, cache, work, loss = self._buffers(B)
        self.forward_dev(Xd)
        check(lib().mpk_mlp_backward(self._p(self.P), self.D, self.H, self._p(Xd), self._p(yd), B, self._p(out),
                                     self._p(cache), self._p(work), self._p(self.G), self._p(loss), self._stream()))
        return self.G, loss

    def gradient(self, X, y):
        g, loss = self.gradient_dev(self._dev(X), self._dev(y))
        return g.cpu().numpy().astype(np.float64), float(loss.cpu().numpy()[0])

    def adam(self, g=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        if g is not None and not isinstance(g, self.torch.Tensor):
            self.G.copy_(self._dev(g))
        self.step += 1
        check(lib().mpk_mlp_adam(self._p(self.P), self._p(self.G), self._p(self.M), self._p(self.V), self.n,
                                 ctypes.c_float(lr), ctypes.c_float(beta1), ctypes.c_float(beta2),
                                 ctypes.c_float(eps), self.step, self._stream()))

    def train(self, X, y, steps=2000, lr=3e-3):
        Xd, yd = self._dev(X), self._dev(y)
        for _ in range(steps):
            self.gradient_dev(Xd, yd)
            self.adam(None, lr=lr)
        _, loss = self.gradient_dev(Xd, yd)
        return float(loss.cpu().numpy()[0])

    def params(self) -> np.ndarray:
        return self.P.cpu().numpy().astype(np.float64)


# ----------------------------------------------------------------------------
# learned tuner (cost model)
# ----------------------------------------------------------------------------

def _group(records):
    by = {}
    for r in records:
        by.setdefault((r["seed"], r["p"]), []).append(r)
    return by


class LearnedTuner:
    """features(matrix, p) + encoding(config) -> log(t / t_default)."""

    def __init__(self, hidden: int = 64, seed: int = 0):
        self.hidden = hidden
        self.seed = seed
        self.net = None
        self.mu = None
        self.sd = None

    def _inputs(self, feats, configs):
        f = (np.asarray(feats, np.float64) - self.mu) / self.sd
        return np.stack([np.concatenate([f, encode_config(c)]) for c in configs])

    def fit(self, records, steps=6000, lr=3e-3):
        groups = _group(records)
        F = np.array([g[0]["features"] for g in groups.values()], np.float64)
        self.mu = F.mean(0)
        self.sd = F.std(0) + 1e-6
        X, y = [], []
        for g in groups.values():
            tdef = [r["ms"] for r in g if r["config"] == DEFAULT][0]
            X.append(self._inputs(g[0]["features"], [r["config"] for r in g]))
            y.extend(math.log(r["ms"] / tdef) for r in g)
        X = np.concatenate(X)
        y = np.array(y)
        self.net = DeviceMLP(X.shape[1], self.hidden, seed=self.seed)
        return self.net.train(X, y, steps=steps, lr=lr)

    def choose(self, features, configs=None):
        return self.shortlist(features, 1, configs)[0]

    def shortlist(self, features, m, configs=None):
        """The m configurations with the smallest predicted time, best first."""
        configs = configs or config_grid()
        pred = self.net.predict(self._inputs(features, configs))
        return [configs[int(i)] for i in np.argsort(pred, kind="stable")[:m]]

    def tune(self, torch, plan: Plan, p: int, run, m: int = 3, **fixed):
        """Learned choice checked by measurement: the plan's features (taken
        at the default configuration, as in the sweep), the model's m best
        configurations, then ``autotune`` over those m on the caller's run.
        m = 1 is the model alone; m = len(config_grid()) is the exhaustive
        sweep.  Returns what ``autotune`` returns."""
        _apply(plan, p, DEFAULT, nrhs=int(fixed.get("nrhs", 1)))
        feats = plan_features(plan)
        return autotune(torch, plan, p, self.shortlist(feats, m), run, **fixed)


def best_static(records):
    """The one configuration with the smallest geometric-mean time relative
    to the default over the given records (the tuner without features)."""
    keys = [json.dumps(c, sort_keys=True) for c in config_grid()]
    logs = {k: [] for k in keys}
    for g in _group(records).values():
        t = {json.dumps(r["config"], sort_keys=True): r["ms"] for r in g}
        tdef = t[json.dumps(DEFAULT, sort_keys=True)]
        for k in keys:
            logs[k].append(math.log(t[k] / tdef))
    best = min(keys, key=lambda k: np.mean(logs[k]))
    return json.loads(best)


def evaluate(tuner: LearnedTuner, records, static=None, shortlist=(3,)):
    """Held-out quality: the measured time of the chosen configuration against
    the sweep's best, the untuned default and (if given) one static
    configuration, per (matrix, p); for every m in ``shortlist``, the same for
    the fastest (by the recorded times) of the model's m best configurations,
    which is what ``LearnedTuner.tune`` measures."""
    ratios, gains, within, sgains = [], [], 0, []
    short = {m: [] for m in shortlist}
    groups = _group(records)
    for g in groups.values():
        cfgs = [r["config"] for r in g]
        ranked = tuner.shortlist(g[0]["features"], max((1,) + tuple(shortlist)), cfgs)
        cfg = ranked[0]
        t = {json.dumps(r["config"], sort_keys=True): r["ms"] for r in g}
        tpick = t[json.dumps(cfg, sort_keys=True)]
        tbest = min(t.values())
        tdef = t[json.dumps(DEFAULT, sort_keys=True)]
        ratios.append(tpick / tbest)
        gains.append(tdef / tpick)
        within += tpick <= 1.05 * tbest
        for m in shortlist:
            short[m].append(min(t[json.dumps(c, sort_keys=True)] for c in ranked[:m]) / tbest)
        if static is not None:
            sgains.append(tdef / t[json.dumps(static, sort_keys=True)])
    n = len(groups)
    out = {"cases": n,
           "geomean_pick_over_best": float(np.exp(np.mean(np.log(ratios)))),
           "within_5pct_of_best": within / max(n, 1),
           "geomean_gain_over_default": float(np.exp(np.mean(np.log(gains)))),
           "geomean_best_gain_over_default": float(np.exp(np.mean(np.log(
               [[r["ms"] for r in g if r["config"] == DEFAULT][0] / min(r["ms"] for r in g)
                for g in groups.values()]))))}
    for m, v in short.items():
        out[f"shortlist{m}_geomean_over_best"] = float(np.exp(np.mean(np.log(v))))
        out[f"shortlist{m}_within_5pct_of_best"] = float(np.mean(np.array(v) <= 1.05))
    if static is not None:
        out["static_config"] = static
        out["geomean_static_gain_over_default"] = float(np.exp(np.mean(np.log(sgains))))
        # the per-matrix choice against the one best static configuration
        out["gain_over_best_static"] = out["geomean_gain_over_default"] / out["geomean_static_gain_over_default"]
        for m in shortlist:
            out[f"shortlist{m}_gain_over_best_static"] = (out["geomean_best_gain_over_default"]
                                                         / out[f"shortlist{m}_geomean_over_best"]
                                                         / out["geomean_static_gain_over_default"])
    return out


def main(argv=None):
    """``sweep FIRST LAST OUT [--n-max N] [--workers W] [--time-limit S]``:
    time every configuration on the corpus seeds FIRST..LAST-1 (GPU),
    appending to OUT (seeds already in OUT are skipped).
    ``compact OUT IN...``: merge sweep files into the compact database."""
    import argparse

    ap = argparse.ArgumentParser(prog="python -m paper_2205_01598_amd.tune")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s1 = sub.add_parser("sweep")
    s1.add_argument("first", type=int)
    s1.add_argument("last", type=int)
    s1.add_argument("out")
    s1.add_argument("--n-max", type=float, default=1e7)
    s1.add_argument("--workers", type=int, default=2)
    s1.add_argument("--time-limit", type=float, default=None)
    s2 = sub.add_parser("compact")
    s2.add_argument("out")
    s2.add_argument("inputs", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "sweep":
        sweep(range(a.first, a.last), a.out, n_max=a.n_max, workers=a.workers, time_limit=a.time_limit,
              log=lambda m: print(m, flush=True))
    else:
        recs = []
        for f in a.inputs:
            recs.extend(load_db(f))
        compact_db(recs, a.out)
        print(f"{len({(r['seed'], r['p']) for r in recs})} (matrix, p) cases -> {a.out}")


if __name__ == "__main__":
    main()

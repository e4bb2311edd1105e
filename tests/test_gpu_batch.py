"""Batched form: many GA runs of uneven size in one persistent launch per
generation.  Every run must end exactly (bit for bit: best MSE, best genes,
final population, generation count) where the same configuration run alone
ends, given the tile width and row ranges the batch chose for it."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def bits(a, dt=np.uint32):
    return np.ascontiguousarray(a).view(dt)


def make_runs(specs, dtype="f32", extra=None):
    """specs: (task, N, F, D, P, max_generations, threshold, seed); extra:
    per-run dicts of further Config fields."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config
    runs = []
    for n, (task, N, F, D, P, G, thr, seed) in enumerate(specs):
        if task == "classification":
            X, t = synth.classification_dataset(N, F, seed=seed)
            basis = "trig"
        else:
            X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=seed)
            basis = "chebyshev"
        kw = extra[n] if extra else {}
        cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                     pop_size=P, max_generations=G, mse_threshold=thr, seed=seed + 1000, **kw)
        runs.append((cfg, dev(X, torch.float32), dev(t, torch.float32)))
    return runs


SPECS = [
    ("classification", 20011, 10, 6, 256, 9, 0.0, 1),
    ("regression", 3001, 5, 4, 64, 6, 0.0, 2),
    ("classification", 7777, 20, 8, 130, 11, 0.0, 3),   # M = 320: narrow tiles
    ("regression", 40000, 8, 8, 512, 5, 0.0, 4),
    ("regression", 1500, 12, 6, 33, 12, 0.0, 5),
    ("classification", 12345, 6, 4, 1000, 7, 0.0, 6),
]


def run_alone(cfg, X, t, tp, rg):
    from paper_1211_5481_amd import Config, Game
    g = Game(Config(**{**cfg.__dict__, "tile_p": tp, "row_groups": rg}), X, t)
    r = g.run()
    pop = host(g.population)
    st = g.state()
    g.close()
    return r, pop, st


def compare_with_alone(batch, runs, results):
    tps, rgs = batch.tiles()
    for i, (cfg, X, t) in enumerate(runs):
        assert tps[i] in (32, 64, 128) and rgs[i] >= 1
        ref, pop, st = run_alone(cfg, X, t, tps[i], rgs[i])
        got = results[i]
        label = f"run {i} tile {tps[i]} ranges {rgs[i]}"
        assert got["generations"] == ref["generations"], label
        assert got["stop_reason"] == ref["stop_reason"], label
        assert bits(np.float64(got["best_mse"]), np.uint64) == bits(np.float64(ref["best_mse"]), np.uint64), label
        assert np.array_equal(bits(got["best_genes"]), bits(ref["best_genes"])), label
        view = batch.context(i)
        assert np.array_equal(bits(host(view.population)), bits(pop)), label
        assert view.state()["generation"] == st["generation"], label


def test_batch_equals_runs_alone():
    from paper_1211_5481_amd import Batch
    runs = make_runs(SPECS)
    announce("batched f32 runs (tuned) vs the same runs alone")
    b = Batch(runs)
    results, lat = b.run(latency=True)
    compare_with_alone(b, runs, results)
    G = max(s[5] for s in SPECS)
    assert lat.shape == (len(SPECS), G)
    for i, s in enumerate(SPECS):
        bred = results[i]["generations"] - 1
        assert np.all(lat[i, :bred] > 0.0) and np.all(lat[i, bred:] == -1.0)
    b.close()


def test_batch_benchmark_geometry_equals_alone():
    """100 000 patterns, 1000 chromosomes in 8 tiles x 64 row ranges: the
    geometry whose ranges end on 32-row units with rotated extra units (the
    placement model prefers it to whole row tiles there), next to a run that
    keeps whole tiles; batched and alone must agree bit for bit."""
    from paper_1211_5481_amd import Batch, Config
    specs = [("classification", 100_000, 10, 6, 1000, 3, 0.0, 31),
             ("regression", 20000, 8, 6, 256, 3, 0.0, 32)]
    runs = make_runs(specs)
    fixed = [(128, 64), (64, 16)]
    runs = [(Config(**{**c.__dict__, "tile_p": tp, "row_groups": rg}), X, t)
            for (c, X, t), (tp, rg) in zip(runs, fixed)]
    announce("batched f32 runs at 100000 x 1000 (8 x 64 items) vs alone")
    b = Batch(runs)
    assert b.tiles() == ([f[0] for f in fixed], [f[1] for f in fixed])
    results = b.run()
    compare_with_alone(b, runs, results)
    b.close()


def test_batch_threshold_and_second_run():
    from paper_1211_5481_amd import Batch, Config, Game
    specs = [("regression", 5000, 6, 4, 128, 30, 0.0, 11),
             ("classification", 9000, 8, 4, 256, 30, 0.0, 12)]
    runs = make_runs(specs)
    # a threshold the first run reaches early: take its best MSE after 4 generations
    cfg0, X0, t0 = runs[0]
    probe = Game(Config(**{**cfg0.__dict__, "max_generations": 4}), X0, t0)
    thr = probe.run()["best_mse"] * (1.0 + 1e-5)   # summation order may differ by an ulp
    probe.close()
    runs[0] = (Config(**{**cfg0.__dict__, "mse_threshold": thr}), X0, t0)
    announce("batched runs with a threshold stop, run twice")
    b = Batch(runs)
    first = b.run()
    assert first[0]["stop_reason"] == "threshold" and first[0]["generations"] <= 4
    assert first[1]["generations"] == 30
    compare_with_alone(b, runs, first)
    # a second batched run continues every run like a second game_run would
    second = b.run()
    tps, rgs = b.tiles()
    for i, (cfg, X, t) in enumerate(runs):
        g = Game(Config(**{**cfg.__dict__, "tile_p": tps[i], "row_groups": rgs[i]}), X, t)
        g.run()
        r2 = g.run()
        assert r2["generations"] == second[i]["generations"]
        assert np.array_equal(bits(r2["best_genes"]), bits(second[i]["best_genes"]))
        assert np.array_equal(bits(host(g.population)), bits(host(b.context(i).population)))
        g.close()
    b.close()


def test_batch_fixed_tiles_and_bf16():
    from paper_1211_5481_amd import Batch, Config
    specs = [("classification", 6000, 16, 8, 300, 6, 0.0, 21),
             ("regression", 3000, 10, 6, 200, 8, 0.0, 22),
             ("classification", 2500, 5, 4, 64, 5, 0.0, 23)]
    runs = make_runs(specs, dtype="bf16")
    fixed = [(32, 5), (64, 2), (128, 1)]
    runs = [(Config(**{**c.__dict__, "tile_p": tp, "row_groups": rg}), X, t)
            for (c, X, t), (tp, rg) in zip(runs, fixed)]
    announce("batched bf16 runs with fixed tiles vs alone")
    b = Batch(runs)
    assert b.tiles() == ([f[0] for f in fixed], [f[1] for f in fixed])
    results = b.run()
    compare_with_alone(b, runs, results)
    assert b.time_fitness(reps=3) > 0.0
    b.close()


def test_full_batched_workload_sampled():
    """The 64-run batched workload at full size, one generation: for sampled
    runs the tracked best chromosome's MSE matches the float64 oracle, and no
    sampled chromosome of that population beats it."""
    torch = require_gpu()
    from oracle import model
    from paper_1211_5481_amd import Batch, Config
    specs = synth.batched_workload(64, synth.data_seed(4))
    runs, data = [], []
    for sp in specs:
        if sp["task"] == "classification":
            X, t = synth.classification_dataset(sp["n"], sp["f"], seed=sp["data_seed"])
        else:
            X, t, _ = synth.regression_dataset(sp["n"], sp["f"], 3, 0.05, seed=sp["data_seed"])
        cfg = Config(n_patterns=sp["n"], n_features=sp["f"], degree=sp["degree"], basis=sp["basis"],
                     task=sp["task"], dtype="f32", pop_size=sp["pop"], max_generations=1,
                     seed=synth.ga_seed(4) + sp["run"])
        runs.append((cfg, dev(X, torch.float32), dev(t, torch.float32)))
        data.append((X, t))
    announce("full batched workload, one generation")
    b = Batch(runs)
    results = b.run()
    cost = [sp["n"] * sp["f"] * sp["degree"] for sp in specs]
    order = np.argsort(cost)
    sample = [int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1])]
    rng = np.random.default_rng(0)
    for i in sample:
        sp, (X, t) = specs[i], data[i]
        Xo = X.astype(np.float32).astype(np.float64)
        to = t.astype(np.float32).astype(np.float64)
        Phi = model.design_matrix(Xo, sp["basis"], sp["degree"])
        best = results[i]["best_genes"].astype(np.float64)[None, :]
        ref = model.evaluate(Xo, to, best, sp["basis"], sp["degree"], sp["task"], Phi=Phi)["mse"][0]
        assert abs(results[i]["best_mse"] - ref) <= 1e-5 * ref, f"run {i}"
        pop = host(b.context(i).population)
        rows = rng.choice(pop.shape[0], 16, replace=False)
        mse = model.evaluate(Xo, to, pop[rows].astype(np.float64), sp["basis"], sp["degree"],
                             sp["task"], Phi=Phi)["mse"]
        assert mse.min() >= ref * (1 - 2e-5), f"run {i}"
    b.close()


def test_batch_with_immigrants_and_shared_model_equals_runs_alone():
    """Runs with random immigrants, the shared-coefficient model and a bias
    gene batch like any other run."""
    from paper_1211_5481_amd import Batch
    extra = [dict(n_immigrants=20), dict(shared=1, bias=1), dict(shared=1, n_immigrants=5),
             dict(bias=1), {}, dict(n_immigrants=100)]
    runs = make_runs(SPECS, extra=extra)
    announce("batched runs with immigrants / shared model vs alone")
    b = Batch(runs)
    results = b.run()
    compare_with_alone(b, runs, results)
    b.close()


def test_batch_with_wheel_selection_equals_runs_alone():
    """Roulette and ranking runs in a batch (each builds its wheel or rank
    order before the batched breed) equal the same runs alone."""
    from paper_1211_5481_amd import Batch
    extra = [dict(selection="roulette"), dict(selection="ranking"), {},
             dict(selection="ranking", n_immigrants=10), dict(selection="roulette", bias=1), {}]
    runs = make_runs(SPECS, extra=extra)
    announce("batched roulette / ranking runs vs alone")
    b = Batch(runs)
    results = b.run()
    compare_with_alone(b, runs, results)
    b.close()


def test_batch_runs_progress_at_their_own_pace():
    """A small run next to a large one: each run's generations take about its
    own work (the small run does not wait for the large one's generation),
    and both still equal the same runs alone."""
    from paper_1211_5481_amd import Batch
    specs = [("classification", 200_000, 12, 6, 1024, 12, 0.0, 41),
             ("regression", 2000, 5, 4, 64, 12, 0.0, 42)]
    runs = make_runs(specs)
    announce("batched large + small run: per-run generation latency")
    b = Batch(runs)
    results, lat = b.run(latency=True)
    compare_with_alone(b, runs, results)
    big = np.median(lat[0, :11])
    small = np.median(lat[1, :11])
    print(f"median generation latency: large {big:.1f} us, small {small:.1f} us")
    assert small > 0.0 and big > 0.0
    assert small < 0.5 * big, (small, big)
    b.close()


def test_batch_longer_than_one_launch_equals_alone():
    """More generations than one scheduler launch breeds (128): the runs
    resume in the next launch exactly where they stopped."""
    from paper_1211_5481_amd import Batch
    specs = [("regression", 1500, 4, 4, 40, 300, 0.0, 51),
             ("classification", 3000, 6, 4, 96, 170, 0.0, 52),
             ("regression", 800, 3, 6, 32, 129, 0.0, 53)]
    runs = make_runs(specs, extra=[dict(selection="ranking"), {}, dict(selection="roulette")])
    announce("batched runs over three scheduler launches vs alone")
    b = Batch(runs)
    results, lat = b.run(latency=True)
    compare_with_alone(b, runs, results)
    for i, s in enumerate(specs):
        assert results[i]["generations"] == s[5]
        assert np.all(lat[i, :s[5] - 1] > 0.0)
    b.close()


def test_batch_tuner_cache_reuses_choices():
    """A second batch of runs with the same shapes takes the tuner's cached
    per-run choices (same tile widths and row ranges) and still equals the
    runs alone."""
    import time
    from paper_1211_5481_amd import Batch
    specs = [("classification", 30011, 12, 6, 512, 4, 0.0, 61),
             ("regression", 9000, 7, 4, 256, 4, 0.0, 62),
             ("classification", 4000, 5, 8, 96, 4, 0.0, 63)]
    runs = make_runs(specs)
    announce("batched tuner, then a batch of the same shapes from its cache")
    t0 = time.perf_counter()
    b1 = Batch(runs)
    t1 = time.perf_counter()
    tiles1 = b1.tiles()
    b1.close()
    t2 = time.perf_counter()
    b2 = Batch(runs)
    t3 = time.perf_counter()
    assert b2.tiles() == tiles1
    print(f"tuned init {t1 - t0:.3f} s, cached init {t3 - t2:.3f} s")
    results = b2.run()
    compare_with_alone(b2, runs, results)
    b2.close()


def test_batch_stall_is_reported_and_poisons(monkeypatch):
    """The scheduler's bounded wait, forced from the host: with a 1 us idle
    bound the workgroups that find nothing to do give up at once (every
    kernel still ends normally); the run reports the stall and the batch
    refuses further work."""
    from paper_1211_5481_amd import Batch
    from paper_1211_5481_amd._lib import GameError
    specs = [("regression", 3000, 4, 4, 64, 40, 0.0, 71)]
    runs = make_runs(specs)
    cfg = runs[0][0]
    runs = [(type(cfg)(**{**cfg.__dict__, "tile_p": 64, "row_groups": 1}), runs[0][1], runs[0][2])]
    monkeypatch.setenv("GAME_FLOW_IDLE_US", "1")
    announce("batched scheduler with a 1 us idle bound: stall reported")
    b = Batch(runs)
    with pytest.raises(GameError, match="no open item"):
        b.run()
    with pytest.raises(GameError, match="poisoned"):
        b.run()
    b.close()

"""Training driver: graph-replayed generations, stop conditions, determinism."""
import numpy as np
import pytest

from oracle import ga, model
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def c1_game(**kw):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    X, t, _ = synth.regression_dataset(1000, 8, 4, 0.05, seed=synth.data_seed(1))
    base = dict(n_patterns=1000, n_features=8, degree=4, basis="chebyshev", task="regression",
                dtype="f64", pop_size=20, max_generations=50, seed=synth.ga_seed(1))
    base.update(kw)
    cfg = Config(**base)
    return Game(cfg, dev(X, cfg.io_dtype), dev(t, cfg.io_dtype)), cfg, X, t


def test_c1_run_to_max_generations():
    announce("c1 game_run 50 generations f64")
    g, cfg, X, t = c1_game()
    res = g.run()
    assert res["stop_reason"] == "max_generations" and res["generations"] == 50
    ref = model.evaluate(X, t, res["best_genes"].astype(np.float64), "chebyshev", 4, "regression")
    assert abs(ref["mse"][0] - res["best_mse"]) <= 1e-12 * ref["mse"][0]
    assert res["best_fitness"] == 1.0 - res["best_mse"]
    st = g.state()
    assert st["generation"] == 49 and st["stopped"]
    # with elitism the best chromosome seen is in the final population
    pop = host(g.population).astype(np.float64)
    r = model.evaluate(X, t, pop, "chebyshev", 4, "regression")
    assert abs(r["mse"].min() - res["best_mse"]) <= 1e-12 * res["best_mse"]
    g.close()


def test_threshold_stops_after_first_generation():
    announce("threshold stop")
    g, cfg, X, t = c1_game(mse_threshold=1e6)
    res = g.run()
    assert res["stop_reason"] == "threshold" and res["generations"] == 1
    g.close()


def test_graph_replay_equals_eager_steps_and_oracle():
    torch = require_gpu()
    announce("advance vs eager")
    a, cfg, X, t = c1_game(dtype="f32", pop_size=64)
    b, _, _, _ = c1_game(dtype="f32", pop_size=64)
    pop0 = host(a.population)
    a.advance(11)                          # one 8-generation graph + a 3-generation graph
    a.prepare(5)                           # replaces the remainder graph, runs nothing
    assert a.state()["generation"] == 11
    a.advance(5)                           # a 5-generation remainder graph
    a.advance(3)                           # a 3-generation one again
    for _ in range(19):
        b.eval_fitness()
        b.step()
    pa, pb = host(a.population), host(b.population)
    assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32))
    assert a.state()["generation"] == 19
    # replay the first generation on the oracle from the device's own fitness vector
    c, _, _, _ = c1_game(dtype="f32", pop_size=64)
    _, _, fit = c.eval_fitness()
    c.step()
    want = ga.ga_step(pop0, host(fit), 0, cfg.seed)
    assert np.array_equal(host(c.population).view(np.uint32), want.view(np.uint32))
    for gme in (a, b, c):
        gme.close()


def test_best_fitness_never_decreases_and_runs_repeat():
    announce("monotone best + determinism")
    g, cfg, X, t = c1_game(dtype="f32", pop_size=50)
    best = -np.inf
    for gen in range(20):
        _, _, fit = g.eval_fitness()
        f = host(fit)
        assert f.max() >= best
        best = f.max()
        g.step()
    h, _, _, _ = c1_game(dtype="f32", pop_size=50)
    h.advance(20)
    assert np.array_equal(host(g.population).view(np.uint32), host(h.population).view(np.uint32))
    g.close()
    h.close()


def test_set_population_then_first_run_uses_the_new_population():
    """A context whose first graph is built after set_population evaluates the
    population it was given (the stale gene tile is repacked)."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    X, t = synth.classification_dataset(4000, 5, seed=8)
    cfg = Config(n_patterns=4000, n_features=5, degree=3, basis="trig", task="classification",
                 dtype="f32", pop_size=64, max_generations=1, seed=5)
    a = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    announce("set_population then run")
    mse_a = host(a.eval_fitness()[0])
    b = Game(Config(**{**cfg.__dict__, "seed": 6}), dev(X, torch.float32), dev(t, torch.float32))
    b.population = a.population.clone()
    r = b.run()
    assert r["generations"] == 1 and r["best_mse"] == mse_a.min()
    a.close()
    b.close()


def test_paper_settings_run():
    """The settings of the paper's experiment (Sec. 5): polytrigo expansion,
    rank-based roulette selection, crossover 0.9, mutation 0.2, two elites,
    MSE threshold 0.001, on a 2100-pattern, 7-feature two-class set (the
    paper's data size); population B*F + 1 (eq. 4).  The best fitness never
    decreases and the run ends by one of its two stop rules."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    X, t = synth.classification_dataset(2100, 7, seed=21)
    for D in (1, 2, 4, 8):
        cfg = Config(n_patterns=2100, n_features=7, degree=D, basis="trig", task="classification",
                     dtype="f32", pop_size=0, elitism=2, selection="ranking", p_crossover=0.9,
                     p_mutation=0.2, mse_threshold=0.001, max_generations=300, seed=D)
        g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
        assert g.P == 2 * 7 + 1
        announce(f"paper settings D={D}")
        best = []
        for _ in range(40):
            g.advance(1)
            best.append(float(np.nanmax(host(g.eval_fitness()[2]))))  # this generation's best
        assert all(b1 >= b0 for b0, b1 in zip(best, best[1:]))
        r = g.run()
        assert r["stop_reason"] in ("threshold", "max_generations")
        assert 0.0 <= r["best_miscls"] <= 1.0 and r["best_mse"] <= 1.0 - best[0] + 1e-12
        g.close()

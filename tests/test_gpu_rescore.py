"""Float32 re-score of the 16-bit forms' elites against the float64 oracle
(tolerance 1e-5 relative, the float32 gate)."""
import numpy as np
import pytest

from oracle import model
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def oracle_mse(X, t, G, basis, D, task, bias=0):
    Xo = X.astype(np.float32).astype(np.float64)
    to = t.astype(np.float32).astype(np.float64)
    return model.evaluate(Xo, to, G.astype(np.float64), basis, D, task, bias)


@pytest.mark.parametrize("dtype,basis,task,bias", [
    ("bf16", "legendre", "classification", 0),
    ("f16", "trig", "regression", 1),
    ("f32", "chebyshev", "classification", 1),
])
def test_rescore_explicit_genes(dtype, basis, task, bias):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 20011, 6, 5, 64
    if task == "classification":
        X, t = synth.classification_dataset(N, F, seed=3)
    else:
        X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=3)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                 bias=bias, pop_size=P)
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    G = synth.random_population(5, g.L, seed=9)
    announce(f"rescore explicit {dtype} {basis} {task}")
    mse, mis = (host(a) for a in g.rescore(dev(G, torch.float32)))
    ref = oracle_mse(X, t, G, basis, D, task, bias)
    np.testing.assert_allclose(mse, ref["mse"], rtol=1e-5)
    if task == "classification":
        np.testing.assert_allclose(mis, ref["miscls"], atol=3.0 / N)
    # deterministic
    again = host(g.rescore(dev(G, torch.float32))[0])
    assert np.array_equal(again, mse)
    g.close()


def test_rescore_counts_one_to_eight_agree():
    """The re-score kernel is compiled per chromosome count (1..8): a set of
    eight scored together gives, bit for bit, what each scored alone gives
    (a chromosome's sums do not depend on its neighbours), and matches the
    oracle."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 9000, 5, 6, 32
    X, t = synth.classification_dataset(N, F, seed=13)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", task="classification",
                 dtype="bf16", bias=1, pop_size=P)
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    G = synth.random_population(8, g.L, seed=17)
    announce("rescore counts 1..8")
    all_mse, all_mis = (host(a) for a in g.rescore(dev(G, torch.float32)))
    ref = oracle_mse(X, t, G, "legendre", D, "classification", 1)
    np.testing.assert_allclose(all_mse, ref["mse"], rtol=1e-5)
    for n in range(1, 8):
        mse, mis = (host(a) for a in g.rescore(dev(G[:n], torch.float32)))
        assert np.array_equal(mse, all_mse[:n]), n
        assert np.array_equal(mis, all_mis[:n]), n
    for i in range(8):
        mse, _ = (host(a) for a in g.rescore(dev(G[i:i + 1], torch.float32)))
        assert np.array_equal(mse, all_mse[i:i + 1]), i
    g.close()


def test_bf16_run_tracks_float32_mse_of_elites():
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 30000, 8, 6, 256
    X, t = synth.classification_dataset(N, F, seed=12)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", task="classification",
                 dtype="bf16", pop_size=P, rescore_top=2, max_generations=12, seed=4)
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    announce("bf16 run with float32 elite re-score")
    res = g.run()
    assert res["generations"] == 12 and res["stop_reason"] == "max_generations"
    ref = oracle_mse(X, t, res["best_genes"][None, :], "legendre", D, "classification")
    assert abs(ref["mse"][0] - res["best_mse"]) <= 1e-5 * ref["mse"][0]
    # explicit re-score of the population's best agrees with the tracked value path
    mse, _ = g.rescore(n=2)
    assert host(mse).min() >= res["best_mse"] - 1e-12
    # a threshold on the float32 MSE stops the run exactly when reached
    h = Game(Config(**{**cfg.__dict__, "mse_threshold": res["best_mse"], "max_generations": 100}),
             dev(X, torch.float32), dev(t, torch.float32))
    r2 = h.run()
    assert r2["stop_reason"] == "threshold" and r2["generations"] <= 12
    assert r2["best_mse"] <= res["best_mse"]
    g.close()
    h.close()


def test_rescore_unsupported_for_f64():
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game, _lib
    cfg = Config(n_patterns=100, n_features=2, degree=2, dtype="f64", pop_size=8)
    g = Game(cfg, dev(np.zeros((100, 2)), torch.float64), dev(np.zeros(100), torch.float64))
    with pytest.raises(_lib.GameError) as ei:
        g.rescore(dev(np.zeros((1, g.L), np.float32), torch.float32))
    assert ei.value.status == _lib.GAME_E_UNSUPPORTED
    g.close()

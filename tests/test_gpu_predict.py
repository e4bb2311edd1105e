"""Test and validation use: predictions and quality metrics of a chromosome on
new patterns against the float64 oracle."""
import math

import numpy as np
import pytest

from oracle import model
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def data(task, n, F, seed):
    if task == "classification":
        return synth.classification_dataset(n, F, seed=seed)
    X, t, _ = synth.regression_dataset(n, F, 3, 0.05, seed=seed)
    return X, t


@pytest.mark.parametrize("dtype,basis,task,bias", [
    ("f64", "chebyshev", "regression", 1),
    ("f32", "trig", "classification", 0),
    ("bf16", "legendre", "classification", 1),
    ("f32", "power", "regression", 0),
])
def test_predict_and_metrics_match_oracle(dtype, basis, task, bias):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game, _lib
    F, D = 6, 4
    X, t = data(task, 5000, F, seed=1)
    Xv, tv = data(task, 3001, F, seed=2)          # held-out patterns
    cfg = Config(n_patterns=5000, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                 bias=bias, pop_size=64, max_generations=5, seed=9)
    io = cfg.io_dtype
    g = Game(cfg, dev(X, io), dev(t, io))
    with pytest.raises(_lib.GameError) as e:        # no best chromosome yet
        g.predict(dev(Xv, io))
    assert e.value.status == _lib.GAME_E_STATE
    announce(f"predict {dtype} {basis} {task}")
    g.run()
    best = g.state(with_genes=True)["best_genes"]
    Xo = Xv if dtype == "f64" else Xv.astype(np.float32).astype(np.float64)
    to = tv if dtype == "f64" else tv.astype(np.float32).astype(np.float64)
    want = model.predict(Xo, best.astype(np.float64), basis, D, task, bias)
    got = host(g.predict(dev(Xv, io)))
    np.testing.assert_allclose(got, want, rtol=1e-12 if dtype == "f64" else 1e-6, atol=1e-30)
    m = g.evaluate(dev(Xv, io), dev(tv, io))
    ref = model.metrics(Xo, to, best.astype(np.float64), basis, D, task, bias)
    assert m["n"] == 3001
    assert abs(m["mse"] - ref["mse"]) <= 1e-10 * ref["mse"]
    assert abs(m["rmse"] - ref["rmse"]) <= 1e-10 * ref["rmse"]
    for k in ("tp", "fp", "tn", "fn"):
        assert m[k] == ref[k], k
    for k in ("accuracy", "completeness", "contamination"):
        assert (math.isnan(m[k]) and math.isnan(ref[k])) or abs(m[k] - ref[k]) < 1e-15, k
    # an explicit chromosome, and repeatability
    G = synth.random_population(1, g.L, seed=4)[0]
    m2 = g.evaluate(dev(Xv, io), dev(tv, io), genes=dev(G, torch.float32))
    ref2 = model.metrics(Xo, to, G.astype(np.float64), basis, D, task, bias)
    assert abs(m2["mse"] - ref2["mse"]) <= 1e-10 * ref2["mse"]
    m3 = g.evaluate(dev(Xv, io), dev(tv, io), genes=dev(G, torch.float32))
    assert all(m3[k] == m2[k] or (math.isnan(m3[k]) and math.isnan(m2[k])) for k in m2)
    g.close()

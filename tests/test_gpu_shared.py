"""The shared-coefficient model (one coefficient per basis function for all
features, eq. 2 and eq. 7; B*d + 1 genes, eq. 5) on the GPU against the
float64 oracle: basis rows, fitness, a run with the paper's settings,
prediction and metrics, and the float32 re-score.  Tolerances are those of
the per-feature tests (f64 1e-12, f32 1e-5, 16-bit 2e-5 against the oracle on
the same rounded values)."""
import numpy as np
import pytest

from oracle import model
import synth
from tests.gpu_util import accumulation_bound, announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

RTOL = {"f64": 1e-12, "f32": 1e-5}


def as_io(a, dtype):
    return a if dtype == "f64" else a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("basis", ["trig", "legendre"])
def test_shared_basis_rows(basis, dtype):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, build_basis
    N, F, D = 1001, 7, 5
    X = np.random.default_rng(2).uniform(-1, 1, (N, F))
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, dtype=dtype, shared=1,
                 pop_size=4)
    io = torch.float64 if dtype == "f64" else torch.float32
    ref = model.design_matrix_shared(as_io(X, dtype), basis, D)
    M = ref.shape[1]
    announce(f"shared basis {basis} {dtype}")
    got = host(build_basis(cfg, dev(X, io), ld=M + 3).to(torch.float64))
    assert np.all(got[:, M:] == 0.0)
    got = got[:, :M]
    if dtype == "f64":
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    else:
        q = model.quantize(ref, dtype)
        ulp = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}[dtype]
        # the device sums in double by recurrences: a value a few 1e-15 from a
        # rounding boundary may round the other way
        assert np.all(np.abs(got - q) <= 2 * ulp * np.maximum(np.abs(q), 2.0 ** -14) + 1e-12)
        assert np.mean(got == q) > 0.999


@pytest.mark.parametrize("dtype,basis,task,bias,N,P", [
    ("f64", "trig", "classification", 1, 2100, 15),
    ("f32", "trig", "regression", 0, 3001, 200),
    ("f32", "chebyshev", "classification", 1, 129, 65),
    ("bf16", "legendre", "regression", 1, 5000, 130),
])
def test_shared_fitness(dtype, basis, task, bias, N, P):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    F, D = 7, 4
    if task == "classification":
        X, t = synth.classification_dataset(N, F, seed=N)
    else:
        X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=N)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                 bias=bias, shared=1, pop_size=P, seed=3)
    g = Game(cfg, dev(X, cfg.io_dtype), dev(t, cfg.io_dtype))
    K = (2 if basis == "trig" else 1) * D
    assert g.L == K + bias
    G = synth.random_population(P, g.L, seed=P)
    announce(f"shared fitness {dtype} {basis} {task} N={N} P={P}")
    mse, miscls, fit = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
    Xo, to, Go = as_io(X, dtype), as_io(t, dtype), G.astype(np.float32).astype(np.float64)
    Phi = model.design_matrix_shared(Xo, basis, D)
    if dtype in ("bf16", "f16"):
        Phi = model.quantize(Phi, dtype)
        Go[:, :K] = model.quantize(Go[:, :K], dtype)
    ref = model.evaluate(Xo, to, Go, basis, D, task, bias, Phi=Phi)
    if dtype in ("bf16", "f16"):
        bound = accumulation_bound(Phi, Go, ref, to, task, K)
        assert np.all(np.abs(mse - ref["mse"]) <= bound)
    else:
        np.testing.assert_allclose(mse, ref["mse"], rtol=RTOL[dtype], atol=0)
    assert np.array_equal(fit, 1.0 - mse)
    if task == "classification":
        z = ref["z"]
        near = (np.abs(z) <= 1e-4 * (np.abs(Phi) @ np.abs(Go[:, :K]).T + 1e-300)).sum(axis=0)
        assert np.all(np.abs(np.round(miscls * N) - np.round(ref["miscls"] * N)) <= near)
    g.close()


def test_shared_paper_settings_run_and_validation():
    """The paper's experiment settings with its literal chromosome: polytrigo
    expansion, 2d + 1 genes (eq. 5), population 2F + 1 (eq. 4), ranking
    selection, crossover 0.9, mutation 0.2, two elites; then the best
    chromosome's predictions and metrics on held-out patterns."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    X, t = synth.classification_dataset(2100, 7, seed=21)
    Xv, tv = synth.classification_dataset(900, 7, seed=22)
    D = 4
    cfg = Config(n_patterns=2100, n_features=7, degree=D, basis="trig", task="classification",
                 dtype="f32", bias=1, shared=1, pop_size=0, elitism=2, selection="ranking",
                 p_crossover=0.9, p_mutation=0.2, mse_threshold=0.001, max_generations=200,
                 seed=5)
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    assert g.P == 15 and g.L == model.paper_gene_count(D, 2) == 9
    announce("shared paper settings run")
    r = g.run()
    best = g.state(with_genes=True)["best_genes"].astype(np.float64)
    ref = model.evaluate(as_io(X, "f32"), as_io(t, "f32"), best[None, :], "trig", D,
                         "classification", 1, shared=True)
    assert abs(r["best_mse"] - ref["mse"][0]) <= 1e-5 * ref["mse"][0]
    pred = host(g.predict(dev(Xv, torch.float32)))
    want = model.predict(as_io(Xv, "f32"), best, "trig", D, "classification", 1, shared=True)
    np.testing.assert_allclose(pred, want, rtol=1e-6, atol=1e-30)
    m = g.evaluate(dev(Xv, torch.float32), dev(tv, torch.float32))
    mref = model.metrics(as_io(Xv, "f32"), as_io(tv, "f32"), best, "trig", D, "classification",
                         1, shared=True)
    assert abs(m["mse"] - mref["mse"]) <= 1e-10 * mref["mse"]
    for k in ("tp", "fp", "tn", "fn"):
        assert m[k] == mref[k], k
    g.close()


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_shared_rescore(dtype):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D = 20011, 9, 5
    X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=4)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="trig", task="regression",
                 dtype=dtype, bias=1, shared=1, pop_size=32)
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    G = synth.random_population(5, g.L, seed=8)
    announce(f"shared rescore {dtype}")
    mse, _ = (host(a) for a in g.rescore(dev(G, torch.float32)))
    ref = model.evaluate(as_io(X, "f32"), as_io(t, "f32"), G.astype(np.float64), "trig", D,
                         "regression", 1, shared=True)
    np.testing.assert_allclose(mse, ref["mse"], rtol=1e-5)
    g.close()

"""Fitness path (basis -> MFMA contraction -> fused error reduce) against the
float64 oracle.

Tolerances (relative, on the MSE of every chromosome):
  f64        1e-12  (double MFMA, double epilogue)
  f32        1e-5   (float32 MFMA and epilogue; double across row tiles)
  bf16/f16   against the oracle evaluated on the same rounded Phi and
             genes (isolates the float32 arithmetic): within the worst-case
             forward error bound of that arithmetic, per chromosome
             (accumulation_bound); the total error against the unrounded
             oracle is reported and only bounded loosely.
Misclassification counts: a pattern whose oracle output z lies within the
accumulation bound of the decision boundary z = 0 may fall either way; every
other pattern must be classified as the oracle does.  The bound, relative to
sum_m |Phi[n, m] G[m]|, is 1e-12 for f64 (double everywhere; the oracle's
closed-form basis and the device's recurrences differ by a few ulp of double)
and (M + 4) 2^-24 for the float32-accumulated forms (M rounded products added
in float32, plus the rounding of Phi to float32 for f32; for bf16/f16 the
reference already holds the rounded Phi and genes).  So the device's count
must lie between the oracle's misses among the far patterns and that number
plus the count of near ones.
"""
import numpy as np
import pytest

from oracle import model
import synth
from tests.gpu_util import accumulation_bound, announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

RTOL = {"f64": 1e-12, "f32": 1e-5}


def miss_window(dtype, M):
    """Relative distance to z = 0 within which the device may classify a
    pattern either way (see the module docstring)."""
    return 1e-12 if dtype == "f64" else (M + 4) * 2.0 ** -24


def make_data(task, N, F, seed):
    if task == "classification-soft":
        X, _ = synth.classification_dataset(N, F, seed=seed)
        return X, np.random.default_rng(seed).uniform(0.0, 1.0, N)
    if task == "classification":
        X, t = synth.classification_dataset(N, F, seed=seed)
    else:
        X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=seed)
    return X, t


def oracle_inputs(X, t, G, dtype):
    """The exact values the device sees: inputs cast to the I/O type."""
    if dtype == "f64":
        return X, t, G.astype(np.float64)
    return (X.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64),
            G.astype(np.float32).astype(np.float64))


def check_against_oracle(X, t, G, basis, D, task, bias, dtype, mse, miscls, fit, label=""):
    Xo, to, Go = oracle_inputs(X, t, G, dtype)
    Phi = model.design_matrix(Xo, basis, D)
    M = Phi.shape[1]
    if dtype in ("bf16", "f16"):
        Phi_r = model.quantize(Phi, dtype)
        G_r = Go.copy()
        G_r[:, :M] = model.quantize(Go[:, :M], dtype)
        ref = model.evaluate(Xo, to, G_r, basis, D, task, bias, Phi=Phi_r)
        total = model.evaluate(Xo, to, Go, basis, D, task, bias, Phi=Phi)
        rel_total = np.max(np.abs(mse - total["mse"]) / np.abs(total["mse"]))
        print(f"{label} {dtype}: max rel error of mse vs unrounded float64 oracle = {rel_total:.3e}")
        assert rel_total < (5e-2 if dtype == "bf16" else 1e-2)
        # the rounded inputs are exact on both sides: what remains is float32
        # arithmetic, bounded per chromosome (accumulation_bound)
        bound = accumulation_bound(Phi_r, G_r, ref, to, task, M)
        err = np.abs(mse - ref["mse"])
        assert np.all(err <= bound), (label, float(np.max(err / bound)))
    else:
        ref = model.evaluate(Xo, to, Go, basis, D, task, bias, Phi=Phi)
        np.testing.assert_allclose(mse, ref["mse"], rtol=RTOL[dtype], atol=0, err_msg=label)
    np.testing.assert_allclose(fit, 1.0 - mse, rtol=0, atol=0)
    N = len(t)
    if task == "classification":
        z = ref["z"]
        Gm = G_r[:, :M] if dtype in ("bf16", "f16") else Go[:, :M]
        scale = np.abs(Phi_r if dtype in ("bf16", "f16") else Phi) @ np.abs(Gm).T
        window = miss_window(dtype, M)
        near = np.abs(z) <= window * scale
        label1 = (to >= 0.5)[:, None]
        miss = (z >= 0.0) != label1
        far_miss = np.sum(miss & ~near, axis=0)
        cnt_got = np.round(miscls * N)
        n_near = near.sum(axis=0)
        assert np.all(cnt_got >= far_miss) and np.all(cnt_got <= far_miss + n_near), (
            label, window, int(np.max(n_near)))
    else:
        assert np.all(miscls == 0.0)


CASES = [
    # basis, dtype, task, bias, N, F, D, P
    ("chebyshev", "f64", "regression", 0, 1000, 8, 4, 20),
    ("power", "f64", "classification", 1, 333, 4, 2, 65),
    ("trig", "f32", "classification", 0, 3001, 10, 6, 300),
    ("legendre", "f32", "regression", 1, 777, 5, 3, 129),
    ("chebyshev", "f32", "regression", 0, 1, 2, 2, 3),
    ("chebyshev", "f32", "classification", 0, 129, 3, 3, 1),
    ("legendre", "bf16", "classification", 0, 2049, 16, 8, 257),
    ("legendre", "f16", "classification", 0, 2049, 16, 8, 257),
    ("trig", "bf16", "regression", 1, 1500, 10, 6, 200),
    ("chebyshev", "f16", "regression", 0, 500, 3, 5, 31),
    ("trig", "f32", "classification-soft", 1, 1000, 6, 4, 150),   # targets in [0, 1]
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_fitness_matches_oracle(case):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    basis, dtype, task, bias, N, F, D, P = case
    X, t = make_data(task, N, F, seed=N + F)
    task = task.replace("-soft", "")
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                 bias=bias, pop_size=P, elitism=min(2, P), seed=5)
    io = cfg.io_dtype
    announce(f"fitness {case}")
    g = Game(cfg, dev(X, io), dev(t, io))
    G = synth.random_population(P, g.L, seed=P)
    mse, miscls, fit = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
    check_against_oracle(X, t, G, basis, D, task, bias, dtype, mse, miscls, fit, label=str(case))
    # the population the library drew itself, through the genes=NULL path
    pop = host(g.population)
    mse2, miscls2, fit2 = (host(a) for a in g.eval_fitness())
    check_against_oracle(X, t, pop, basis, D, task, bias, dtype, mse2, miscls2, fit2, label="pop")
    # bit-reproducible
    again = host(g.eval_fitness()[0])
    assert np.array_equal(again.view(np.uint64), mse2.view(np.uint64))
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_alternating_populations_never_mix(dtype):
    """Two populations evaluated in turn, twelve times each: every evaluation
    equals that population's first bit for bit, so a launch's tail reads the
    partial rows of its own launch only (values the previous launch left in
    the same buffers would change the sums), and the first ones match the
    oracle."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 20_000, 10, 6, 1000
    X, t = synth.classification_dataset(N, F, seed=41)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="trig", task="classification",
                 dtype=dtype, pop_size=P, seed=43)
    announce(f"alternating populations {dtype} N={N} P={P}")
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    pops = [synth.random_population(P, g.L, seed=s) for s in (1, 2)]
    first = []
    for G in pops:
        mse, miscls, fit = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
        first.append((mse.copy(), miscls.copy()))
    check_against_oracle(X, t, pops[0], "trig", D, "classification", bool(cfg.bias), dtype,
                         first[0][0], first[0][1], 1.0 - first[0][0], label="population A")
    assert not np.array_equal(first[0][0], first[1][0])
    for _ in range(12):
        for G, (mse0, mis0) in zip(pops, first):
            mse, miscls, _ = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
            assert np.array_equal(mse.view(np.uint64), mse0.view(np.uint64))
            assert np.array_equal(miscls.view(np.uint64), mis0.view(np.uint64))
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_special_chromosomes(dtype):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D = 1000, 4, 3
    X, t = synth.classification_dataset(N, F, seed=21)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="chebyshev", task="classification",
                 dtype=dtype, pop_size=16)
    g = Game(cfg, dev(X, cfg.io_dtype), dev(t, cfg.io_dtype))
    G = np.zeros((3, g.L), dtype=np.float32)
    announce(f"special chromosomes {dtype}")
    mse, miscls, _ = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
    assert np.all(mse == 0.25)                       # sigmoid(0) = 1/2 on every pattern
    assert np.all(miscls == np.mean(t == 0.0))       # z = 0 predicts class 1
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_workload_c2_full_size_sampled(dtype):
    """100k patterns, 10 features, trig D=6, P=1000, sigmoid: the benchmarked shape."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 100_000, 10, 6, 1000
    X, t = synth.classification_dataset(N, F, seed=synth.data_seed(2))
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="trig", task="classification",
                 dtype=dtype, pop_size=P, seed=synth.ga_seed(2))
    announce(f"c2 full size {dtype}")
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    mse, miscls, fit = (host(a) for a in g.eval_fitness())
    pop = host(g.population)
    idx = np.concatenate([np.random.default_rng(2).choice(P, 62, replace=False), [0, P - 1]])
    check_against_oracle(X, t, pop[idx], "trig", D, "classification", 0, dtype, mse[idx],
                         miscls[idx], fit[idx], label="c2")
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_workload_c3_full_size_sampled(dtype):
    """1M patterns, 16 features, Legendre D=8 (128 genes), P=2048."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 1_000_000, 16, 8, 2048
    X, t = synth.classification_dataset(N, F, seed=synth.data_seed(3))
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", task="classification",
                 dtype=dtype, pop_size=P, seed=synth.ga_seed(3))
    announce(f"c3 full size {dtype}")
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    mse, miscls, fit = (host(a) for a in g.eval_fitness())
    pop = host(g.population)
    idx = np.concatenate([[0, 1, P - 1], np.random.default_rng(3).choice(
        np.arange(2, P - 1), 61, replace=False)])
    check_against_oracle(X, t, pop[idx], "legendre", D, "classification", 0, dtype, mse[idx],
                         miscls[idx], fit[idx], label="c3")
    g.close()


def test_workload_c3_first_10k_rows_precision():
    """The precision forms against the float64 oracle on the first 10 000
    rows of the 1M-pattern Legendre workload (whole population of 2048): the
    relative MSE error of FP32, BF16 and FP16 against the unrounded oracle is
    printed (max and median) and bounded; FP16, whose 11-bit significand
    holds every Phi and gene value in [-1, 1] more finely than BF16's 8, must
    be the closer of the two; and the FP32 re-score of the 16-bit runs'
    elites meets the FP32 tolerance."""
    torch = require_gpu()
    import json
    from paper_1211_5481_amd import Config, Game
    N_all, N, F, D, P = 1_000_000, 10_000, 16, 8, 2048
    X, t = synth.classification_dataset(N_all, F, seed=synth.data_seed(3))
    X, t = X[:N].copy(), t[:N].copy()
    Xo = X.astype(np.float32).astype(np.float64)
    to = t.astype(np.float32).astype(np.float64)
    stats = {}
    ref = None
    for dtype in ("f32", "bf16", "f16"):
        cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre",
                     task="classification", dtype=dtype, pop_size=P, seed=synth.ga_seed(3))
        announce(f"c3 first 10k rows, {dtype}")
        g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
        pop = host(g.population)
        mse_t, _, fit_t = g.eval_fitness()
        mse, fit = host(mse_t), host(fit_t)
        if ref is None:
            ref = model.evaluate(Xo, to, pop.astype(np.float64), "legendre", D,
                                 "classification")["mse"]
        rel = np.abs(mse - ref) / ref
        stats[dtype] = {"max": float(rel.max()), "median": float(np.median(rel))}
        if dtype != "f32":
            # the elites re-scored in float32 meet the float32 tolerance
            r_mse = host(g.rescore(None, 2)[0])
            order = np.lexsort((np.arange(P), -fit))   # fitness desc, index asc
            np.testing.assert_allclose(r_mse, ref[order[:2]], rtol=1e-5)
        g.close()
    print("precision c3 first 10k rows, relative MSE error vs float64 oracle: "
          + json.dumps(stats))
    assert stats["f32"]["max"] <= 1e-5
    assert stats["f16"]["max"] <= 1e-3 and stats["bf16"]["max"] <= 1e-2
    assert stats["f16"]["median"] < stats["bf16"]["median"]


TILE_CASES = [
    # basis, dtype, task, N, F, D, P, tile_p, row_groups
    ("legendre", "f32", "regression", 3001, 5, 3, 200, 32, 0),
    ("legendre", "f32", "regression", 3001, 5, 3, 200, 64, 7),
    ("legendre", "f32", "regression", 3001, 5, 3, 200, 128, 1),
    ("trig", "f32", "classification", 5000, 20, 8, 130, 0, 0),     # M = 320: 64-wide tiles
    ("trig", "f32", "classification", 5000, 20, 8, 130, 32, 3),
    ("legendre", "bf16", "classification", 4097, 16, 8, 300, 32, 5),
    ("legendre", "f16", "regression", 4097, 16, 8, 300, 64, 0),
]


@pytest.mark.parametrize("case", TILE_CASES, ids=lambda c: "-".join(map(str, c)))
def test_tile_widths_and_row_groups(case):
    """Every tile width and row split agrees with the oracle; a fixed
    (tile_p, row_groups) pair gives the same bits in a second context."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    basis, dtype, task, N, F, D, P, tp, rg = case
    X, t = make_data(task, N, F, seed=N + P)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                 pop_size=P, tile_p=tp, row_groups=rg, seed=3)
    announce(f"tile widths {case}")
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    G = synth.random_population(P, g.L, seed=P + 1)
    mse, miscls, fit = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
    check_against_oracle(X, t, G, basis, D, task, 0, dtype, mse, miscls, fit, label=str(case))
    h = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    again = host(h.eval_fitness(dev(G, torch.float32))[0])
    assert np.array_equal(again.view(np.uint64), mse.view(np.uint64))
    g.close()
    h.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_nan_and_saturating_chromosomes(dtype):
    """A NaN gene makes every output NaN: the MSE is NaN and, z >= 0 being
    false, every class-1 pattern counts as missed; a chromosome of huge genes
    saturates the sigmoid, so its error is exactly the share of patterns on
    the wrong side (oracle in float64, boundary patterns excepted)."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D = 1000, 4, 3
    X, t = synth.classification_dataset(N, F, seed=22)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="chebyshev", task="classification",
                 dtype=dtype, pop_size=16)
    g = Game(cfg, dev(X, cfg.io_dtype), dev(t, cfg.io_dtype))
    G = synth.random_population(3, g.L, seed=5)
    G[0, 3] = np.nan
    G[1] = np.sign(G[1]) * 1e20
    announce(f"nan / saturating chromosomes {dtype}")
    mse, miscls, fit = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
    lab1 = np.mean(t >= 0.5)
    assert np.isnan(mse[0]) and np.isnan(fit[0])
    assert miscls[0] == lab1
    Xo, to, Go = oracle_inputs(X, t, G, dtype)
    ref = model.evaluate(Xo, to, Go[1:2], "chebyshev", D, "classification")
    # saturated: each pattern's error is 0 or 1, so mse equals the miss rate
    assert abs(mse[1] - miscls[1]) <= 1.0 / N
    assert abs(miscls[1] - ref["miscls"][0]) <= 3.0 / N
    check_against_oracle(X, t, G[2:3], "chebyshev", D, "classification", 0, dtype, mse[2:3],
                         miscls[2:3], fit[2:3], label="finite")
    g.close()

"""The largest chromosome the library accepts (L = 4096 genes: 256 features,
trig D = 8) against the float64 oracle, on every dtype; the gene tile of
such a chromosome does not fit the LDS-staged kernel, so this covers the
streaming fitness kernel, the basis kernel's one-row blocks and the GA at
its widest rows."""
import numpy as np
import pytest

from oracle import ga, model
import synth
from tests.gpu_util import accumulation_bound, announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

RTOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_largest_chromosome(dtype):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    N, F, D, P = 613, 256, 8, 37
    X, t = synth.classification_dataset(N, F, seed=8)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="trig", task="classification",
                 dtype=dtype, pop_size=P, seed=12)
    g = Game(cfg, dev(X, cfg.io_dtype), dev(t, cfg.io_dtype))
    assert g.L == 4096
    G = synth.random_population(P, g.L, seed=3)
    announce(f"largest chromosome {dtype} L=4096 N={N} P={P}")
    mse, miscls, fit = (host(a) for a in g.eval_fitness(dev(G, torch.float32)))
    Xo = X if dtype == "f64" else X.astype(np.float32).astype(np.float64)
    to = t.astype(np.float64) if dtype == "f64" else t.astype(np.float32).astype(np.float64)
    Go = G.astype(np.float32).astype(np.float64)
    Phi = model.design_matrix(Xo, "trig", D)
    if dtype == "bf16":
        Phi = model.quantize(Phi, "bf16")
        Go = model.quantize(Go, "bf16")
    ref = model.evaluate(Xo, to, Go, "trig", D, "classification", Phi=Phi)
    if dtype == "bf16":
        bound = accumulation_bound(Phi, Go, ref, to, "classification", Phi.shape[1])
        assert np.all(np.abs(mse - ref["mse"]) <= bound)
    else:
        np.testing.assert_allclose(mse, ref["mse"], rtol=RTOL[dtype], atol=0)
    assert np.array_equal(fit, 1.0 - mse)
    # one GA step on the widest rows is bit-exact with the oracle's
    pop = host(g.population)
    f0 = host(g.eval_fitness()[2])
    want = ga.ga_step(pop, f0, 0, cfg.seed, elitism=cfg.elitism, k=cfg.tournament_k,
                      p_crossover=cfg.p_crossover, p_mutation=cfg.p_mutation,
                      sigma=cfg.mutation_sigma)
    g.step()
    assert np.array_equal(host(g.population).view(np.uint32), want.astype(np.float32).view(np.uint32))
    g.close()

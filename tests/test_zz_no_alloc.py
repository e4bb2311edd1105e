"""The allocation-free re-score (game_rescore_noalloc: no context, no
workspace, its scratch a fixed array inside the library) against
game_rescore on a context built from the same configuration and patterns,
bit for bit, over two calls in a row, the second with a smaller input (fewer
patterns and chromosomes), so that what the first call leaves in the shared
scratch cannot leak into the second; the first call's values also against
the float64 oracle.  And its argument checks, which launch nothing."""
import numpy as np
import pytest

from oracle import model
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # dtype, basis, task, bias, shared, F, D
    ("bf16", "legendre", "classification", 0, 0, 16, 8),
    ("f32", "trig", "regression", 1, 0, 6, 4),
    ("f16", "chebyshev", "classification", 1, 1, 5, 6),
]


def _data(task, N, F, seed):
    if task == "classification":
        return synth.classification_dataset(N, F, seed=seed)
    X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=seed)
    return X, t


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_noalloc_rescore_equals_context_rescore(case):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game, rescore_noalloc
    dtype, basis, task, bias, shared, F, D = case
    inputs = []
    for N, n, seed in ((50_000, 8, 1), (3001, 3, 2)):
        X, t = _data(task, N, F, seed)
        cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, task=task, dtype=dtype,
                     bias=bias, shared=shared, pop_size=16, seed=seed)
        Xd, td = dev(X, torch.float32), dev(t, torch.float32)
        g = Game(cfg, Xd, td)
        genes = dev(synth.random_population(n, g.L, seed=seed + 10), torch.float32)
        announce(f"context re-score {case} N={N} n={n}")
        want = tuple(host(a).copy() for a in g.rescore(genes))
        g.close()
        inputs.append((cfg, X, t, Xd, td, genes, want))
    got = []
    for cfg, _, _, Xd, td, genes, _ in inputs:      # two calls in a row, the second smaller
        announce(f"allocation-free re-score {case} N={cfg.n_patterns} n={genes.shape[0]}")
        got.append(tuple(host(a).copy() for a in rescore_noalloc(cfg, Xd, td, genes)))
    for (cfg, X, t, _, _, genes, want), (mse, mis) in zip(inputs, got):
        assert np.array_equal(mse.view(np.uint64), want[0].view(np.uint64)), cfg.n_patterns
        assert np.array_equal(mis.view(np.uint64), want[1].view(np.uint64)), cfg.n_patterns
    cfg, X, t, _, _, genes, _ = inputs[0]
    Xo = X.astype(np.float32).astype(np.float64)
    to = t.astype(np.float32).astype(np.float64)
    ref = model.evaluate(Xo, to, host(genes).astype(np.float64), basis, D, task, bias,
                         shared=bool(shared))
    np.testing.assert_allclose(got[0][0], ref["mse"], rtol=1e-5)


def test_noalloc_rescore_rejects_bad_arguments():
    torch = require_gpu()
    from paper_1211_5481_amd import Config, rescore_noalloc
    from paper_1211_5481_amd._lib import GAME_E_INVALID, GAME_E_UNSUPPORTED, GameError
    N, F, D = 100, 3, 2
    X, t = synth.classification_dataset(N, F, seed=3)
    Xd, td = dev(X, torch.float32), dev(t, torch.float32)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", task="classification",
                 dtype="f32", pop_size=16)
    announce("allocation-free re-score: argument checks")
    with pytest.raises(GameError) as e:                   # more chromosomes than the scratch holds
        rescore_noalloc(cfg, Xd, td, torch.zeros((9, F * D), dtype=torch.float32, device="cuda"))
    assert e.value.status == GAME_E_INVALID and "at most 8" in str(e.value)
    cfg64 = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", task="classification",
                   dtype="f64", pop_size=16)
    with pytest.raises(GameError) as e:
        rescore_noalloc(cfg64, Xd.double(), td.double(),
                        torch.zeros((2, F * D), dtype=torch.float32, device="cuda"))
    assert e.value.status == GAME_E_UNSUPPORTED

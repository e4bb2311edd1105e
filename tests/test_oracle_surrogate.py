"""Pins of the surrogate oracle (MLP, Adam, Spearman, selection rules) against
library routines, finite differences and closed forms."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ga, mlp, rank
import synth


def tiny_params(seed=0, L=5, H1=4, H2=3):
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, 0.7, (H1, L)), b1=rng.normal(0, 0.3, H1),
                W2=rng.normal(0, 0.7, (H2, H1)), b2=rng.normal(0, 0.3, H2),
                w3=rng.normal(0, 0.7, H2), b3=rng.normal(0, 0.3, 1))


def test_gelu_against_normal_cdf_and_derivative():
    a = np.linspace(-6, 6, 241)
    np.testing.assert_allclose(mlp.gelu(a), a * stats.norm.cdf(a), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(a), fd, rtol=1e-7, atol=1e-8)


def test_gradients_against_central_differences():
    p = tiny_params()
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (7, 5))
    y = rng.normal(0, 1, 7)
    loss, g = mlp.loss_and_grads(p, X, y)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        num = np.zeros_like(flat)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grads(p, X, y)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grads(p, X, y)
            flat[i] = old
            num[i] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(np.asarray(g[k]).reshape(-1), num, rtol=1e-4, atol=1e-8,
                                   err_msg=k)


def test_zero_weights_output_bias_and_first_adam_step():
    p = {k: np.zeros_like(v) for k, v in tiny_params().items()}
    p["b3"] = np.array([0.75])
    X = np.random.default_rng(2).uniform(-1, 1, (4, 5))
    np.testing.assert_array_equal(mlp.forward(p, X)["y"], np.full(4, 0.75))
    # first Adam step: m_hat = g, v_hat = g^2  ->  delta = -lr g / (|g| + eps)
    q = tiny_params(3)
    _, g = mlp.loss_and_grads(q, X, np.zeros(4))
    zeros = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in q.items()}
    new, _, _ = mlp.adam_step(q, g, zeros, zeros, 1, lr=1e-3)
    for k in q:
        gk = np.asarray(g[k], np.float64)
        np.testing.assert_allclose(new[k] - q[k], -1e-3 * gk / (np.abs(gk) + 1e-8), rtol=1e-9,
                                   atol=1e-15)


def test_he_uniform_init_statistics():
    p = mlp.init_params(128, 256, 256, seed=5)
    for k, fan in (("W1", 128), ("W2", 256)):
        w = p[k].astype(np.float64)
        bound = math.sqrt(6.0 / fan)
        assert np.abs(w).max() < bound
        assert abs(w.mean()) < 0.01 * bound
        assert abs(w.var() - bound ** 2 / 3) < 0.05 * bound ** 2 / 3
    assert np.all(p["b1"] == 0) and np.all(p["b2"] == 0) and p["b3"][0] == 0
    assert not np.array_equal(p["W1"], mlp.init_params(128, 256, 256, seed=6)["W1"])


def test_spearman_and_ranks_against_scipy():
    rng = np.random.default_rng(8)
    for n in (2, 7, 256, 1000):
        a = rng.integers(0, max(2, n // 4), n).astype(np.float64)   # many ties
        b = a + rng.normal(0, 2, n)
        np.testing.assert_allclose(rank.average_ranks(a), stats.rankdata(a), rtol=0, atol=0)
        assert abs(rank.spearman(a, b) - stats.spearmanr(a, b).statistic) < 1e-12
    assert rank.spearman(np.arange(10.0), np.arange(10.0) ** 3) == pytest.approx(1.0)
    assert rank.spearman(np.arange(10.0), -np.arange(10.0)) == pytest.approx(-1.0)


def test_smallest_k_against_lexsort():
    keys = np.random.default_rng(3).integers(0, 50, 500).astype(np.float64)
    order = np.lexsort((np.arange(500), keys))
    assert rank.smallest_k(keys, 123) == list(order[:123])


def test_minibatch_slots_range_and_spread():
    s = mlp.minibatch_slots(17, 4096, 50000, seed=3)
    assert s.min() >= 0 and s.max() < 50000
    assert stats.kstest(s / 50000.0, "uniform").pvalue > 1e-3
    assert not np.array_equal(s, mlp.minibatch_slots(18, 4096, 50000, seed=3))


def test_minibatch_recent_rows_come_from_latest_append():
    # ring of 1000 slots, full, latest append of 120 rows ended just before slot 50:
    # those rows sit in slots 930..999 and 0..49
    B, n_rec = 512, mlp.recent_rows(512, 0.75)
    assert n_rec == 384
    s = mlp.minibatch_slots(5, B, 1000, seed=11, n_recent=n_rec, head=50, last=120, cap=1000)
    old, rec = s[:B - n_rec], s[B - n_rec:]
    window = set(range(930, 1000)) | set(range(0, 50))
    assert set(rec.tolist()) <= window
    assert len(set(rec.tolist())) > 100          # spread over the window
    # the uniform part is the plain rule on the same words
    np.testing.assert_array_equal(old, mlp.minibatch_slots(5, B, 1000, seed=11)[:B - n_rec])
    # brute force on a tiny case: with last = 1 every recent row is slot head - 1
    s1 = mlp.minibatch_slots(2, 8, 10, seed=1, n_recent=3, head=0, last=1, cap=10)
    assert s1[5:].tolist() == [9, 9, 9]
    assert mlp.recent_rows(1024, 0.0) == 0 and mlp.recent_rows(1024, 1.0) == 1024
    assert mlp.recent_rows(3, 0.5) == 2           # halves round up


def test_standardise_is_the_population_standard_deviation():
    import statistics
    v = np.random.default_rng(8).normal(-3.0, 0.7, 501)
    mu, sd = mlp.standardise(v)
    assert abs(mu - statistics.fmean(v)) <= 1e-12 * abs(mu)
    assert abs(sd - statistics.pstdev(v)) <= 1e-12 * sd
    assert abs(sd - statistics.stdev(v)) > 1e-6 * sd          # not the sample (n - 1) form
    # two values a, b: population std |a - b| / 2
    assert mlp.standardise([1.0, 4.0]) == (2.5, 1.5)
    assert mlp.standardise([2.0, 2.0, 2.0]) == (2.0, 1.0)      # constant: unit scale


def test_random_keys_are_word_zero_of_the_counter_blocks():
    from oracle import philox
    keys = rank.random_keys(37, g=5, tag=rank.TAG_AUDIT, seed=12345)
    for i in (0, 1, 17, 36):
        assert keys[i] == philox.philox_block((i, 0, 5, rank.TAG_AUDIT), 12345)[0]
    other = rank.random_keys(37, g=5, tag=rank.TAG_PRESCREEN, seed=12345)
    assert other[3] == philox.philox_block((3, 0, 5, rank.TAG_PRESCREEN), 12345)[0]
    assert not np.array_equal(keys, other)
    assert keys.min() >= 0 and keys.max() < 2 ** 32 and np.array_equal(keys, np.floor(keys))


def test_merge_survivors_keeps_elites_and_best_candidates():
    pop = synth.random_population(10, 4, seed=1)
    fit_pop = synth.random_fitness(10, seed=2)
    cand = synth.random_population(30, 4, seed=3)
    fit_cand = synth.random_fitness(30, seed=4, n_ties=5, n_nan=2)
    genes, fit = ga.merge_survivors(pop, fit_pop, cand, fit_cand, 2)
    e = ga.elites(fit_pop, 2)
    np.testing.assert_array_equal(genes[:2], pop[e])
    key = np.where(np.isnan(fit_cand), -np.inf, fit_cand)
    best = np.lexsort((np.arange(30), -key))[:8]
    np.testing.assert_array_equal(genes[2:], cand[best])
    np.testing.assert_array_equal(fit[2:], fit_cand[best])


def test_gradients_and_adam_against_torch():
    """The same network in torch float64: autograd gradients and torch.optim.Adam."""
    import torch
    p = tiny_params(5)
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (9, 5))
    y = rng.normal(0, 1, 9)
    loss, g = mlp.loss_and_grads(p, X, y)
    tp = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in p.items()}
    Xt = torch.tensor(X)
    h1 = torch.nn.functional.gelu(Xt @ tp["W1"].T + tp["b1"])
    h2 = torch.nn.functional.gelu(h1 @ tp["W2"].T + tp["b2"])
    out = h2 @ tp["w3"] + tp["b3"][0]
    tl = ((out - torch.tensor(y)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-12 * loss
    for k in p:
        np.testing.assert_allclose(np.asarray(g[k]), tp[k].grad.numpy(), rtol=1e-10, atol=1e-14,
                                   err_msg=k)
    # three Adam steps with the same gradients
    opt = torch.optim.Adam(list(tp.values()), lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    cur = {k: np.asarray(v, np.float64) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in cur.items()}
    v = {k: np.zeros_like(val) for k, val in cur.items()}
    for step in (1, 2, 3):
        for k in tp:
            tp[k].grad = torch.tensor(np.asarray(g[k], np.float64) * step)
        opt.step()
        cur, m, v = mlp.adam_step(cur, {k: np.asarray(g[k]) * step for k in g}, m, v, step, lr=3e-3)
    for k in p:
        np.testing.assert_allclose(cur[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15, err_msg=k)

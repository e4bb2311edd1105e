"""Pins of the oracle's genetic operators: closed-form distributions, exact
enumeration and invariants that any correct implementation must satisfy."""
import collections
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ga, model
import synth


def test_probability_thresholds_and_index_draws():
    assert ga.prob_threshold(0.0) == 0
    assert ga.prob_threshold(1.0) == 2 ** 32
    assert ga.prob_threshold(0.5) == 2 ** 31
    assert ga.prob_threshold(0.9) == math.floor(0.9 * 2 ** 32)
    assert ga.index_draw(0, 17) == 0 and ga.index_draw(2 ** 32 - 1, 17) == 16
    # every index receives floor or ceil of 2^32 / n words
    n = 7
    edges = [-(-(i * 2 ** 32) // n) for i in range(n + 1)]
    for i in range(n):
        assert ga.index_draw(edges[i], n) == i and ga.index_draw(edges[i + 1] - 1, n) == i


def test_init_population_grid_and_range():
    pop = ga.init_population(64, 50, seed=123)
    assert pop.dtype == np.float32 and pop.shape == (64, 50)
    assert pop.min() >= -1.0 and pop.max() < 1.0
    scaled = (pop.astype(np.float64) + 1.0) * 2 ** 23
    np.testing.assert_array_equal(scaled, np.round(scaled))   # exact 2^-23 grid
    assert abs(pop.mean()) < 0.02
    assert stats.kstest(pop.ravel(), stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    assert not np.array_equal(pop, ga.init_population(64, 50, seed=124))


def test_elites_match_library_sort_with_ties_and_nan():
    fit = synth.random_fitness(200, seed=9, n_ties=40, n_nan=7)
    key = np.where(np.isnan(fit), -np.inf, fit)
    order = np.lexsort((np.arange(200), -key))           # fitness desc, index asc
    assert ga.rank_order(fit) == list(order)
    assert ga.elites(fit, 5) == list(order[:5])


def test_tournament_win_probability_closed_form():
    # rank r (1 = best) wins a size-k tournament with replacement with
    # probability ((P - r + 1)^k - (P - r)^k) / P^k.
    P, k, trials = 20, 3, 20000
    fit = np.linspace(1.0, 0.0, P)                        # index i has rank i + 1
    wins = np.zeros(P)
    for j in range(trials // 2):
        for s in (0, 1):
            wins[ga.tournament(fit, j, s, 0, k, seed=31)] += 1
    r = np.arange(1, P + 1)
    prob = ((P - r + 1) ** k - (P - r) ** k) / P ** k
    assert abs(prob[0] - 0.142625) < 1e-12 and abs(prob[-1] - 1.25e-4) < 1e-12
    expect = prob * trials
    # pool the sparse tail so every cell has an expected count >= 5
    cut = np.argmax(np.cumsum(expect[::-1]) >= 5)
    obs = np.concatenate([wins[:P - cut - 1], [wins[P - cut - 1:].sum()]])
    exp = np.concatenate([expect[:P - cut - 1], [expect[P - cut - 1:].sum()]])
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_irwin_hall_term_exact_enumeration():
    # z = sum_12 (2u + 1 - 2^24) / 2^25 with u uniform on 0..2^24-1: enumerate every u.
    u = np.arange(1 << 24, dtype=np.int64)
    term = 2 * u + 1 - (1 << 24)
    assert term.sum() == 0                                # mean exactly 0
    sq = sum(int((c * c).sum()) for c in np.split(term, 1 << 10))   # exact: chunks fit int64
    assert 3 * sq == (1 << 24) * ((1 << 48) - 1)          # E[term^2] = (2^48 - 1)/3
    var_z = 12 * sq / (1 << 24) / 2.0 ** 50
    assert var_z == 1.0 - 2.0 ** -48
    # the oracle's scalar Gaussian reproduces the extreme values
    assert ga.gaussian_ih12([0] * 12) == np.float32(-(12 * (2 ** 24 - 1)) / 2 ** 25)
    assert ga.gaussian_ih12([2 ** 32 - 1] * 12) == np.float32(12 * (2 ** 24 - 1) / 2 ** 25)
    assert ga.gaussian_ih12([2 ** 31] * 6 + [2 ** 31 - 256] * 6) == 0.0


def test_vectorised_mutation_equals_scalar_definition():
    pop = synth.random_population(40, 33, seed=2)
    out = ga.mutate(pop, g=5, seed=77, p_mutation=0.3, sigma=0.25)
    thr = ga.prob_threshold(0.3)
    n_mut = 0
    for c in range(40):
        for l in range(33):
            dec, words = ga._mutation_words(c, l, 5, 77)
            if int(dec) < thr:
                n_mut += 1
                want = ga.mutate_gene(pop[c, l], [int(w) for w in words], np.float32(0.25))
            else:
                want = pop[c, l]
            assert out[c, l].view(np.uint32) == np.float32(want).view(np.uint32)
    assert n_mut > 0


def _f32(hexbits: str) -> np.float32:
    return np.array([int(hexbits, 16)], dtype=np.uint32).view(np.float32)[0]


def _hex(v) -> str:
    return "%08x" % int(np.array([v], dtype=np.float32).view(np.uint32)[0])


def test_mutation_hand_derived_float32_bits(golden_dir):
    """Bits derived by hand with exact arithmetic (tests/golden/mutation_bits.json):
    float32 rounding of the integer sum S, of sigma * z and of g + delta, each
    on its own.  A fused multiply-add, a float64 delta or an unrounded S give
    the other bit patterns the fixture lists."""
    import json
    import os
    gold = json.load(open(os.path.join(golden_dir, "mutation_bits.json")))
    sigma = _f32(gold["sigma_bits"])
    assert sigma == np.float32(0.1)
    cases = gold["cases"]
    for case in cases:
        words = [int(w, 16) for w in case["words"]]
        assert sum(2 * (w >> 8) + 1 for w in words) - 12 * (1 << 24) == case["S"]
        z = ga.gaussian_ih12(words)
        assert z == np.float32(case["float32_S"] / 2.0 ** 25)
        got = ga.mutate_gene(_f32(case["gene_bits"]), words, sigma)
        assert _hex(got) == case["want_bits"]
        assert case["want_bits"] not in case["not_bits"].values()
        # the vectorised path computes the same delta and sum
        delta = np.float32(sigma * z)
        assert _hex(delta) == case["delta_bits"]
    for cc in gold["clamp_cases"]:
        words = [int(w, 16) for w in cases[cc.get("words_of_case", 0)]["words"]]
        got = ga.mutate_gene(_f32(cc["gene_bits"]), words, sigma)
        assert _hex(got) == cc["want_bits"], cc["why"]


def test_vectorised_mutation_clamps_nan_and_inf_like_the_scalar_rule():
    pop = synth.random_population(6, 5, seed=4)
    pop[0, 0] = np.nan
    pop[1, 1] = np.inf
    pop[2, 2] = -np.inf
    pop[3, 3] = np.array([0x7fa00001], dtype=np.uint32).view(np.float32)[0]   # signalling NaN
    with np.errstate(invalid="ignore"):          # the signalling NaN raises 'invalid'
        out = ga.mutate(pop, g=2, seed=9, p_mutation=1.0, sigma=0.1)
    assert out[0, 0] == -1.0 and out[1, 1] == 1.0 and out[2, 2] == -1.0 and out[3, 3] == -1.0
    assert np.isfinite(out).all() and out.min() >= -1.0 and out.max() <= 1.0
    # without mutation a NaN gene is copied bit for bit
    same = ga.mutate(pop, g=2, seed=9, p_mutation=0.0, sigma=0.1)
    np.testing.assert_array_equal(same.view(np.uint32), pop.view(np.uint32))


def test_mutation_statistics():
    n, L = 400, 64
    pop = np.zeros((n, L), dtype=np.float32)
    out = ga.mutate(pop, g=1, seed=5, p_mutation=0.05, sigma=0.1)
    hit = out != 0
    rate = hit.mean()
    assert abs(rate - 0.05) < 4 * math.sqrt(0.05 * 0.95 / (n * L))
    z = out[hit].astype(np.float64) / 0.1
    assert abs(z.mean()) < 4 / math.sqrt(z.size) and abs(z.var() - 1) < 0.1
    assert np.abs(out).max() <= 0.6
    # clamping: genes at the bound never leave [-1, 1]
    edge = np.ones((n, L), dtype=np.float32)
    out = ga.mutate(edge, g=1, seed=5, p_mutation=1.0, sigma=2.0)
    assert out.max() <= 1.0 and out.min() >= -1.0 and (out == 1.0).mean() > 0.4


@pytest.mark.parametrize("P,L,E", [(20, 32, 2), (21, 7, 2), (8, 1, 1), (16, 12, 0), (5, 9, 5)])
def test_ga_step_invariants(P, L, E):
    pop = ga.init_population(P, L, seed=P * L)
    fit = synth.random_fitness(P, seed=L, n_ties=3, n_nan=1)
    new = ga.ga_step(pop, fit, g=3, seed=99, elitism=E)
    assert new.shape == pop.shape and new.dtype == np.float32
    assert new.min() >= -1.0 and new.max() <= 1.0
    for e, idx in enumerate(ga.elites(fit, E)):
        np.testing.assert_array_equal(new[e].view(np.uint32), pop[idx].view(np.uint32))


def test_without_mutation_children_inherit_loci():
    P, L = 30, 25
    pop = ga.init_population(P, L, seed=1)
    fit = synth.random_fitness(P, seed=2)
    new = ga.ga_step(pop, fit, g=0, seed=4, elitism=2, p_mutation=0.0)
    for c in range(2, P):
        for l in range(L):
            assert new[c, l] in pop[:, l]
    copies = ga.ga_step(pop, fit, g=0, seed=4, elitism=2, p_mutation=0.0, p_crossover=0.0)
    rows = {r.tobytes() for r in pop}
    assert all(r.tobytes() in rows for r in copies)


def test_crossover_children_are_complementary_and_cut_uniform():
    P, L = 12, 9
    pop = np.arange(P * L, dtype=np.float32).reshape(P, L) / (P * L)   # every gene unique
    fit = synth.random_fitness(P, seed=3)
    cuts = []
    for g in range(300):
        kids = ga.make_offspring(pop, fit, g, 2, seed=8, p_crossover=1.0, p_mutation=0.0)
        a = int(np.argmax((pop[:, 0] == kids[0, 0])))
        b = int(np.argmax((pop[:, 0] == kids[1, 0])))
        cut = next((l for l in range(L) if kids[0, l] != pop[a, l]), L)
        np.testing.assert_array_equal(kids[0], np.concatenate([pop[a, :cut], pop[b, cut:]]))
        np.testing.assert_array_equal(kids[1], np.concatenate([pop[b, :cut], pop[a, cut:]]))
        if a != b:
            cuts.append(cut)
    counts = np.bincount(cuts, minlength=L)[1:]
    assert counts.min() > 0 and counts.sum() == len(cuts)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_best_fitness_never_decreases_with_elitism():
    X, t, _ = synth.regression_dataset(300, 3, 3, 0.05, seed=10)
    pop = ga.init_population(24, 9, seed=5)
    best = -np.inf
    for g in range(15):
        fit = model.evaluate(X, t, pop, "chebyshev", 3, "regression")["fitness"]
        assert fit.max() >= best
        best = fit.max()
        pop = ga.ga_step(pop, fit, g, seed=5, elitism=2)


# ---------------------------------------------------------------- roulette / ranking / immigrants
def test_roulette_weights_definition_and_edge_cases():
    f = [0.5, 0.2, float("nan"), 0.9]
    w = ga.roulette_weights(f)
    assert w[1] == 0 and w[2] == 0 and w[3] == 2 ** 32
    assert w[0] == int(np.floor((0.5 - 0.2) / (0.9 - 0.2) * 2.0 ** 32))
    assert ga.roulette_weights([0.3, 0.3, float("nan")]) == [1, 1, 0]
    assert ga.roulette_weights([float("nan")] * 3) == [1, 1, 1]


def test_pick_cumulative_against_linear_scan():
    rng = np.random.default_rng(0)
    cdf = ga.cumulative([3, 0, 5, 1, 0, 7])
    for _ in range(2000):
        r = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        t = (r * cdf[-1]) >> 64
        want = next(k for k, c in enumerate(cdf) if c > t)
        assert ga.pick_cumulative(cdf, r) == want
    # every target value of a small wheel: zero-weight slots are never chosen
    for t in range(cdf[-1]):
        r = -(-(t << 64) // cdf[-1])  # smallest r with floor(r * T / 2^64) == t
        k = ga.pick_cumulative(cdf, r)
        assert cdf[k] > t and (k == 0 or cdf[k - 1] <= t)
        assert [3, 0, 5, 1, 0, 7][k] > 0


def test_rank_cdf_closed_form_and_inversion():
    for P in (1, 2, 5, 17):
        w = [P - q for q in range(P)]
        cum = np.cumsum(w)
        assert [ga.rank_cdf(q, P) for q in range(P)] == cum.tolist()
    # exhaustive inversion at P = 5: every target value, through pick_rank
    P = 5
    T = P * (P + 1) // 2
    seen = collections.Counter()
    for t in range(T):
        r = -(-(t << 64) // T)  # smallest 64-bit draw whose target is t
        q = ga.pick_rank(P, r)
        assert q == next(q for q in range(P) if sum(P - x for x in range(q + 1)) > t)
        seen[q] += 1
    assert [seen[q] for q in range(P)] == [5, 4, 3, 2, 1]


def test_roulette_and_ranking_frequencies_chi2():
    P, g, seed, n = 12, 3, 777, 6000
    fit = np.linspace(0.1, 0.9, P)[::-1].copy()  # chromosome 0 best
    fit[7] = np.nan
    w = np.array(ga.roulette_weights(fit), dtype=np.float64)
    cdf = ga.cumulative(w)
    counts = np.zeros(P)
    for j in range(n // 2):
        for s in (0, 1):
            counts[ga.roulette(cdf, j, s, g, seed)] += 1
    assert counts[7] == 0 and counts[int(np.nanargmin(fit))] == 0
    exp = w / w.sum() * n
    m = exp > 0
    assert stats.chisquare(counts[m], exp[m]).pvalue > 1e-3
    order = ga.rank_order(fit)
    rc = np.zeros(P)
    for j in range(n // 2):
        for s in (0, 1):
            rc[order.index(ga.ranking(order, j, s, g, seed))] += 1
    expr = np.array([P - q for q in range(P)], dtype=np.float64)
    expr = expr / expr.sum() * n
    assert stats.chisquare(rc, expr).pvalue > 1e-3


def test_immigrants_replace_the_last_children():
    pop = synth.random_population(20, 9, seed=4)
    fit = synth.random_fitness(20, seed=5)
    for sel in (ga.SEL_TOURNAMENT, ga.SEL_ROULETTE, ga.SEL_RANKING):
        base = ga.make_offspring(pop, fit, 6, 11, 99, selection=sel)
        imm = ga.make_offspring(pop, fit, 6, 11, 99, selection=sel, n_immigrants=3)
        np.testing.assert_array_equal(base[:8], imm[:8])
        for c in range(8, 11):
            np.testing.assert_array_equal(imm[c], ga.immigrant(c, 9, 6, 99))
        assert np.all(imm >= -1.0) and np.all(imm < 1.0)
        grid = (imm[8:].astype(np.float64) + 1.0) * 2.0 ** 23
        assert np.all(grid == np.floor(grid))


def test_paper_selection_modes_keep_population_invariants():
    pop = synth.random_population(30, 12, seed=6)
    fit = synth.random_fitness(30, seed=7, n_ties=5, n_nan=2)
    for sel in (ga.SEL_ROULETTE, ga.SEL_RANKING):
        new = ga.ga_step(pop, fit, 2, 5, elitism=2, selection=sel, p_mutation=0.2, n_immigrants=4)
        assert new.shape == pop.shape
        e = ga.elites(fit, 2)
        np.testing.assert_array_equal(new[:2], pop[e])
        assert np.all(np.abs(new) <= 1.0)

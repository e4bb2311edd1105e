"""Device genetic operators against the oracle, bit for bit, given the same
fitness vector (the Philox counter layout and the float32 mutation arithmetic
fix every decision and every gene)."""
import numpy as np
import pytest

from oracle import ga
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def make_game(P, L_genes, E=2, k=3, pc=0.9, pm=0.05, sigma=0.1, seed=99, selection="tournament",
              n_imm=0):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    # L genes = F * D with the power basis and D = 1 (bias adds one)
    cfg = Config(n_patterns=64, n_features=L_genes, degree=1, basis="power", dtype="f32",
                 pop_size=P, elitism=E, tournament_k=k, p_crossover=pc, p_mutation=pm,
                 mutation_sigma=sigma, seed=seed, selection=selection, n_immigrants=n_imm)
    X = np.random.default_rng(0).uniform(-1, 1, (64, L_genes))
    t = np.zeros(64)
    return Game(cfg, dev(X, torch.float32), dev(t, torch.float32)), cfg


@pytest.mark.parametrize("P,L", [(20, 32), (1000, 120), (2048, 128), (7, 1)])
def test_init_population_bit_exact(P, L):
    announce(f"init population P={P} L={L}")
    g, cfg = make_game(P, L, E=min(2, P), seed=12345678901)
    got = host(g.population)
    want = ga.init_population(P, L, cfg.seed)
    assert np.array_equal(bits(got), bits(want))
    g.close()


STEP_CASES = [
    # P, L, E, k, p_c, p_m, sigma
    (20, 32, 2, 3, 0.9, 0.05, 0.1),
    (21, 7, 2, 3, 0.9, 0.05, 0.1),      # odd number of children
    (8, 1, 1, 3, 0.9, 0.2, 0.3),        # one gene: no crossover point
    (16, 12, 0, 1, 1.0, 1.0, 0.5),      # no elitism, k = 1, every gene mutates
    (5, 9, 5, 3, 0.9, 0.05, 0.1),       # all elites, no children
    (33, 40, 3, 16, 0.5, 0.2, 2.0),     # four Philox blocks per tournament, heavy clamping
    (1000, 120, 2, 3, 0.9, 0.05, 0.1),  # 100k-pattern classification workload shape
    (2048, 128, 2, 3, 0.9, 0.05, 0.1),  # 1M-pattern Legendre workload shape
]


@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: "-".join(map(str, c)))
def test_step_bit_exact_over_generations(case):
    torch = require_gpu()
    P, L, E, k, pc, pm, sigma = case
    seed = 424242 + P
    g, cfg = make_game(P, L, E, k, pc, pm, sigma, seed=seed)
    pop = host(g.population)
    for gen in range(3):
        fit = synth.random_fitness(P, seed=gen + P, n_ties=P // 4, n_nan=1 if P > 4 else 0)
        announce(f"step {case} generation {gen}")
        g.step(dev(fit, torch.float64))
        got = host(g.population)
        want = ga.ga_step(pop, fit, gen, seed, elitism=E, k=k, p_crossover=pc, p_mutation=pm,
                          sigma=sigma)
        bad = np.argwhere(bits(got) != bits(want))
        assert bad.size == 0, f"generation {gen}: first mismatches {bad[:5].tolist()}"
        assert g.state()["generation"] == gen + 1
        pop = want
    g.close()


def test_step_after_eval_uses_internal_fitness():
    torch = require_gpu()
    g, cfg = make_game(40, 16, seed=3)
    pop = host(g.population)
    mse, _, fit = g.eval_fitness()
    fit_h = host(fit)
    announce("step(NULL) after eval(NULL)")
    g.step()
    want = ga.ga_step(pop, fit_h, 0, cfg.seed)
    assert np.array_equal(bits(host(g.population)), bits(want))
    g.close()


def test_set_population_then_evolve_from_odd_generation():
    """Populations written in after an odd number of generations (the second
    population buffer is current) evolve exactly like the oracle."""
    torch = require_gpu()
    g, cfg = make_game(24, 10, seed=77)
    fit0 = synth.random_fitness(24, seed=1)
    g.step(dev(fit0, torch.float64))                       # generation 1: buffers swapped
    mine = synth.random_population(24, 10, seed=5)
    g.population = dev(mine, torch.float32)
    assert np.array_equal(bits(host(g.population)), bits(mine))
    fit1 = synth.random_fitness(24, seed=2, n_ties=5)
    announce("set population at generation 1, then step")
    g.step(dev(fit1, torch.float64))
    want = ga.ga_step(mine, fit1, 1, cfg.seed)
    assert np.array_equal(bits(host(g.population)), bits(want))
    # the fitness path sees the written population too
    mse, _, _ = g.eval_fitness()
    ref, _, _ = g.eval_fitness(dev(want, torch.float32))
    assert np.array_equal(host(mse), host(ref))
    g.close()


SEL = {"tournament": ga.SEL_TOURNAMENT, "roulette": ga.SEL_ROULETTE, "ranking": ga.SEL_RANKING}
WHEEL_CASES = [
    # selection, P, L, E, n_immigrants, p_mutation, fitness kind
    ("roulette", 20, 32, 2, 0, 0.05, "ties+nan"),
    ("roulette", 1000, 120, 2, 0, 0.2, "ties+nan"),
    ("roulette", 33, 9, 2, 5, 0.2, "all-equal"),
    ("roulette", 17, 5, 1, 0, 0.05, "all-nan"),
    ("ranking", 20, 32, 2, 0, 0.05, "ties+nan"),
    ("ranking", 2048, 128, 2, 0, 0.2, "ties+nan"),
    ("ranking", 8192, 7, 2, 30, 0.2, "ties+nan"),   # largest ranked population
    ("tournament", 64, 16, 2, 7, 0.05, "ties+nan"),
    ("ranking", 21, 7, 0, 21, 0.2, "ties+nan"),     # every child an immigrant
]


def wheel_fitness(kind, P, seed):
    if kind == "all-equal":
        return np.full(P, 0.25)
    if kind == "all-nan":
        return np.full(P, np.nan)
    return synth.random_fitness(P, seed=seed, n_ties=P // 4, n_nan=2 if P > 4 else 0)


@pytest.mark.parametrize("case", WHEEL_CASES, ids=lambda c: "-".join(map(str, c)))
def test_wheel_selection_and_immigrants_bit_exact(case):
    torch = require_gpu()
    sel, P, L, E, n_imm, pm, kind = case
    seed = 5150 + P
    g, cfg = make_game(P, L, E, pm=pm, seed=seed, selection=sel, n_imm=n_imm)
    pop = host(g.population)
    for gen in range(3):
        fit = wheel_fitness(kind, P, gen + P)
        announce(f"wheel step {case} generation {gen}")
        g.step(dev(fit, torch.float64))
        got = host(g.population)
        want = ga.ga_step(pop, fit, gen, seed, elitism=E, k=3, p_crossover=0.9, p_mutation=pm,
                          sigma=0.1, selection=SEL[sel], n_immigrants=n_imm)
        bad = np.argwhere(bits(got) != bits(want))
        assert bad.size == 0, f"generation {gen}: first mismatches {bad[:5].tolist()}"
        pop = want
    g.close()


@pytest.mark.parametrize("pm", [1.0, 0.3])
def test_non_finite_and_out_of_range_genes_bit_exact(pm):
    """Genes the library accepts through set_population but the operators
    never produce: NaN, +-inf and values outside [-1, 1].  A mutated gene is
    clamped with IEEE maxNum/minNum (a NaN sum lands on -1, +-inf on +-1), an
    unmutated one is copied bit for bit, NaN included; the device and the
    oracle agree bit for bit over three generations."""
    torch = require_gpu()
    P, L, seed = 24, 12, 31415
    g, cfg = make_game(P, L, pm=pm, sigma=0.5, seed=seed)
    pop = synth.random_population(P, L, seed=9)
    rng = np.random.default_rng(10)
    specials = np.array([np.nan, np.inf, -np.inf, 3.5, -7.25, 1e30, -0.0], dtype=np.float32)
    cells = rng.choice(P * L, 60, replace=False)
    pop.reshape(-1)[cells] = specials[np.arange(60) % specials.size]
    g.population = dev(pop, torch.float32)
    assert np.array_equal(bits(host(g.population)), bits(pop))
    for gen in range(3):
        fit = synth.random_fitness(P, seed=gen + 50, n_ties=4, n_nan=1)
        announce(f"non-finite genes p_m={pm} generation {gen}")
        g.step(dev(fit, torch.float64))
        got = host(g.population)
        want = ga.ga_step(pop, fit, gen, seed, p_mutation=pm, sigma=0.5)
        bad = np.argwhere(bits(got) != bits(want))
        assert bad.size == 0, f"generation {gen}: first mismatches {bad[:5].tolist()}"
        if pm == 1.0:
            # every child gene went through the clamp
            assert np.all(np.abs(want[2:]) <= 1.0)
        pop = want
    g.close()

"""Genetic operators of GAME -- oracle side, test infrastructure only.

The paper lists the operators (Sec. 3: crossover, mutation, roulette/ranking
selection, elitism; genes drawn at random in [-1, +1] and kept there), says
that randomly generated chromosomes replace older individuals during the
evolution (Sec. 4), and gives the settings of its experiment (Sec. 5:
ranking and roulette selection, crossover rate 0.9, mutation rate 0.2, 2
elite chromosomes per generation, MSE threshold 0.001).  The operator
variants used here: selection by tournament, by fitness-proportionate
roulette, or by rank-based roulette (linear ranking weights); one-point
crossover producing two complementary children; per-gene Gaussian mutation
with clamping to [-1, 1] (a mutated gene always lands in the gene range of
Sec. 3: a NaN sum goes to -1, as the IEEE 754 maxNum/minNum operations
give); optionally the last n_imm children of a generation replaced by random
immigrants.

Every random decision is a pure function of a Philox4x32-10 block
(``oracle.philox``) addressed by a counter (a, b, generation, tag) under the
key = seed, so a device implementation that follows the same addressing
reproduces each decision bit for bit.  Counter addressing:

  init      gene (p, l):           (p, l, 0, INIT) word 0
  selection pair j, parent s, draw i (i < k <= 16):
                                    (j, 4*s + i // 4, g, SEL) word i % 4
  crossover pair j:                 (j, 8, g, SEL) words 0 (decision), 1 (point)
  mutation  child c, gene l:        (c, l, g, MUT) word 0 (decision); Gaussian
            from (c,l,g,MUT) words 1..3, (c,l,g,MUT1) words 0..3,
            (c,l,g,MUT2) words 0..3, (c,l,g,MUT3) word 0
  roulette  pair j, parent s:       (j, s, g, ROULETTE) words 0, 1 -> a 64-bit draw
  immigrant child c, gene l:        (c, l, g, IMMIGRANT) word 0, as at init

Arithmetic is exact integer arithmetic except the mutation update, which is
done in IEEE float32 one operation at a time (numpy float32 scalars), exactly
as a float32 device computes it without fused multiply-add.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32_10

TAG_INIT = 1
TAG_SEL = 2
TAG_MUT = 3
TAG_MUT1 = 4
TAG_MUT2 = 5
TAG_MUT3 = 6
TAG_ROULETTE = 11
TAG_IMMIGRANT = 12

SEL_TOURNAMENT, SEL_ROULETTE, SEL_RANKING = 0, 1, 2

TWO32 = 1 << 32


def prob_threshold(p: float) -> int:
    """A decision with probability p fires iff a uniform u32 word < floor(p * 2^32)."""
    if not (0.0 <= p <= 1.0):
        raise ValueError("probability out of [0, 1]")
    return int(math.floor(p * 4294967296.0))


def index_draw(word: int, n: int) -> int:
    """Uniform index in [0, n) from a u32 word: floor(word * n / 2^32)."""
    return (int(word) * int(n)) >> 32


def init_population(P: int, L: int, seed: int) -> np.ndarray:
    """Genes U[-1, 1): (w >> 8) * 2^-23 - 1 from block (p, l, 0, INIT) word 0 (Sec. 3)."""
    p = np.arange(P, dtype=np.uint64)[:, None]
    l = np.arange(L, dtype=np.uint64)[None, :]
    w0, _, _, _ = philox4x32_10(p, l, 0, TAG_INIT, seed)
    u24 = (w0 >> np.uint32(8)).astype(np.float64)
    return (u24 * 2.0 ** -23 - 1.0).astype(np.float32)  # exact in float32


def _rank_key(f: float) -> float:
    return -math.inf if math.isnan(f) else float(f)


def better(fit, a: int, b: int) -> bool:
    """a ranks above b: higher fitness, ties to the lower index, NaN worst."""
    fa, fb = _rank_key(fit[a]), _rank_key(fit[b])
    return fa > fb or (fa == fb and a < b)


def rank_order(fit) -> list:
    """All indices, best first (fitness descending, index ascending, NaN last)."""
    return sorted(range(len(fit)), key=lambda i: (-_rank_key(fit[i]), i))


def elites(fit, E: int) -> list:
    return rank_order(fit)[:E]


def tournament(fit, j: int, s: int, g: int, k: int, seed: int) -> int:
    """Best of k indices drawn with replacement (Sec. 3 selection operator)."""
    P = len(fit)
    winner = None
    for i in range(k):
        blk = philox4x32_10(j, 4 * s + i // 4, g, TAG_SEL, seed)
        cand = index_draw(int(blk[i % 4]), P)
        if winner is None or better(fit, cand, winner):
            winner = cand
    return winner


def roulette_weights(fit) -> list:
    """Integer weights of fitness-proportionate selection, shifted so the worst
    chromosome weighs 0: w_i = floor((f_i - f_min) / (f_max - f_min) * 2^32)
    (float64 arithmetic); NaN fitness weighs 0; when every finite fitness is
    equal each finite one weighs 1 (all NaN: every chromosome weighs 1)."""
    f = [float(x) for x in fit]
    fin = [x for x in f if not math.isnan(x)]
    if not fin:
        return [1] * len(f)
    lo, hi = min(fin), max(fin)
    if not hi > lo:
        return [0 if math.isnan(x) else 1 for x in f]
    span = hi - lo
    return [0 if math.isnan(x) else int(math.floor((x - lo) / span * 4294967296.0)) for x in f]


def cumulative(weights) -> list:
    out, acc = [], 0
    for w in weights:
        acc += int(w)
        out.append(acc)
    return out


def wide_draw(j: int, s: int, g: int, seed: int) -> int:
    """64-bit uniform draw of parent s of pair j: words 0 (low) and 1 (high)."""
    blk = philox4x32_10(j, s, g, TAG_ROULETTE, seed)
    return (int(blk[1]) << 32) | int(blk[0])


def pick_cumulative(cdf, r: int) -> int:
    """Smallest k with cdf[k] > t, t = floor(r * total / 2^64)."""
    t = (r * int(cdf[-1])) >> 64
    lo, hi = 0, len(cdf) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if cdf[mid] > t:
            hi = mid
        else:
            lo = mid + 1
    return lo


def rank_cdf(q: int, P: int) -> int:
    """Cumulative linear-ranking weight of ranks 0..q (rank 0 = best weighs P)."""
    return (q + 1) * P - q * (q + 1) // 2


def roulette(cdf, j: int, s: int, g: int, seed: int) -> int:
    return pick_cumulative(cdf, wide_draw(j, s, g, seed))


def pick_rank(P: int, r: int) -> int:
    """Rank q (0 = best) of a linear-ranking draw: smallest q with
    rank_cdf(q) > floor(r * P(P+1)/2 / 2^64)."""
    t = (r * (P * (P + 1) // 2)) >> 64
    lo, hi = 0, P - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if rank_cdf(mid, P) > t:
            hi = mid
        else:
            lo = mid + 1
    return lo


def ranking(order, j: int, s: int, g: int, seed: int) -> int:
    """Rank-based roulette: rank q (0 = best) is drawn with weight P - q."""
    return order[pick_rank(len(order), wide_draw(j, s, g, seed))]


def immigrant(c: int, L: int, g: int, seed: int) -> np.ndarray:
    """Random chromosome for child c of generation g, drawn like the initial genes."""
    l = np.arange(L, dtype=np.uint64)
    w0, _, _, _ = philox4x32_10(c, l, g, TAG_IMMIGRANT, seed)
    return ((w0 >> np.uint32(8)).astype(np.float64) * 2.0 ** -23 - 1.0).astype(np.float32)


def gaussian_ih12(words) -> np.float32:
    """Irwin-Hall sum of 12 bin-midpoint uniforms, centred: mean 0, variance 1 - 2^-48.

    S = sum(2 * (w >> 8) + 1) - 12 * 2^24 as an integer, z = float32(S) * 2^-25.
    """
    words = [int(w) for w in words]
    assert len(words) == 12
    s = sum(2 * (w >> 8) + 1 for w in words) - 12 * (1 << 24)
    return np.float32(s) * np.float32(2.0 ** -25)


def clamp_gene(v):
    """Clamp to [-1, 1] with IEEE 754 maxNum/minNum: a NaN operand yields the
    other one, so a NaN sum becomes -1 and the result is always a gene value."""
    return np.fmin(np.fmax(v, np.float32(-1.0)), np.float32(1.0))


def mutate_gene(gene: np.float32, words12, sigma32: np.float32) -> np.float32:
    """g' = clamp(fl(g + fl(sigma * z)), -1, 1), float32, no fused multiply-add."""
    z = gaussian_ih12(words12)
    delta = np.float32(sigma32 * z)
    v = np.float32(np.float32(gene) + delta)
    return np.float32(clamp_gene(v))


def _mutation_words(c, l, g: int, seed: int):
    """Decision word and the 12 Gaussian words for child c, gene l (arrays)."""
    b0 = philox4x32_10(c, l, g, TAG_MUT, seed)
    b1 = philox4x32_10(c, l, g, TAG_MUT1, seed)
    b2 = philox4x32_10(c, l, g, TAG_MUT2, seed)
    b3 = philox4x32_10(c, l, g, TAG_MUT3, seed)
    gauss = [b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3],
             b2[0], b2[1], b2[2], b2[3], b3[0]]
    return b0[0], gauss


def mutate(children: np.ndarray, g: int, seed: int, p_mutation: float,
           sigma: float) -> np.ndarray:
    """Per-gene Gaussian mutation of every child (row = child ordinal).

    Same arithmetic as ``mutate_gene``, applied elementwise to float32 arrays
    (numpy float32 array operations round each operation like the scalars).
    """
    children = np.array(children, dtype=np.float32, copy=True)
    n, L = children.shape
    if n == 0:
        return children
    thr_m = prob_threshold(p_mutation)
    c = np.arange(n, dtype=np.uint64)[:, None]
    l = np.arange(L, dtype=np.uint64)[None, :]
    dec, _ = _mutation_words(c, l, g, seed)
    hit = dec.astype(np.uint64) < np.uint64(thr_m)
    ci, li = np.nonzero(hit)
    if ci.size == 0:
        return children
    _, words = _mutation_words(ci.astype(np.uint64), li.astype(np.uint64), g, seed)
    s = np.zeros(ci.size, dtype=np.int64)
    for w in words:
        s += 2 * (w.astype(np.int64) >> 8) + 1
    s -= 12 * (1 << 24)
    z = s.astype(np.float32) * np.float32(2.0 ** -25)
    delta = np.float32(sigma) * z
    v = children[ci, li] + delta
    children[ci, li] = clamp_gene(v)
    return children


def make_offspring(pop, fit, g: int, n_children: int, seed: int, k: int = 3,
                   p_crossover: float = 0.9, p_mutation: float = 0.05,
                   sigma: float = 0.1, selection: int = SEL_TOURNAMENT,
                   n_immigrants: int = 0) -> np.ndarray:
    """n_children children from selected pairs, crossover, then mutation; the
    last n_immigrants children are random immigrants instead.

    Pair j yields child ordinals 2j and 2j+1; an odd count drops the last one.
    """
    pop = np.asarray(pop, dtype=np.float32)
    P, L = pop.shape
    if not 1 <= k <= 16:
        raise ValueError("tournament size must be in [1, 16]")
    if not 0 <= n_immigrants <= n_children:
        raise ValueError("n_immigrants out of range")
    thr_c = prob_threshold(p_crossover)
    if selection == SEL_ROULETTE:
        cdf = cumulative(roulette_weights(fit))
        pick = lambda j, s: roulette(cdf, j, s, g, seed)
    elif selection == SEL_RANKING:
        order = rank_order(fit)
        pick = lambda j, s: ranking(order, j, s, g, seed)
    elif selection == SEL_TOURNAMENT:
        pick = lambda j, s: tournament(fit, j, s, g, k, seed)
    else:
        raise ValueError("unknown selection")
    out = np.empty((n_children, L), dtype=np.float32)
    for j in range((n_children + 1) // 2):
        a = pick(j, 0)
        b = pick(j, 1)
        blk = philox4x32_10(j, 8, g, TAG_SEL, seed)
        ca, cb = pop[a].copy(), pop[b].copy()
        if int(blk[0]) < thr_c and L >= 2:
            cut = 1 + index_draw(int(blk[1]), L - 1)
            ca = np.concatenate([pop[a][:cut], pop[b][cut:]])
            cb = np.concatenate([pop[b][:cut], pop[a][cut:]])
        out[2 * j] = ca
        if 2 * j + 1 < n_children:
            out[2 * j + 1] = cb
    out = mutate(out, g, seed, p_mutation, sigma)
    for c in range(n_children - n_immigrants, n_children):
        out[c] = immigrant(c, L, g, seed)
    return out


def ga_step(pop, fit, g: int, seed: int, elitism: int = 2, **kw) -> np.ndarray:
    """Generation g -> g+1: the E elites (best first) then P - E children."""
    pop = np.asarray(pop, dtype=np.float32)
    P, L = pop.shape
    if not 0 <= elitism <= P:
        raise ValueError("elitism out of range")
    new = np.empty_like(pop)
    for e, idx in enumerate(elites(fit, elitism)):
        new[e] = pop[idx]
    if P > elitism:
        new[elitism:] = make_offspring(pop, fit, g, P - elitism, seed, **kw)
    return new


def merge_survivors(pop, fit_pop, cand, fit_cand, elitism: int):
    """Next population of the offspring form: the E best of the current
    population (unchanged, best first), then the P - E best candidates by
    exact fitness (descending, ties to the lower candidate index, NaN last).
    Returns (genes, fitness)."""
    pop = np.asarray(pop, dtype=np.float32)
    cand = np.asarray(cand, dtype=np.float32)
    P = pop.shape[0]
    if cand.shape[0] < P - elitism:
        raise ValueError("not enough candidates")
    keep = elites(fit_pop, elitism)
    best = rank_order(fit_cand)[:P - elitism]
    genes = np.concatenate([pop[keep], cand[best]], axis=0)
    fit = np.concatenate([np.asarray(fit_pop, np.float64)[keep],
                          np.asarray(fit_cand, np.float64)[best]])
    return genes, fit

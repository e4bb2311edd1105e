"""Offspring form and learned prescreen on the GPU against the oracle.

* The surrogate MLP's initialisation (bit for bit), forward pass, gradients
  and Adam step (float32 tolerances) against oracle/mlp.py.
* One offspring generation without a prescreen, with the random prescreen
  and with an untrained MLP prescreen: the children, the chosen subset and the
  next population bit for bit, given the device's own fitness values (which
  the same kernel reproduces for the same rows).
* The replay buffer's contents and the two Adam steps trained on it.
* The Spearman statistics of the log, graph-replayed runs equal to eager
  steps, and a learned prescreen ahead of the random one.
"""
from collections import Counter

import numpy as np
import pytest

from oracle import ga, mlp, rank
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

K_TOURN, PC, PM, SIGMA = 3, 0.9, 0.05, 0.1


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def make(surrogate="none", P=32, n_off=96, frac=0.25, audit=0, steps=0, batch=64, H=32,
         buffer=4096, E=2, seed=77, N=5000, F=4, D=3, **kw):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    X, t, _ = synth.regression_dataset(N, F, 3, 0.05, seed=5)
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", dtype="f32", pop_size=P,
                 elitism=E, n_offspring=n_off, surrogate=surrogate, prescreen_frac=frac,
                 audit=audit, surrogate_steps=steps, surrogate_batch=batch, surrogate_hidden=H,
                 surrogate_buffer=buffer, tournament_k=K_TOURN, p_crossover=PC, p_mutation=PM,
                 mutation_sigma=SIGMA, seed=seed, **kw)
    return Game(cfg, dev(X, torch.float32), dev(t, torch.float32)), cfg


def split_params(flat, L, H):
    flat = np.asarray(flat)
    o = 0
    out = {}
    for name, shape in (("W1", (H, L)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                        ("w3", (H,)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    assert o == flat.size
    return out


def join_params(p):
    return np.concatenate([np.ravel(p[k]) for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def drawn_from(pool, rows) -> bool:
    """Every row of `rows` is a row of `pool`, none used more often than it
    occurs there (children can repeat: a pair without crossover or mutation
    copies its parents)."""
    have = Counter(bits(r).tobytes() for r in pool)
    need = Counter(bits(r).tobytes() for r in rows)
    return all(have[key] >= n for key, n in need.items())


def children_of(pop, fit, gen, n_off, seed):
    return ga.make_offspring(pop, fit, gen, n_off, seed, k=K_TOURN, p_crossover=PC,
                             p_mutation=PM, sigma=SIGMA)


# ----------------------------------------------------------------- the MLP
def test_mlp_init_bit_exact():
    g, cfg = make("mlp", H=48, n_off=256)
    announce("mlp init")
    got = host(g.mlp_params())
    want = join_params(mlp.init_params(g.L, 48, 48, cfg.seed))
    assert np.array_equal(bits(got), bits(want))
    g.close()


@pytest.mark.parametrize("H,B,F,D,bias", [
    (64, 200, 4, 3, 0),     # L = 12
    (48, 77, 3, 3, 1),      # ragged: L = 10, H not a multiple of 32, B not of 4
    (33, 5, 7, 2, 0),       # L = 14, one partial row tile
])
def test_mlp_forward_grads_adam(H, B, F, D, bias):
    torch = require_gpu()
    g, cfg = make("mlp", H=H, batch=256, n_off=300, F=F, D=D, bias=bias)
    L = g.L
    rng = np.random.default_rng(3)
    Xh = rng.uniform(-1, 1, (B, L)).astype(np.float32)
    th = rng.normal(0, 1, B).astype(np.float32)
    announce(f"mlp forward H={H} B={B} L={g.L}")
    p0 = split_params(host(g.mlp_params()), L, H)
    y = host(g.mlp_forward(dev(Xh, torch.float32)))
    ref = mlp.forward(p0, Xh)
    scale = max(1.0, np.abs(ref["y"]).max())
    assert np.abs(y - ref["y"]).max() <= 1e-5 * scale
    announce("mlp grads")
    gr, loss = g.mlp_grads(dev(Xh, torch.float32), dev(th, torch.float32))
    gr = host(gr)
    ref_loss, ref_g = mlp.loss_and_grads(p0, Xh, th)
    assert abs(float(host(loss)[0]) - ref_loss) <= 1e-5 * ref_loss
    got = split_params(gr, L, H)
    for k in ref_g:
        tol = 1e-4 * np.abs(ref_g[k]).max() + 1e-9
        assert np.abs(got[k] - ref_g[k]).max() <= tol, k
    announce("mlp adam, two steps")
    m = {k: np.zeros_like(v, dtype=np.float64) for k, v in p0.items()}
    v = {k: np.zeros_like(v, dtype=np.float64) for k, v in p0.items()}
    pref = {k: np.asarray(x, np.float64) for k, x in p0.items()}
    for t in (1, 2):
        gflat = gr if t == 1 else host(g.mlp_grads(dev(Xh, torch.float32),
                                                    dev(th, torch.float32))[0])
        g.mlp_adam(dev(gflat, torch.float32))
        pref, m, v = mlp.adam_step(pref, split_params(gflat.astype(np.float64), L, H), m, v, t,
                                   lr=cfg.surrogate_lr)
        got = host(g.mlp_params())
        assert np.abs(got - join_params(pref)).max() <= 2e-6
    g.close()


@pytest.mark.parametrize("B", [2048, 2000])
def test_mlp_training_at_benchmarked_shape(B):
    """The surrogate's training products at the benchmarked shape: 128 genes
    (16 features, Legendre D = 8), two hidden layers of 256 units, minibatches
    of 2048 rows and a ragged 2000.  Every tile product then runs several
    16-wide contraction groups per wave (the next group's operands are loaded
    while the current one multiplies), which the small cases above never
    reach.  Forward scores, the loss, every gradient element and two Adam
    steps against the float64 oracle."""
    torch = require_gpu()
    H = 256
    g, cfg = make("mlp", H=H, batch=2048, n_off=2048, F=16, D=8, N=3000)
    L = g.L
    assert L == 128
    rng = np.random.default_rng(B)
    Xh = rng.uniform(-1, 1, (B, L)).astype(np.float32)
    th = rng.normal(0, 1, B).astype(np.float32)
    announce(f"mlp forward at the benchmarked shape H={H} B={B} L={L}")
    p0 = split_params(host(g.mlp_params()), L, H)
    y = host(g.mlp_forward(dev(Xh, torch.float32)))
    ref = mlp.forward(p0, Xh)
    assert np.abs(y - ref["y"]).max() <= 1e-5 * max(1.0, np.abs(ref["y"]).max())
    announce(f"mlp grads at the benchmarked shape B={B}")
    gr, loss = g.mlp_grads(dev(Xh, torch.float32), dev(th, torch.float32))
    gr = host(gr)
    ref_loss, ref_g = mlp.loss_and_grads(p0, Xh, th)
    assert abs(float(host(loss)[0]) - ref_loss) <= 1e-5 * ref_loss
    got = split_params(gr, L, H)
    for k in ref_g:
        tol = 1e-4 * np.abs(ref_g[k]).max() + 1e-9
        err = np.abs(got[k] - ref_g[k])
        assert err.max() <= tol, (k, float(err.max()), tol)
    announce(f"mlp adam at the benchmarked shape B={B}, two steps")
    m = {k: np.zeros_like(v, dtype=np.float64) for k, v in p0.items()}
    v = {k: np.zeros_like(v, dtype=np.float64) for k, v in p0.items()}
    pref = {k: np.asarray(x, np.float64) for k, x in p0.items()}
    for t in (1, 2):
        gflat = gr if t == 1 else host(g.mlp_grads(dev(Xh, torch.float32),
                                                    dev(th, torch.float32))[0])
        g.mlp_adam(dev(gflat, torch.float32))
        pref, m, v = mlp.adam_step(pref, split_params(gflat.astype(np.float64), L, H), m, v, t,
                                   lr=cfg.surrogate_lr)
        assert np.abs(host(g.mlp_params()) - join_params(pref)).max() <= 2e-6
    g.close()


# ----------------------------------------------------- offspring generations
def test_offspring_plain_bit_exact():
    torch = require_gpu()
    P, E, n_off, seed = 32, 2, 96, 5150
    g, cfg = make("none", P=P, E=E, n_off=n_off, seed=seed)
    pop = host(g.population)
    fit = host(g.eval_fitness()[2])
    for gen in range(3):
        announce(f"offspring plain generation {gen}")
        children = children_of(pop, fit, gen, n_off, seed)
        g.step()
        cf = host(g.eval_fitness(dev(children, torch.float32))[2])
        want, want_fit = ga.merge_survivors(pop, fit, children, cf, E)
        got = host(g.population)
        bad = np.argwhere(bits(got) != bits(want))
        assert bad.size == 0, f"generation {gen}: {bad[:5].tolist()}"
        st = g.state()
        assert st["generation"] == gen + 1
        assert st["best_fitness"] == want_fit.max()
        pop, fit = want, want_fit
    g.close()


def test_offspring_random_prescreen_bit_exact():
    torch = require_gpu()
    P, E, n_off, seed = 32, 2, 128, 99
    g, cfg = make("random", P=P, E=E, n_off=n_off, frac=0.5, seed=seed)
    k = 64
    pop = host(g.population)
    fit = host(g.eval_fitness()[2])
    for gen in range(3):
        announce(f"offspring random prescreen generation {gen}")
        children = children_of(pop, fit, gen, n_off, seed)
        sel = rank.smallest_k(rank.random_keys(n_off, gen, rank.TAG_PRESCREEN, seed), k)
        g.step()
        cand = children[sel]
        cf = host(g.eval_fitness(dev(cand, torch.float32))[2])
        want, want_fit = ga.merge_survivors(pop, fit, cand, cf, E)
        got = host(g.population)
        assert np.array_equal(bits(got), bits(want)), f"generation {gen}"
        pop, fit = want, want_fit
    g.close()


def test_offspring_untrained_mlp_prescreen_bit_exact():
    torch = require_gpu()
    P, E, n_off, seed = 32, 2, 256, 31337
    g, cfg = make("mlp", P=P, E=E, n_off=n_off, frac=0.25, steps=0, audit=0, seed=seed)
    k = 64
    pop = host(g.population)
    fit = host(g.eval_fitness()[2])
    for gen in range(2):
        announce(f"offspring untrained mlp prescreen generation {gen}")
        children = children_of(pop, fit, gen, n_off, seed)
        yhat = host(g.mlp_forward(dev(children, torch.float32)))
        sel = rank.smallest_k(yhat, k)
        g.step()
        cand = children[sel]
        cf = host(g.eval_fitness(dev(cand, torch.float32))[2])
        want, want_fit = ga.merge_survivors(pop, fit, cand, cf, E)
        assert np.array_equal(bits(host(g.population)), bits(want)), f"generation {gen}"
        pop, fit = want, want_fit
    log = g.surrogate_log()
    assert log.shape == (2, 3) and np.all(log[:, 2] == 0.0)
    g.close()


def test_spearman_log_matches_oracle():
    torch = require_gpu()
    P, E, n_off, A, seed = 32, 2, 256, 40, 2024
    g, cfg = make("mlp", P=P, E=E, n_off=n_off, frac=0.25, steps=0, audit=A, seed=seed)
    k = 64
    pop = host(g.population)
    fit = host(g.eval_fitness()[2])
    children = children_of(pop, fit, 0, n_off, seed)
    yhat = host(g.mlp_forward(dev(children, torch.float32)))
    sel = rank.smallest_k(yhat, k)
    aud = rank.smallest_k(rank.random_keys(n_off, 0, rank.TAG_AUDIT, seed), A)
    announce("spearman log")
    g.step()
    mse_sel = host(g.eval_fitness(dev(children[sel], torch.float32))[0])
    mse_aud = host(g.eval_fitness(dev(children[aud], torch.float32))[0])
    log = g.surrogate_log()
    assert log.shape == (1, 3)
    assert abs(log[0, 0] - rank.spearman(yhat[aud], mse_aud)) <= 1e-6
    assert abs(log[0, 1] - rank.spearman(yhat[sel], mse_sel)) <= 1e-6
    # the next population: the elites, then distinct children of the prescreened set
    got = host(g.population)
    assert np.array_equal(bits(got[:E]), bits(pop[ga.elites(fit, E)]))
    assert drawn_from(children[sel], got[E:])
    g.close()


def test_replay_buffer_and_training():
    torch = require_gpu()
    P, E, n_off, A, B, H, seed = 32, 2, 256, 16, 64, 32, 4711
    g, cfg = make("mlp", P=P, E=E, n_off=n_off, frac=0.25, steps=1, audit=A, batch=B, H=H,
                  seed=seed)
    k, L = 64, g.L
    pop = host(g.population)
    mse_pop, _, fit_t = g.eval_fitness()
    mse_pop, fit = host(mse_pop), host(fit_t)
    children = children_of(pop, fit, 0, n_off, seed)
    aud = rank.smallest_k(rank.random_keys(n_off, 0, rank.TAG_AUDIT, seed), A)
    announce("replay buffer after one generation")
    g.step()
    genes, y, count, head, mu, sigma = g.surrogate_buffer()
    genes, y = host(genes), host(y)
    n = P + k + A
    assert count == n and head == n
    assert np.array_equal(bits(genes[:P]), bits(pop))
    np.testing.assert_allclose(y[:P], np.log(mse_pop), rtol=1e-6)
    assert drawn_from(children, genes[P:P + k])
    assert np.array_equal(bits(genes[P + k:n]), bits(children[aud]))
    mse_new = host(g.eval_fitness(dev(genes[P:n], torch.float32))[0])
    np.testing.assert_allclose(y[P:n], np.log(mse_new), rtol=1e-5)
    mu_ref, sd_ref = mlp.standardise(y[:n])
    assert abs(mu - mu_ref) <= 1e-5 * abs(mu_ref) and abs(sigma - sd_ref) <= 1e-5 * sd_ref
    # the two Adam steps: one at set-up on the population, one after the generation
    p = {kk: np.asarray(v, np.float64) for kk, v in mlp.init_params(L, H, H, seed).items()}
    m = {kk: np.zeros_like(v) for kk, v in p.items()}
    v = {kk: np.zeros_like(val) for kk, val in p.items()}
    loss = None
    n_rec = mlp.recent_rows(B, cfg.surrogate_recent)
    assert n_rec > 0
    # (step, pairs stored, ring head, rows of the latest append)
    for step, cnt, hd, last in ((0, P, P, P), (1, n, n, k + A)):
        mu_s, sd_s = mlp.standardise(y[:cnt])
        slots = mlp.minibatch_slots(step, B, cnt, seed, n_recent=n_rec, head=hd, last=last,
                                    cap=cfg.surrogate_buffer)
        loss, gr = mlp.loss_and_grads(p, genes[slots], (y[slots] - mu_s) / sd_s)
        p, m, v = mlp.adam_step(p, gr, m, v, step + 1, lr=cfg.surrogate_lr)
    got = host(g.mlp_params())
    diff = np.abs(got - join_params(p))
    # an update at step 1 is +-lr times the sign of each gradient, so an element
    # whose gradient is zero to rounding may move the other way
    assert np.mean(diff <= 1e-5) >= 0.995
    assert diff.max() <= 4.0 * cfg.surrogate_lr + 1e-5
    log = g.surrogate_log()
    assert abs(log[0, 2] - loss) <= 1e-3 * loss
    g.close()


def test_replay_training_at_benchmarked_shape():
    """One generation of the learned prescreen with the benchmarked network
    and minibatch (128 genes, 256-256 hidden, 2048 rows drawn from the
    replay ring, three quarters of them from the latest generation): the
    parameters after the set-up step and the generation's step equal the
    oracle's two Adam steps on the same ring slots and standardised targets."""
    torch = require_gpu()
    P, E, n_off, A, B, H, seed = 256, 2, 2048, 256, 2048, 256, 9001
    g, cfg = make("mlp", P=P, E=E, n_off=n_off, frac=0.25, steps=1, audit=A, batch=B, H=H,
                  buffer=50000, F=16, D=8, N=3000, seed=seed)
    k, L = 512, g.L
    assert L == 128
    announce("replay training at the benchmarked shape: one generation")
    g.step()
    genes, y, count, head, mu, sigma = g.surrogate_buffer()
    genes, y = host(genes), host(y)
    n = P + k + A
    assert count == n and head == n
    p = {kk: np.asarray(val, np.float64) for kk, val in mlp.init_params(L, H, H, seed).items()}
    m = {kk: np.zeros_like(val) for kk, val in p.items()}
    v = {kk: np.zeros_like(val) for kk, val in p.items()}
    n_rec = mlp.recent_rows(B, cfg.surrogate_recent)
    loss = None
    for step, cnt, hd, last in ((0, P, P, P), (1, n, n, k + A)):
        mu_s, sd_s = mlp.standardise(y[:cnt])
        slots = mlp.minibatch_slots(step, B, cnt, seed, n_recent=n_rec, head=hd, last=last,
                                    cap=cfg.surrogate_buffer)
        loss, gr = mlp.loss_and_grads(p, genes[slots], (y[slots] - mu_s) / sd_s)
        p, m, v = mlp.adam_step(p, gr, m, v, step + 1, lr=cfg.surrogate_lr)
    got = host(g.mlp_params())
    diff = np.abs(got - join_params(p))
    # Adam's first steps move each parameter by about lr times the sign of its
    # gradient, so an element whose gradient is zero to rounding may move the
    # other way
    assert np.mean(diff <= 1e-5) >= 0.995
    assert diff.max() <= 4.0 * cfg.surrogate_lr + 1e-5
    log = g.surrogate_log()
    assert abs(log[0, 2] - loss) <= 1e-3 * loss
    g.close()


def test_run_replays_equal_eager_steps():
    announce("offspring run (graph) vs eager steps")
    kw = dict(P=48, n_off=384, frac=0.25, steps=2, audit=24, batch=64, H=32, seed=8080,
              max_generations=5)
    a, _ = make("mlp", **kw)
    b, _ = make("mlp", **kw)
    res = a.run()
    assert res["generations"] == 5 and res["stop_reason"] == "max_generations"
    for _ in range(5):
        b.step()
    assert np.array_equal(bits(host(a.population)), bits(host(b.population)))
    assert np.array_equal(bits(host(a.mlp_params())), bits(host(b.mlp_params())))
    la, lb = a.surrogate_log(), b.surrogate_log()
    assert la.shape == (5, 3) and np.array_equal(bits(la), bits(lb))
    sa, sb = a.state(), b.state()
    assert sa["generation"] == sb["generation"] == 5
    assert sa["best_mse"] == sb["best_mse"] == res["best_mse"]
    # a second run continues from where the first stopped
    res2 = a.run()
    assert res2["generations"] == 5 and a.state()["generation"] == 10
    assert res2["best_mse"] <= res["best_mse"]
    a.close()
    b.close()


def test_learned_prescreen_beats_random():
    """Same budget of exact evaluations per generation (the audit aside): the
    MLP's choices rank better than chance and reach a lower MSE."""
    announce("learned vs random prescreen")
    # a small network on a short run: the larger step size suits it (the
    # library default, 3e-4, is the one measured best at the 1M-pattern,
    # 128-gene workload over hundreds of generations)
    kw = dict(P=64, n_off=1024, frac=0.125, steps=32, audit=64, batch=256, H=64, buffer=16384,
              N=20000, F=6, D=6, seed=606, max_generations=40, surrogate_lr=3e-3)
    a, _ = make("mlp", **kw)
    b, _ = make("random", **kw)
    ra, rb = a.run(), b.run()
    log = a.surrogate_log()
    rho_audit = float(np.mean(log[20:, 0]))
    print(f"mlp best {ra['best_mse']:.6g} random best {rb['best_mse']:.6g} "
          f"rho_audit(last 20) {rho_audit:.3f} rho_sel {np.mean(log[20:, 1]):.3f}")
    assert np.all(np.isfinite(log))
    assert rho_audit > 0.2
    assert ra["best_mse"] < rb["best_mse"]
    a.close()
    b.close()


def test_advance_equals_steps_in_offspring_form():
    announce("offspring advance (graph) vs eager steps")
    kw = dict(P=32, n_off=160, frac=0.5, steps=1, audit=8, batch=32, H=16, seed=99)
    a, _ = make("mlp", **kw)
    b, _ = make("mlp", **kw)
    a.advance(11)          # one chunk of 8 and a 3-generation graph
    for _ in range(11):
        b.step()
    assert np.array_equal(bits(host(a.population)), bits(host(b.population)))
    assert np.array_equal(bits(host(a.mlp_params())), bits(host(b.mlp_params())))
    assert a.state() == b.state()
    a.close()
    b.close()


def test_workload_c5_full_size_sampled():
    """The surrogate workload at its benchmarked shape (1M patterns, 16
    features, Legendre D = 8, P = 2048, 8192 offspring, MLP 128-256-256-1,
    16 steps of 2048 rows, 256-child audit), one generation after the
    warm-up: the children are the oracle's, the MLP scores (sampled) match
    the oracle's forward pass, the prescreen keeps the elites and only
    children from the oracle's selection by those scores, the survivors'
    exact MSE (sampled) match the float64 oracle, and the logged Spearman
    statistics match the oracle's on the device's scores and errors."""
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    from oracle import model
    N, F, D, P, n_off, A, k = 1_000_000, 16, 8, 2048, 8192, 256, 2048
    X, t = synth.classification_dataset(N, F, seed=synth.data_seed(3))
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", task="classification",
                 dtype="f32", pop_size=P, n_offspring=n_off, surrogate="mlp", prescreen_frac=0.25,
                 audit=A, surrogate_hidden=256, surrogate_buffer=50000, surrogate_batch=2048,
                 surrogate_steps=16, tournament_k=K_TOURN, p_crossover=PC, p_mutation=PM,
                 mutation_sigma=SIGMA, seed=synth.ga_seed(5))
    g = Game(cfg, dev(X, torch.float32), dev(t, torch.float32))
    announce("c5 full size: warm-up and generation 0")
    g.step()
    pop = host(g.population)
    fit = host(g.eval_fitness()[2])
    children = children_of(pop, fit, 1, n_off, cfg.seed)
    params = split_params(host(g.mlp_params()), g.L, 256)
    announce("c5 full size: scores of the 8192 children")
    yhat = host(g.mlp_forward(dev(children, torch.float32)))
    rows = np.random.default_rng(5).choice(n_off, 256, replace=False)
    ref_y = mlp.forward(params, children[rows])["y"]
    assert np.abs(yhat[rows] - ref_y).max() <= 1e-4 * max(1.0, np.abs(ref_y).max())
    sel = rank.smallest_k(yhat, k)
    aud = rank.smallest_k(rank.random_keys(n_off, 1, rank.TAG_AUDIT, cfg.seed), A)
    announce("c5 full size: generation 1")
    g.step()
    new = host(g.population)
    E = cfg.elitism
    assert np.array_equal(bits(new[:E]), bits(pop[ga.elites(fit, E)]))
    assert drawn_from(children[sel], new[E:])
    mse_new = host(g.eval_fitness()[0])
    # the survivors' exact MSE against the float64 oracle (sampled)
    idx = np.array([0, E, P - 1])
    Xo = X.astype(np.float32).astype(np.float64)
    to = t.astype(np.float32).astype(np.float64)
    ref = model.evaluate(Xo, to, new[idx].astype(np.float64), "legendre", D, "classification")
    np.testing.assert_allclose(mse_new[idx], ref["mse"], rtol=1e-5)
    # the logged rank statistics of generation 1, from the device's values
    mse_sel = host(g.eval_fitness(dev(children[sel], torch.float32))[0])
    mse_aud = host(g.eval_fitness(dev(children[aud], torch.float32))[0])
    log = g.surrogate_log()
    assert log.shape[0] == 2
    assert abs(log[1, 0] - rank.spearman(yhat[aud], mse_aud)) <= 1e-5
    assert abs(log[1, 1] - rank.spearman(yhat[sel], mse_sel)) <= 1e-5
    g.close()

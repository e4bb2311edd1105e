"""Checkpoint and resume: a context that loads a checkpoint continues bit for
bit as the context that saved it (the random draws are counter based)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def make(**kw):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, Game
    X, t = synth.classification_dataset(6000, 6, seed=31)
    cfg = Config(n_patterns=6000, n_features=6, degree=4, basis="trig", task="classification",
                 dtype="f32", pop_size=96, max_generations=6, seed=77, **kw)
    Xd, td = dev(X, torch.float32), dev(t, torch.float32)
    return (lambda c=cfg: Game(c, Xd, td)), cfg


def test_resume_generational_form():
    new, cfg = make()
    a = new()
    announce("checkpoint: generational form")
    a.run()
    blob = a.save()
    ra = a.run()
    b = new()
    b.load(blob)
    rb = b.run()
    assert ra["generations"] == rb["generations"] == 6
    assert np.array_equal(bits(ra["best_genes"]), bits(rb["best_genes"]))
    assert np.array_equal(bits(host(a.population)), bits(host(b.population)))
    assert a.state() == b.state()
    # resuming with other run limits is allowed; stepping after a load works
    from paper_1211_5481_amd import Config
    c = new(Config(**{**cfg.__dict__, "max_generations": 3}))
    c.load(blob)
    rc = c.run()
    assert rc["generations"] == 3
    a.close(); b.close(); c.close()


def test_resume_surrogate_form():
    new, cfg = make(n_offspring=512, surrogate="mlp", prescreen_frac=0.25, audit=16,
                    surrogate_steps=2, surrogate_batch=64, surrogate_hidden=32,
                    surrogate_buffer=4096)
    a = new()
    announce("checkpoint: surrogate form")
    a.run()
    blob = a.save()
    a.run()
    b = new()
    b.load(blob)
    b.run()
    assert np.array_equal(bits(host(a.population)), bits(host(b.population)))
    assert np.array_equal(bits(host(a.mlp_params())), bits(host(b.mlp_params())))
    la, lb = a.surrogate_log(), b.surrogate_log()
    assert la.shape == lb.shape == (12, 3) and np.array_equal(bits(la), bits(lb))
    ga, ya, *ra = a.surrogate_buffer()
    gb, yb, *rb = b.surrogate_buffer()
    assert ra == rb and np.array_equal(bits(host(ga)), bits(host(gb)))
    a.close(); b.close()


def test_load_rejects_foreign_checkpoints():
    from paper_1211_5481_amd import Config, _lib
    new, cfg = make()
    a = new()
    announce("checkpoint: mismatches")
    a.run()
    blob = a.save()
    other = new(Config(**{**cfg.__dict__, "seed": 78}))
    with pytest.raises(_lib.GameError) as e:
        other.load(blob)
    assert e.value.status == _lib.GAME_E_INVALID
    with pytest.raises(_lib.GameError):
        new().load(blob[:100])
    with pytest.raises(_lib.GameError):
        new().load(b"X" * len(blob))
    a.close(); other.close()

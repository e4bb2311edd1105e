"""Host-side checks of the C ABI: the library loads, exports every function
include/game.h declares, and validates configurations before any launch.
No call here touches a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1211_5481_amd import _lib as L
from paper_1211_5481_amd.game import Config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "game.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(game_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 15
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in game.h but not exported"
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def test_struct_layouts_match_the_header():
    # sizes computed by the C compiler for the declared structs
    assert C.sizeof(L.GameConfig) == 168
    assert C.sizeof(L.GameDims) == 40
    assert C.sizeof(L.GameResult) == 40
    assert C.sizeof(L.GameState) == 40


def _query(**kw):
    base = dict(n_patterns=1000, n_features=8, degree=4, basis="chebyshev", dtype="f64", pop_size=20)
    base.update(kw)
    d = L.GameDims()
    st = L.lib().game_query(C.byref(Config(**base).to_c()), C.byref(d))
    return st, d


def test_query_derived_sizes():
    st, d = _query()
    assert st == L.GAME_OK
    assert (d.K, d.M, d.L, d.M_pad, d.P, d.n_offspring) == (4, 32, 32, 32, 20, 18)
    assert d.N_pad == 1024
    st, d = _query(n_patterns=100000, n_features=10, degree=6, basis="trig", task="classification",
                   dtype="f32", pop_size=1000)
    assert (d.K, d.M, d.L, d.M_pad) == (12, 120, 120, 120)
    st, d = _query(n_features=10, degree=6, basis="trig", dtype="bf16", bias=1, pop_size=0)
    assert (d.M, d.L, d.M_pad, d.P) == (120, 121, 128, 21)     # P = B*F + 1 (eq. 4)
    assert d.workspace_bytes % 256 == 0 and d.workspace_bytes > 0
    # shared-coefficient model: B*d genes plus a_0 (eq. 5), P = B*F + 1 (eq. 4)
    st, d = _query(n_features=7, degree=4, basis="trig", dtype="f32", bias=1, shared=1, pop_size=0)
    assert st == L.GAME_OK and (d.K, d.M, d.L, d.P) == (8, 8, 9, 15)


@pytest.mark.parametrize("kw,status", [
    (dict(n_patterns=0), L.GAME_E_INVALID),
    (dict(n_features=0), L.GAME_E_INVALID),
    (dict(degree=0), L.GAME_E_INVALID),
    (dict(pop_size=-1), L.GAME_E_INVALID),
    (dict(elitism=21), L.GAME_E_INVALID),
    (dict(elitism=65, pop_size=100), L.GAME_E_INVALID),
    (dict(tournament_k=0), L.GAME_E_INVALID),
    (dict(tournament_k=17), L.GAME_E_INVALID),
    (dict(p_crossover=1.5), L.GAME_E_INVALID),
    (dict(p_mutation=-0.1), L.GAME_E_INVALID),
    (dict(mutation_sigma=float("inf")), L.GAME_E_INVALID),
    (dict(mse_threshold=float("nan")), L.GAME_E_INVALID),
    (dict(max_generations=0), L.GAME_E_INVALID),
    (dict(bias=2), L.GAME_E_INVALID),
    (dict(n_features=600, degree=8, basis="trig"), L.GAME_E_INVALID),
    (dict(n_features=256, degree=8, basis="trig"), L.GAME_OK),              # L = 4096, the limit
    (dict(n_features=256, degree=8, basis="trig", bias=1), L.GAME_E_INVALID),  # L = 4097
    (dict(n_offspring=7), L.GAME_E_INVALID),            # cannot refill P - elitism
    (dict(n_offspring=9000), L.GAME_E_INVALID),
    (dict(surrogate="mlp", n_offspring=80, prescreen_frac=0.1), L.GAME_E_INVALID),
    (dict(surrogate="mlp", n_offspring=80, prescreen_frac=0.0), L.GAME_E_INVALID),
    (dict(surrogate="mlp", n_offspring=80, surrogate_hidden=8), L.GAME_E_INVALID),
    (dict(surrogate="mlp", n_offspring=80, surrogate_buffer=10, surrogate_batch=64), L.GAME_E_INVALID),
    (dict(surrogate="mlp", n_offspring=80, audit=5000), L.GAME_E_INVALID),
    (dict(surrogate="random", n_offspring=80, surrogate_lr=0.0), L.GAME_OK),
    (dict(surrogate="mlp", n_offspring=80, surrogate_recent=1.5), L.GAME_E_INVALID),
    (dict(n_offspring=40, dtype="f32", rescore_top=1), L.GAME_E_UNSUPPORTED),
    (dict(tile_p=128), L.GAME_E_INVALID),                       # F64 tiles are 64 wide
    (dict(dtype="f32", tile_p=48), L.GAME_E_INVALID),
    (dict(dtype="f32", tile_p=128, n_features=20, degree=8, basis="trig"), L.GAME_E_INVALID),
    (dict(dtype="f32", tile_p=64, n_features=20, degree=8, basis="trig"), L.GAME_OK),
    (dict(dtype="f32", row_groups=-1), L.GAME_E_INVALID),
])
def test_invalid_configs_rejected(kw, status):
    st, _ = _query(**kw)
    assert st == status
    if status != L.GAME_OK:
        assert L.lib().game_last_error()


def test_offspring_form_sizes():
    st, d = _query(n_offspring=40)
    assert st == L.GAME_OK and d.n_offspring == 40
    st0, d0 = _query()
    st1, d1 = _query(surrogate="mlp", n_offspring=80, prescreen_frac=0.25, audit=16)
    assert st1 == L.GAME_OK and d1.workspace_bytes > d0.workspace_bytes


def test_bad_enum_and_struct_size():
    c = Config(n_patterns=10, n_features=2).to_c()
    c.struct_size = 8
    assert L.lib().game_query(C.byref(c), C.byref(L.GameDims())) == L.GAME_E_INVALID
    c = Config(n_patterns=10, n_features=2).to_c()
    c.basis = 9
    assert L.lib().game_query(C.byref(c), C.byref(L.GameDims())) == L.GAME_E_INVALID
    c.basis = 0
    c.dtype = 7
    assert L.lib().game_query(C.byref(c), C.byref(L.GameDims())) == L.GAME_E_INVALID


def test_init_rejects_bad_arguments_without_launching():
    cfg = Config(n_patterns=100, n_features=3, pop_size=8).to_c()
    ctx = C.c_void_p()
    need = C.c_size_t()
    assert L.lib().game_workspace_size(C.byref(cfg), C.byref(need)) == L.GAME_OK
    # NULL device pointers, misaligned or small workspaces: all refused before any launch
    assert L.lib().game_init(C.byref(cfg), None, None, None, 0, None, C.byref(ctx)) == L.GAME_E_INVALID
    fake = 1 << 40
    assert L.lib().game_init(C.byref(cfg), fake, fake, fake + 8, need.value, None,
                             C.byref(ctx)) == L.GAME_E_INVALID
    assert L.lib().game_init(C.byref(cfg), fake, fake, fake, need.value - 256, None,
                             C.byref(ctx)) == L.GAME_E_OOM
    assert ctx.value is None
    assert L.lib().game_eval_fitness(None, None, 8, None, None, None) == L.GAME_E_INVALID
    assert L.lib().game_step(None, None) == L.GAME_E_INVALID
    assert L.lib().game_status_str(L.GAME_E_OOM) == b"GAME_E_OOM"


def _batch_size(cfgs):
    arr = (L.GameConfig * len(cfgs))(*[c.to_c() for c in cfgs])
    need = C.c_size_t()
    return L.lib().game_batch_workspace_size(arr, len(cfgs), C.byref(need)), need.value


def test_batch_validation_without_launching():
    a = Config(n_patterns=1000, n_features=4, degree=3, dtype="f32", pop_size=64)
    b = Config(n_patterns=5000, n_features=6, degree=4, basis="trig", task="classification",
               dtype="f32", pop_size=256)
    st, need = _batch_size([a, b])
    assert st == L.GAME_OK
    sa, na = _query_ws(a)
    sb, nb = _query_ws(b)
    assert need > na + nb
    assert _batch_size([a, Config(**{**b.__dict__, "dtype": "bf16"})])[0] == L.GAME_E_INVALID
    assert _batch_size([Config(**{**a.__dict__, "dtype": "f64"})])[0] == L.GAME_E_UNSUPPORTED
    assert _batch_size([Config(**{**a.__dict__, "n_offspring": 128})])[0] == L.GAME_E_UNSUPPORTED
    assert _batch_size([Config(**{**a.__dict__, "rescore_top": 1})])[0] == L.GAME_E_UNSUPPORTED
    assert _batch_size([])[0] == L.GAME_E_INVALID
    # a batch needs device memory: init refuses a NULL workspace before any launch
    arr = (L.GameConfig * 1)(a.to_c())
    xs = (C.c_void_p * 1)(None)
    out = C.c_void_p()
    assert L.lib().game_batch_init(arr, 1, xs, xs, None, 0, None, C.byref(out)) != L.GAME_OK


def _query_ws(cfg):
    need = C.c_size_t()
    return L.lib().game_workspace_size(C.byref(cfg.to_c()), C.byref(need)), need.value


def test_checkpoint_arguments_without_a_context():
    n = C.c_size_t()
    assert L.lib().game_save(None, None, C.byref(n)) == L.GAME_E_INVALID
    assert L.lib().game_load(None, None, 0) == L.GAME_E_INVALID


def test_selection_and_immigrant_validation():
    st, _ = _query(selection="ranking", pop_size=9000, dtype="f32")
    assert st == L.GAME_E_INVALID
    assert _query(selection="roulette", n_immigrants=18)[0] == L.GAME_OK
    assert _query(n_immigrants=19)[0] == L.GAME_E_INVALID        # more than P - E children
    assert _query(n_immigrants=-1)[0] == L.GAME_E_INVALID
    c = Config(n_patterns=100, n_features=2).to_c()
    c.selection = 3
    assert L.lib().game_query(C.byref(c), C.byref(L.GameDims())) == L.GAME_E_INVALID
    c.selection = 0
    c.shared = 2
    assert L.lib().game_query(C.byref(c), C.byref(L.GameDims())) == L.GAME_E_INVALID

"""ctypes declarations of libgame.so (the C ABI in include/game.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgame.so")

GAME_OK, GAME_E_INVALID, GAME_E_OOM, GAME_E_DEVICE, GAME_E_STATE, GAME_E_UNSUPPORTED = range(6)
BASIS = {"power": 0, "chebyshev": 1, "legendre": 2, "trig": 3}
TASK = {"regression": 0, "classification": 1}
DTYPE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
STOP = {0: "none", 1: "threshold", 2: "max_generations"}
SURROGATE = {"none": 0, "mlp": 1, "random": 2}
SELECTION = {"tournament": 0, "roulette": 1, "ranking": 2}


class GameMetrics(C.Structure):
    _fields_ = [("n", C.c_int64), ("mse", C.c_double), ("rmse", C.c_double),
                ("accuracy", C.c_double), ("completeness", C.c_double),
                ("contamination", C.c_double), ("tp", C.c_int64), ("fp", C.c_int64),
                ("tn", C.c_int64), ("fn", C.c_int64)]


class GameConfig(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("basis", C.c_int32),
        ("n_patterns", C.c_int64),
        ("n_features", C.c_int32),
        ("degree", C.c_int32),
        ("task", C.c_int32),
        ("dtype", C.c_int32),
        ("bias", C.c_int32),
        ("pop_size", C.c_int32),
        ("n_offspring", C.c_int32),
        ("elitism", C.c_int32),
        ("selection", C.c_int32),
        ("tournament_k", C.c_int32),
        ("n_immigrants", C.c_int32),
        ("shared", C.c_int32),
        ("max_generations", C.c_int32),
        ("rescore_top", C.c_int32),
        ("tile_p", C.c_int32),
        ("row_groups", C.c_int32),
        ("surrogate", C.c_int32),
        ("surrogate_hidden", C.c_int32),
        ("surrogate_buffer", C.c_int32),
        ("surrogate_steps", C.c_int32),
        ("surrogate_batch", C.c_int32),
        ("audit", C.c_int32),
        ("prescreen_frac", C.c_double),
        ("surrogate_lr", C.c_double),
        ("surrogate_recent", C.c_double),
        ("p_crossover", C.c_double),
        ("p_mutation", C.c_double),
        ("mutation_sigma", C.c_double),
        ("mse_threshold", C.c_double),
        ("seed", C.c_uint64),
    ]


class GameDims(C.Structure):
    _fields_ = [
        ("K", C.c_int32),
        ("M", C.c_int32),
        ("L", C.c_int32),
        ("M_pad", C.c_int32),
        ("P", C.c_int32),
        ("n_offspring", C.c_int32),
        ("N_pad", C.c_int64),
        ("workspace_bytes", C.c_size_t),
    ]


class GameResult(C.Structure):
    _fields_ = [
        ("best_mse", C.c_double),
        ("best_fitness", C.c_double),
        ("best_miscls", C.c_double),
        ("generations", C.c_int32),
        ("stop_reason", C.c_int32),
        ("best_genes", C.POINTER(C.c_float)),
    ]


class GameState(C.Structure):
    _fields_ = [
        ("generation", C.c_int32),
        ("stopped", C.c_int32),
        ("best_index", C.c_int32),
        ("stop_reason", C.c_int32),
        ("best_mse", C.c_double),
        ("best_fitness", C.c_double),
        ("best_miscls", C.c_double),
    ]


# name -> (restype, argtypes); the exported symbols of include/game.h
_VP = C.c_void_p
SIGNATURES = {
    "game_config_default": (None, [C.POINTER(GameConfig)]),
    "game_query": (C.c_int, [C.POINTER(GameConfig), C.POINTER(GameDims)]),
    "game_workspace_size": (C.c_int, [C.POINTER(GameConfig), C.POINTER(C.c_size_t)]),
    "game_build_basis": (C.c_int, [C.POINTER(GameConfig), _VP, _VP, C.c_int64, _VP]),
    "game_init": (C.c_int, [C.POINTER(GameConfig), _VP, _VP, _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "game_eval_fitness": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP]),
    "game_step": (C.c_int, [_VP, _VP]),
    "game_advance": (C.c_int, [_VP, C.c_int32]),
    "game_advance_prepare": (C.c_int, [_VP, C.c_int32]),
    "game_run": (C.c_int, [_VP, C.POINTER(GameResult)]),
    "game_rescore": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP]),
    "game_rescore_noalloc": (C.c_int, [C.POINTER(GameConfig), _VP, _VP, _VP, C.c_int32, _VP, _VP,
                                       _VP]),
    "game_surrogate_log": (C.c_int, [_VP, _VP, C.c_int32, C.POINTER(C.c_int32)]),
    "game_surrogate_buffer": (C.c_int, [_VP, _VP, _VP, C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "game_mlp_params": (C.c_int, [_VP, _VP, C.c_int32]),
    "game_mlp_forward": (C.c_int, [_VP, _VP, C.c_int32, _VP]),
    "game_mlp_grads": (C.c_int, [_VP, _VP, _VP, C.c_int32, _VP, _VP]),
    "game_mlp_adam": (C.c_int, [_VP, _VP]),
    "game_batch_workspace_size": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_size_t)]),
    "game_batch_init": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "game_batch_tiles": (C.c_int, [_VP, _VP, _VP]),
    "game_batch_context": (C.c_int, [_VP, C.c_int32, C.POINTER(_VP)]),
    "game_batch_time_fitness": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_float)]),
    "game_batch_run": (C.c_int, [_VP, _VP, _VP]),
    "game_batch_destroy": (None, [_VP]),
    "game_run_batched": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, C.c_size_t, _VP, _VP, _VP]),
    "game_predict": (C.c_int, [_VP, _VP, _VP, C.c_int64, _VP]),
    "game_evaluate": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int64, C.POINTER(GameMetrics)]),
    "game_save": (C.c_int, [_VP, _VP, C.POINTER(C.c_size_t)]),
    "game_load": (C.c_int, [_VP, _VP, C.c_size_t]),
    "game_get_population": (C.c_int, [_VP, _VP]),
    "game_set_population": (C.c_int, [_VP, _VP]),
    "game_get_state": (C.c_int, [_VP, C.POINTER(GameState), _VP]),
    "game_time_fitness": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_float)]),
    "game_destroy": (None, [_VP]),
    "game_status_str": (C.c_char_p, [C.c_int]),
    "game_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1211_5481_amd.build` "
                "(the GAME hot path has no CPU fallback)")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


class GameError(RuntimeError):
    def __init__(self, status: int, where: str):
        name = lib().game_status_str(status).decode()
        msg = lib().game_last_error().decode()
        super().__init__(f"{where}: {name}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != GAME_OK:
        raise GameError(status, where)

"""Python binding of libgame with the C ABI's names.

PyTorch provides device memory (the workspace, inputs and outputs) and the
stream; every step of the fitness path and of the genetic operators runs in
the library's HIP kernels.  Nothing here computes on the CPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _lib as L


@dataclass
class Config:
    """Mirror of game_config (include/game.h) with readable enum values."""
    n_patterns: int
    n_features: int
    degree: int = 4
    basis: str = "chebyshev"          # power | chebyshev | legendre | trig
    task: str = "regression"          # regression | classification
    dtype: str = "f32"                # f64 | f32 | bf16 | f16
    bias: int = 0
    shared: int = 0                   # 1: one coefficient per basis function for all features
    pop_size: int = 0                 # 0 -> B*F + 1 (eq. 4)
    n_offspring: int = 0
    elitism: int = 2
    tournament_k: int = 3
    selection: str = "tournament"     # tournament | roulette | ranking
    n_immigrants: int = 0
    max_generations: int = 100
    rescore_top: int = 0              # per-generation float32 re-score of the top-k
    tile_p: int = 0                   # fitness tile width: 0 (library's choice) | 32 | 64 | 128
    row_groups: int = 0               # fitness row ranges: 0 (library's choice) | R
    surrogate: str = "none"           # offspring form prescreen: none | mlp | random
    surrogate_hidden: int = 256
    surrogate_buffer: int = 50000
    surrogate_steps: int = 16
    surrogate_batch: int = 2048
    audit: int = 256
    prescreen_frac: float = 0.25
    surrogate_lr: float = 3e-4
    surrogate_recent: float = 0.75
    p_crossover: float = 0.9
    p_mutation: float = 0.05
    mutation_sigma: float = 0.1
    mse_threshold: float = 0.0
    seed: int = 0

    def to_c(self) -> L.GameConfig:
        c = L.GameConfig()
        L.lib().game_config_default(C.byref(c))
        c.basis = L.BASIS[self.basis]
        c.n_patterns = int(self.n_patterns)
        c.n_features = int(self.n_features)
        c.degree = int(self.degree)
        c.task = L.TASK[self.task]
        c.dtype = L.DTYPE[self.dtype]
        c.bias = int(self.bias)
        c.shared = int(self.shared)
        c.pop_size = int(self.pop_size)
        c.n_offspring = int(self.n_offspring)
        c.elitism = int(self.elitism)
        c.selection = L.SELECTION[self.selection]
        c.n_immigrants = int(self.n_immigrants)
        c.tournament_k = int(self.tournament_k)
        c.max_generations = int(self.max_generations)
        c.rescore_top = int(self.rescore_top)
        c.tile_p = int(self.tile_p)
        c.row_groups = int(self.row_groups)
        c.surrogate = L.SURROGATE[self.surrogate]
        c.surrogate_hidden = int(self.surrogate_hidden)
        c.surrogate_buffer = int(self.surrogate_buffer)
        c.surrogate_steps = int(self.surrogate_steps)
        c.surrogate_batch = int(self.surrogate_batch)
        c.audit = int(self.audit)
        c.prescreen_frac = float(self.prescreen_frac)
        c.surrogate_lr = float(self.surrogate_lr)
        c.surrogate_recent = float(self.surrogate_recent)
        c.p_crossover = float(self.p_crossover)
        c.p_mutation = float(self.p_mutation)
        c.mutation_sigma = float(self.mutation_sigma)
        c.mse_threshold = float(self.mse_threshold)
        c.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        return c

    @property
    def io_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def query(cfg: Config) -> L.GameDims:
    d = L.GameDims()
    L.check(L.lib().game_query(C.byref(cfg.to_c()), C.byref(d)), "game_query")
    return d


def workspace_size(cfg: Config) -> int:
    n = C.c_size_t()
    L.check(L.lib().game_workspace_size(C.byref(cfg.to_c()), C.byref(n)), "game_workspace_size")
    return n.value


_STORAGE = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}


def build_basis(cfg: Config, X, ld: Optional[int] = None, stream=None):
    """Phi (N x ld, storage dtype) for device patterns X (N x F)."""
    torch = _torch()
    d = query(cfg)
    ld = d.M if ld is None else int(ld)
    X = X.contiguous()
    if X.dtype != cfg.io_dtype or not X.is_cuda:
        raise ValueError(f"X must be a {cfg.io_dtype} CUDA tensor")
    phi = torch.empty((cfg.n_patterns, ld), dtype=getattr(torch, _STORAGE[cfg.dtype]), device=X.device)
    L.check(L.lib().game_build_basis(C.byref(cfg.to_c()), _ptr(X), _ptr(phi), ld,
                                     _stream_handle(stream)), "game_build_basis")
    return phi


def rescore_noalloc(cfg: Config, X, t, genes, stream=None):
    """Float32 (mse, miscls) of n <= 8 chromosomes (n x L) on device patterns
    X (N x F) and targets t, with no context and no allocation inside the
    library (game_rescore_noalloc; the outputs are allocated here)."""
    torch = _torch()
    d = query(cfg)
    X, t, genes = X.contiguous(), t.contiguous(), genes.contiguous()
    if genes.dtype != torch.float32 or genes.dim() != 2 or genes.shape[1] != d.L:
        raise ValueError("genes must be a float32 n x L CUDA tensor")
    n = genes.shape[0]
    out = torch.empty((2, n), dtype=torch.float64, device=genes.device)
    L.check(L.lib().game_rescore_noalloc(C.byref(cfg.to_c()), _ptr(X), _ptr(t), _ptr(genes), int(n),
                                         _ptr(out[0]), _ptr(out[1]), _stream_handle(stream)),
            "game_rescore_noalloc")
    return out[0], out[1]


class Game:
    """A GAME training context (game_init ... game_destroy)."""

    def __init__(self, cfg: Config, X, t, stream=None):
        torch = _torch()
        self.cfg = cfg
        self.dims = query(cfg)
        if X.shape != (cfg.n_patterns, cfg.n_features) or t.shape != (cfg.n_patterns,):
            raise ValueError("X must be N x F and t must have N entries")
        for name, a in (("X", X), ("t", t)):
            if a.dtype != cfg.io_dtype or not a.is_cuda:
                raise ValueError(f"{name} must be a {cfg.io_dtype} CUDA tensor")
        self.device = X.device
        self._stream = stream
        self._X = X.contiguous()
        self._t = t.contiguous()
        self.workspace = torch.empty(self.dims.workspace_bytes + 256, dtype=torch.uint8,
                                     device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        ctx = C.c_void_p()
        L.check(L.lib().game_init(C.byref(cfg.to_c()), _ptr(self._X), _ptr(self._t),
                                  self._ws_ptr, self.dims.workspace_bytes,
                                  _stream_handle(stream), C.byref(ctx)), "game_init")
        self._ctx = ctx

    @property
    def P(self) -> int:
        return self.dims.P

    @property
    def L(self) -> int:
        return self.dims.L

    def eval_fitness(self, genes=None):
        """(mse, miscls, fitness) float64 device tensors for genes (P x L) or the population."""
        torch = _torch()
        if genes is not None:
            genes = genes.contiguous()
            if genes.dtype != torch.float32 or genes.dim() != 2 or genes.shape[1] != self.L:
                raise ValueError("genes must be a float32 P x L CUDA tensor")
            P = genes.shape[0]
        else:
            P = self.P
        out = torch.empty((3, P), dtype=torch.float64, device=self.device)
        L.check(L.lib().game_eval_fitness(self._ctx, _ptr(genes), P, _ptr(out[0]),
                                          _ptr(out[1]), _ptr(out[2])), "game_eval_fitness")
        return out[0], out[1], out[2]

    def step(self, fitness=None):
        if fitness is not None:
            fitness = fitness.contiguous()
            if fitness.dtype != _torch().float64 or fitness.shape != (self.P,):
                raise ValueError("fitness must be a float64 CUDA tensor of P entries")
        L.check(L.lib().game_step(self._ctx, _ptr(fitness)), "game_step")

    def advance(self, n_generations: int):
        L.check(L.lib().game_advance(self._ctx, int(n_generations)), "game_advance")

    def prepare(self, n_generations: int):
        """Capture the graphs advance(n_generations) replays, running nothing."""
        L.check(L.lib().game_advance_prepare(self._ctx, int(n_generations)),
                "game_advance_prepare")

    def run(self) -> dict:
        genes = (C.c_float * self.L)()
        r = L.GameResult()
        r.best_genes = C.cast(genes, C.POINTER(C.c_float))
        L.check(L.lib().game_run(self._ctx, C.byref(r)), "game_run")
        return dict(best_mse=r.best_mse, best_fitness=r.best_fitness, best_miscls=r.best_miscls,
                    generations=r.generations, stop_reason=L.STOP.get(r.stop_reason),
                    best_genes=np.frombuffer(genes, dtype=np.float32).copy())

    def rescore(self, genes=None, n: int = None):
        """Float32 (mse, miscls) of n chromosomes: genes (n x L) or the population's n best."""
        torch = _torch()
        if genes is not None:
            genes = genes.contiguous()
            if genes.dtype != torch.float32 or genes.dim() != 2 or genes.shape[1] != self.L:
                raise ValueError("genes must be a float32 n x L CUDA tensor")
            n = genes.shape[0]
        elif n is None:
            n = 1
        out = torch.empty((2, n), dtype=torch.float64, device=self.device)
        L.check(L.lib().game_rescore(self._ctx, _ptr(genes), int(n), _ptr(out[0]), _ptr(out[1])),
                "game_rescore")
        return out[0], out[1]

    def surrogate_log(self, n_max: int = 4096):
        """Per-generation (rho_audit, rho_selected, loss) of the offspring form, oldest first."""
        buf = (C.c_float * (4 * n_max))()
        n = C.c_int32()
        L.check(L.lib().game_surrogate_log(self._ctx, buf, int(n_max), C.byref(n)), "game_surrogate_log")
        return np.frombuffer(buf, dtype=np.float32)[:4 * n.value].reshape(n.value, 4)[:, :3].copy()

    def surrogate_buffer(self):
        """Replay buffer: (genes cap x L, log-MSE targets, count, head, mu, sigma)."""
        torch = _torch()
        cap = self.cfg.surrogate_buffer
        genes = torch.empty((cap, self.L), dtype=torch.float32, device=self.device)
        y = torch.empty(cap, dtype=torch.float32, device=self.device)
        ch = (C.c_int32 * 2)()
        ms = (C.c_float * 2)()
        L.check(L.lib().game_surrogate_buffer(self._ctx, _ptr(genes), _ptr(y), ch, ms),
                "game_surrogate_buffer")
        return genes, y, int(ch[0]), int(ch[1]), float(ms[0]), float(ms[1])

    def mlp_params(self, params=None):
        """Get (params None) or set the surrogate's flat float32 parameter vector."""
        torch = _torch()
        if params is None:
            n = self.mlp_size()
            out = torch.empty(n, dtype=torch.float32, device=self.device)
            L.check(L.lib().game_mlp_params(self._ctx, _ptr(out), 0), "game_mlp_params")
            return out
        params = params.contiguous()
        L.check(L.lib().game_mlp_params(self._ctx, _ptr(params), 1), "game_mlp_params")
        self._mlp_keep = params

    def mlp_size(self) -> int:
        H, Lg = self.cfg.surrogate_hidden, self.L
        return H * Lg + H + H * H + H + H + 1

    def _rows(self, X):
        X = X.contiguous()
        if X.dtype != _torch().float32 or X.dim() != 2 or X.shape[1] != self.L or not X.is_cuda:
            raise ValueError("rows must be a float32 n x L CUDA tensor")
        return X

    def mlp_forward(self, X):
        torch = _torch()
        X = self._rows(X)
        y = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        L.check(L.lib().game_mlp_forward(self._ctx, _ptr(X), X.shape[0], _ptr(y)), "game_mlp_forward")
        return y

    def mlp_grads(self, X, target):
        torch = _torch()
        X, target = self._rows(X), target.contiguous()
        if target.dtype != torch.float32 or target.shape != (X.shape[0],):
            raise ValueError("target must be a float32 CUDA tensor of n entries")
        g = torch.empty(self.mlp_size(), dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        L.check(L.lib().game_mlp_grads(self._ctx, _ptr(X), _ptr(target), X.shape[0], _ptr(g),
                                       _ptr(loss)), "game_mlp_grads")
        return g, loss

    def mlp_adam(self, grads):
        grads = grads.contiguous()
        L.check(L.lib().game_mlp_adam(self._ctx, _ptr(grads)), "game_mlp_adam")
        self._grad_keep = grads

    @property
    def population(self):
        torch = _torch()
        out = torch.empty((self.P, self.L), dtype=torch.float32, device=self.device)
        L.check(L.lib().game_get_population(self._ctx, _ptr(out)), "game_get_population")
        return out

    @population.setter
    def population(self, genes):
        torch = _torch()
        genes = genes.contiguous()
        if genes.dtype != torch.float32 or tuple(genes.shape) != (self.P, self.L):
            raise ValueError("population must be a float32 P x L CUDA tensor")
        L.check(L.lib().game_set_population(self._ctx, _ptr(genes)), "game_set_population")
        self._pop_keep = genes  # keep alive until the async copy has run

    def state(self, with_genes: bool = False) -> dict:
        s = L.GameState()
        genes = (C.c_float * self.L)() if with_genes else None
        L.check(L.lib().game_get_state(self._ctx, C.byref(s), genes), "game_get_state")
        d = dict(generation=s.generation, stopped=bool(s.stopped), best_index=s.best_index,
                 stop_reason=L.STOP.get(s.stop_reason), best_mse=s.best_mse,
                 best_fitness=s.best_fitness, best_miscls=s.best_miscls)
        if with_genes:
            d["best_genes"] = np.frombuffer(genes, dtype=np.float32).copy()
        return d

    def _patterns(self, X, name="X"):
        X = X.contiguous()
        if X.dtype != self.cfg.io_dtype or not X.is_cuda:
            raise ValueError(f"{name} must be a {self.cfg.io_dtype} CUDA tensor")
        return X

    def predict(self, X, genes=None):
        """Model output on patterns X (n x F): z, or sigmoid(z) for classification."""
        torch = _torch()
        X = self._patterns(X)
        if X.dim() != 2 or X.shape[1] != self.cfg.n_features:
            raise ValueError("X must be n x F")
        if genes is not None:
            genes = genes.contiguous().to(torch.float32)
        out = torch.empty(X.shape[0], dtype=self.cfg.io_dtype, device=self.device)
        L.check(L.lib().game_predict(self._ctx, _ptr(genes), _ptr(X), X.shape[0], _ptr(out)),
                "game_predict")
        self._keep = (X, genes)
        return out

    def evaluate(self, X, t, genes=None) -> dict:
        """MSE, RMSE and (classification) confusion counts and rates on (X, t)."""
        torch = _torch()
        X, t = self._patterns(X), self._patterns(t, "t")
        if X.dim() != 2 or X.shape[1] != self.cfg.n_features or t.shape != (X.shape[0],):
            raise ValueError("X must be n x F and t must have n entries")
        if genes is not None:
            genes = genes.contiguous().to(torch.float32)
        m = L.GameMetrics()
        L.check(L.lib().game_evaluate(self._ctx, _ptr(genes), _ptr(X), _ptr(t), X.shape[0],
                                      C.byref(m)), "game_evaluate")
        return {k: getattr(m, k) for k, _ in L.GameMetrics._fields_}

    def save(self) -> bytes:
        """Checkpoint (game_save) as bytes."""
        n = C.c_size_t()
        L.check(L.lib().game_save(self._ctx, None, C.byref(n)), "game_save")
        buf = (C.c_ubyte * n.value)()
        L.check(L.lib().game_save(self._ctx, buf, C.byref(n)), "game_save")
        return bytes(buf)

    def load(self, blob: bytes):
        """Resume from a checkpoint taken with the same configuration (game_load)."""
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        L.check(L.lib().game_load(self._ctx, buf, len(blob)), "game_load")

    def time_fitness(self, reps: int = 20) -> float:
        """Mean duration (ms) of one fitness-kernel launch over the population."""
        ms = C.c_float()
        L.check(L.lib().game_time_fitness(self._ctx, int(reps), C.byref(ms)), "game_time_fitness")
        return ms.value

    def close(self):
        if getattr(self, "_ctx", None):
            if getattr(self, "_owned", True):
                L.lib().game_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent GA runs advanced together (game_batch_init ... game_batch_destroy).

    runs: list of (Config, X, t) with device tensors as for Game."""

    def __init__(self, runs, stream=None):
        torch = _torch()
        if not runs:
            raise ValueError("at least one run is required")
        self.cfgs = [r[0] for r in runs]
        self._X = [r[1].contiguous() for r in runs]
        self._t = [r[2].contiguous() for r in runs]
        for cfg, X, t in zip(self.cfgs, self._X, self._t):
            if X.shape != (cfg.n_patterns, cfg.n_features) or t.shape != (cfg.n_patterns,):
                raise ValueError("X must be N x F and t must have N entries")
            if X.dtype != cfg.io_dtype or t.dtype != cfg.io_dtype or not X.is_cuda or not t.is_cuda:
                raise ValueError(f"X and t must be {cfg.io_dtype} CUDA tensors")
        n = len(runs)
        self.n = n
        carr = (L.GameConfig * n)(*[c.to_c() for c in self.cfgs])
        self._carr = carr
        need = C.c_size_t()
        L.check(L.lib().game_batch_workspace_size(carr, n, C.byref(need)), "game_batch_workspace_size")
        self.device = self._X[0].device
        self.workspace = torch.empty(need.value + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) & ~255
        xs = (C.c_void_p * n)(*[x.data_ptr() for x in self._X])
        ts = (C.c_void_p * n)(*[t.data_ptr() for t in self._t])
        b = C.c_void_p()
        L.check(L.lib().game_batch_init(carr, n, xs, ts, ws, need.value, _stream_handle(stream),
                                        C.byref(b)), "game_batch_init")
        self._b = b

    def tiles(self):
        """(tile_p, row_groups) the batch uses, one entry per run."""
        tp = (C.c_int32 * self.n)()
        rg = (C.c_int32 * self.n)()
        L.check(L.lib().game_batch_tiles(self._b, tp, rg), "game_batch_tiles")
        return list(tp), list(rg)

    def context(self, i: int) -> Game:
        """Run i as a Game view (owned by the batch: closing it releases nothing)."""
        ctx = C.c_void_p()
        L.check(L.lib().game_batch_context(self._b, int(i), C.byref(ctx)), "game_batch_context")
        g = Game.__new__(Game)
        g.cfg = self.cfgs[i]
        g.dims = query(self.cfgs[i])
        g.device = self.device
        g._stream = None
        g._ctx = ctx
        g._owned = False
        return g

    def time_fitness(self, reps: int = 10) -> float:
        ms = C.c_float()
        L.check(L.lib().game_batch_time_fitness(self._b, int(reps), C.byref(ms)),
                "game_batch_time_fitness")
        return ms.value

    def run(self, latency: bool = False):
        """Per-run result dicts (as Game.run) and, with latency, an n x G array (us, -1 = none)."""
        n = self.n
        res = (L.GameResult * n)()
        genes = [(C.c_float * query(c).L)() for c in self.cfgs]
        for r, g in zip(res, genes):
            r.best_genes = C.cast(g, C.POINTER(C.c_float))
        G = max(c.max_generations for c in self.cfgs)
        lat = np.full(n * G, -1.0) if latency else None
        L.check(L.lib().game_batch_run(self._b, res,
                                       lat.ctypes.data_as(C.c_void_p) if latency else None),
                "game_batch_run")
        out = [dict(best_mse=r.best_mse, best_fitness=r.best_fitness, best_miscls=r.best_miscls,
                    generations=r.generations, stop_reason=L.STOP.get(r.stop_reason),
                    best_genes=np.frombuffer(g, dtype=np.float32).copy())
               for r, g in zip(res, genes)]
        return (out, lat.reshape(n, G)) if latency else out

    def close(self):
        if getattr(self, "_b", None):
            L.lib().game_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

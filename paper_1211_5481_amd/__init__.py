"""GAME fitness hot path for MI355X (gfx950): Python binding of libgame.so.

The genetic algorithm of Cavuoti et al. (arXiv:1211.5481): chromosomes hold
the coefficients of per-feature polynomial expansions, are scored by their
training error over all patterns, and evolve by elitism, tournament
selection, crossover and mutation.  All of it runs in hand-written HIP
kernels behind the C ABI in include/game.h; this package only marshals
arguments and borrows device memory and streams from PyTorch.
"""
from .game import Batch, Config, Game, build_basis, query, rescore_noalloc, workspace_size  # noqa: F401
from . import _lib  # noqa: F401

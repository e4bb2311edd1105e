"""CPU oracle for the GAME fitness hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 restatement of what the GPU path computes, written from
the paper (Cavuoti et al., "Genetic Algorithm Modeling with GPU Parallel
Computing Technology", arXiv:1211.5481) and from the published definitions it
relies on (Philox4x32-10 of Salmon et al., SC'11; textbook orthogonal
polynomials).  Only the tests, the smoke check of ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_1211_5481_amd``) never does, and the oracle never imports the product
path: the two share no code, constants or tables.

Modules
-------
model    -- basis functions (closed forms), per-feature polynomial output
            (eq. 1-2, 6), squared error (eq. 3), MSE, fitness = 1 - error (Sec. 3)
philox   -- Philox4x32-10 counter-based generator (Salmon et al., SC'11)
ga       -- the genetic operators: random init in [-1, 1), elitism,
            tournament selection, one-point crossover, Gaussian mutation
            (Sec. 3 operator list, Sec. 5 settings), on float32 genes
mlp      -- float64 forward/backward/Adam of the fitness surrogate MLP
rank     -- Spearman rank correlation with average ranks for ties

Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (hand-expanded values, library routines, closed forms,
invariants); see the tests named ``test_oracle_*``.
"""

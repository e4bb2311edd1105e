/*
 * game.h -- C ABI of libgame.so, the MI355X (gfx950) fitness hot path of GAME,
 * the genetic algorithm of Cavuoti et al., "Genetic Algorithm Modeling with GPU
 * Parallel Computing Technology" (arXiv:1211.5481).
 *
 * What the library computes (Sec. 3 of the paper):
 *   - every pattern (f_1..f_F, t) has each feature expanded in a polynomial
 *     sequence of degree D (eq. 1; the trigonometric "polytrigo" sequence of
 *     eq. 6 has cos and sin groups, B = 2), giving the basis row
 *     Phi[n, i*K + k] = phi_{k+1}(x[n, i]),  K = B*D,  M = F*K
 *     (with `shared`, the paper's literal model of one coefficient per basis
 *     function for all features: Phi[n, k] = sum_i phi_{k+1}(x[n, i]), M = K);
 *   - a chromosome holds one coefficient (gene) per basis column, plus an
 *     optional constant a_0 stored last (L = M or M + 1 genes), and its output
 *     on pattern n is z = sum_m Phi[n, m] G[m] (+ a_0)  (eq. 2);
 *   - the error of a pattern is (t - z)^2 for regression and
 *     (l - sigmoid(z))^2 for classification, l = [t >= 0.5] the class label
 *     (eq. 3 with the logistic output); a chromosome's error is the mean over
 *     all patterns (MSE) and its fitness is 1 - MSE; a pattern counts as
 *     misclassified when [z >= 0] differs from l;
 *   - a generation applies elitism, tournament, roulette or ranking
 *     selection, one-point crossover, Gaussian mutation and optional random
 *     immigrants, with genes kept in [-1, 1] (Sec. 3 operator list; Sec. 4;
 *     Sec. 5 rates), every random draw coming from a Philox4x32-10 counter
 *     (Salmon et al., SC'11) keyed by the seed;
 *   - training repeats evaluation and evolution until a generation count or
 *     an error threshold is reached (Sec. 4).
 *
 * Conventions for every entry point:
 *   - Every call returns a game_status; nothing throws or aborts across the ABI.
 *   - The library never allocates device memory.  The caller owns the inputs,
 *     the workspace, every output buffer and the stream; the workspace must
 *     stay allocated and untouched while the context lives.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked "async" only enqueue work on that stream.
 *   - Arguments are validated before any launch; an invalid argument returns
 *     GAME_E_INVALID and changes nothing.  A HIP error returns GAME_E_DEVICE
 *     and poisons the context: later calls on it return GAME_E_STATE.
 *   - game_last_error() returns a message describing the last failure of the
 *     calling thread.
 */
#ifndef GAME_H
#define GAME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct game_ctx game_ctx; /* opaque; created by game_init, freed by game_destroy */

typedef enum {
  GAME_OK = 0,
  GAME_E_INVALID = 1,     /* bad argument or configuration                        */
  GAME_E_OOM = 2,         /* workspace too small for the configuration            */
  GAME_E_DEVICE = 3,      /* a HIP call failed; the context is poisoned          */
  GAME_E_STATE = 4,       /* context poisoned, or call out of order               */
  GAME_E_UNSUPPORTED = 5  /* valid but not implemented combination                */
} game_status;

/* Basis families.  B = 1 except TRIG (B = 2: cos(1x)..cos(Dx), sin(1x)..sin(Dx)). */
typedef enum {
  GAME_BASIS_POWER = 0,     /* x^k, k = 1..D                                      */
  GAME_BASIS_CHEBYSHEV = 1, /* T_k(x), k = 1..D                                   */
  GAME_BASIS_LEGENDRE = 2,  /* P_k(x), k = 1..D                                   */
  GAME_BASIS_TRIG = 3       /* eq. 6 polytrigo                                    */
} game_basis;

typedef enum { GAME_REGRESSION = 0, GAME_CLASSIFICATION = 1 } game_task;

/* Storage/compute type of Phi and the gene tile.  F64: x and t are double and the
 * contraction runs in double.  F32: x, t float, FP32 MFMA.  BF16/F16: x, t float,
 * Phi and genes rounded (nearest even) to 16 bits, FP32 accumulation. */
typedef enum { GAME_F64 = 0, GAME_F32 = 1, GAME_BF16 = 2, GAME_F16 = 3 } game_dtype;

/*
 * Parent selection (Sec. 3 lists roulette and ranking; the experiments of
 * Sec. 5 use them):
 *   TOURNAMENT: best of tournament_k uniform draws (with replacement);
 *   ROULETTE:   fitness-proportionate wheel with weights
 *               floor((f - f_min) / (f_max - f_min) * 2^32) (NaN weighs 0);
 *   RANKING:    rank-based wheel, rank q (0 = best) weighs P - q (P <= 8192).
 * Wheel draws are 64-bit Philox draws scaled to the wheel's integer total.
 */
typedef enum { GAME_SEL_TOURNAMENT = 0, GAME_SEL_ROULETTE = 1, GAME_SEL_RANKING = 2 } game_selection;

/* Prescreen of the offspring form.  NONE: every child is evaluated exactly.
 * MLP: a 2-hidden-layer GELU perceptron trained online (Adam) on the
 * (chromosome, standardised log MSE) pairs evaluated so far ranks the
 * children and only the best prescreen_frac are evaluated exactly.
 * RANDOM: the same number chosen at random (control). */
typedef enum { GAME_SURROGATE_NONE = 0, GAME_SURROGATE_MLP = 1, GAME_SURROGATE_RANDOM = 2 } game_surrogate;

typedef enum {
  GAME_STOP_NONE = 0,       /* still running / never run                          */
  GAME_STOP_THRESHOLD = 1,  /* best MSE <= mse_threshold                          */
  GAME_STOP_MAX_GEN = 2     /* max_generations generations evaluated              */
} game_stop_reason;

typedef struct {
  uint32_t struct_size;     /* must equal sizeof(game_config)                     */
  int32_t  basis;           /* game_basis                                         */
  int64_t  n_patterns;      /* N >= 1                                             */
  int32_t  n_features;      /* F >= 1                                             */
  int32_t  degree;          /* D >= 1                                             */
  int32_t  task;            /* game_task                                          */
  int32_t  dtype;           /* game_dtype                                         */
  int32_t  bias;            /* 0 | 1: gene a_0 stored at index M                  */
  int32_t  pop_size;        /* P; 0 -> B*F + 1 (eq. 4)                            */
  int32_t  n_offspring;     /* 0 -> P - elitism (generational replacement);       */
                            /* other values select the offspring form: each       */
                            /* generation breeds n_offspring children (<= 8192),  */
                            /* evaluates some exactly and keeps the E elites plus */
                            /* the best P - E evaluated children                  */
  int32_t  elitism;         /* E in [0, min(P, 64)] (the paper's runs use 2)      */
  int32_t  selection;       /* game_selection                                     */
  int32_t  tournament_k;    /* k in [1, 16]                                       */
  int32_t  n_immigrants;    /* the last n_immigrants children of each generation  */
                            /* are random chromosomes instead (the paper's random */
                            /* chromosomes that replace older individuals, Sec. 4)*/
  int32_t  shared;          /* 0: one coefficient per feature and basis function  */
                            /* (M = F*B*D genes); 1: the paper's literal model,   */
                            /* one coefficient per basis function shared by all   */
                            /* features (eq. 2 and eq. 7; M = B*D genes, eq. 5),  */
                            /* so Phi[n, k] = sum_i phi_{k+1}(x[n, i])            */
  int32_t  max_generations; /* >= 1, used by game_run                             */
  int32_t  rescore_top;     /* 0..8: every generation re-scores the top-k ranked   */
                            /* chromosomes in float32 and tracks the best and     */
                            /* tests the stop rule on those float32 MSEs (meant   */
                            /* for BF16/F16; not available with F64)              */
  int32_t  tile_p;          /* chromosomes per fitness workgroup tile: 0 = chosen */
                            /* by the library; 32 | 64 | 128 select the LDS-staged */
                            /* kernel with that tile (F32/BF16/F16; the tile must */
                            /* fit the kernel's 96 KiB of LDS); F64 uses 64       */
  int32_t  row_groups;      /* 0 = chosen by the library; R > 0 splits the rows  */
                            /* into R ranges whose partial sums are added in      */
                            /* order (this fixes the summation order, so equal    */
                            /* tile_p and row_groups give bit-identical sums)     */
  int32_t  surrogate;       /* offspring form prescreen: game_surrogate           */
  int32_t  surrogate_hidden;/* hidden width of both MLP layers, 16..1024          */
  int32_t  surrogate_buffer;/* replay ring capacity (pairs), >= surrogate_batch    */
  int32_t  surrogate_steps; /* Adam steps per generation                          */
  int32_t  surrogate_batch; /* minibatch rows                                     */
  int32_t  audit;           /* MLP prescreen: offspring also evaluated exactly,   */
                            /* drawn at random each generation, to measure the    */
                            /* surrogate's rank error (0..4096, capped at         */
                            /* n_offspring; unused by the other modes)            */
  double   prescreen_frac;  /* fraction of the offspring evaluated exactly        */
  double   surrogate_lr;    /* Adam learning rate                                 */
  double   surrogate_recent;/* fraction of each minibatch drawn from the latest   */
                            /* generation's exact evaluations, [0, 1]; the rest   */
                            /* is drawn uniformly from the whole replay buffer    */
  double   p_crossover;     /* [0, 1] per child pair                              */
  double   p_mutation;      /* [0, 1] per gene                                    */
  double   mutation_sigma;  /* >= 0, standard deviation of the Gaussian step      */
  double   mse_threshold;   /* game_run stops once best MSE <= this               */
  uint64_t seed;            /* Philox key                                         */
} game_config;

/* Sizes the library derives from a configuration. */
typedef struct {
  int32_t  K;               /* basis columns per feature, B*D                     */
  int32_t  M;               /* basis columns, F*K                                 */
  int32_t  L;               /* genes per chromosome, M + bias                     */
  int32_t  M_pad;           /* row stride of Phi and of the gene tile (elements)  */
  int32_t  P;               /* population size after defaults                     */
  int32_t  n_offspring;     /* offspring per generation after defaults            */
  int64_t  N_pad;           /* rows of Phi in the workspace (N rounded up)        */
  size_t   workspace_bytes; /* bytes game_init needs                              */
} game_dims;

/* Result of game_run. */
typedef struct {
  double   best_mse;        /* MSE of the best chromosome seen                    */
  double   best_fitness;    /* 1 - best_mse                                       */
  double   best_miscls;     /* its misclassification rate (0 for regression)      */
  int32_t  generations;     /* generations evaluated by this call                 */
  int32_t  stop_reason;     /* game_stop_reason                                   */
  float*   best_genes;      /* caller-provided HOST buffer of L floats, or NULL   */
} game_result;

/* Snapshot of the device-side run state (blocking copy). */
typedef struct {
  int32_t generation;       /* generations completed since game_init              */
  int32_t stopped;          /* 1 once a game_run stop condition held              */
  int32_t best_index;       /* index of the best chromosome of the last ranking   */
  int32_t stop_reason;
  double  best_mse, best_fitness, best_miscls;   /* best seen since game_init     */
} game_state;

/* Fill *cfg with the defaults: Chebyshev D=4, F32, regression, E=2, k=3,
 * p_crossover 0.9, p_mutation 0.05, sigma 0.1, 100 generations, threshold 0.
 * n_patterns / n_features must still be set by the caller. */
void game_config_default(game_config* cfg);

/* Validate cfg and report derived sizes (no device work). */
game_status game_query(const game_config* cfg, game_dims* dims);

/* Bytes of device workspace game_init needs for cfg. */
game_status game_workspace_size(const game_config* cfg, size_t* bytes);

/*
 * Basis expansion alone (eq. 1 and 6), async.
 *   X_dev:   N x F row-major, double if dtype == F64 else float (device).
 *   phi_dev: N x ld row-major in the dtype's storage type (device, caller-owned);
 *            ld >= M; columns M..ld-1 are written as zero.
 * Returns GAME_E_INVALID for a bad cfg or ld < M.
 */
game_status game_build_basis(const game_config* cfg, const void* X_dev, void* phi_dev,
                             int64_t ld, void* stream);

/*
 * Create a context: validates cfg, carves the workspace, builds Phi once for
 * the whole training (the sin/cos precompute of Sec. 4), copies t, and draws
 * the initial population (genes uniform in [-1, 1), Sec. 3).  Async; X and t
 * may be freed once the stream has passed this call.
 *   X_dev: N x F row-major (double if F64 else float); t_dev: N targets of the
 *   same type (classification targets are 0 or 1).
 *   workspace_dev: >= game_workspace_size bytes, 256-byte aligned.
 */
game_status game_init(const game_config* cfg, const void* X_dev, const void* t_dev,
                      void* workspace_dev, size_t ws_bytes, void* stream, game_ctx** out);

/*
 * Fitness of a set of chromosomes over all N patterns, async (eq. 2, 3, MSE,
 * fitness = 1 - MSE).
 *   genes_dev: P x L row-major float chromosomes (device), or NULL for the
 *              current population (then P must equal the population size).
 *   P:         1 <= P <= max(population size, n_offspring) in the generational
 *              form; <= max(population size, children evaluated exactly per
 *              generation) in the offspring form.
 *   mse_dev, miscls_dev, fitness_dev: P doubles each (device) or NULL.
 * The results for the current population are also kept for game_step(NULL).
 */
game_status game_eval_fitness(game_ctx* ctx, const float* genes_dev, int32_t P,
                              double* mse_dev, double* miscls_dev, double* fitness_dev);

/*
 * One generation of the genetic operators on the current population, async
 * (the operators Sec. 3 lists, applied at the rates and elitism of the
 * experiments of Sec. 5; genes stay in the [-1, 1] range of Sec. 3):
 * elitism (the E best, fitness descending, ties to the lower index, NaN worst,
 * copied unchanged), then P - E children from the configured selection
 * (size-k tournaments, roulette or ranking), one-point crossover and per-gene
 * Gaussian mutation clamped to [-1, 1] (IEEE maxNum/minNum: a NaN sum becomes
 * -1), the last n_immigrants children replaced by random chromosomes (Sec. 4).
 *   fitness_dev: P doubles of the current population (device), or NULL to use
 *                the last game_eval_fitness(NULL) result (GAME_E_STATE if none).
 * Increments the generation counter that keys the random draws.
 * Offspring form (n_offspring != P - elitism or a surrogate): fitness_dev must
 * be NULL (GAME_E_UNSUPPORTED otherwise); one call breeds n_offspring children
 * from the current population, prescreens them (surrogate MLP scores, or a
 * uniformly random subset), evaluates the chosen ones exactly and keeps the E
 * elites plus the best P - E of them; with the MLP it also stores the exact
 * results in the replay buffer and trains on it.
 */
game_status game_step(game_ctx* ctx, const double* fitness_dev);

/*
 * n generations of (evaluate current population, rank, evolve), async,
 * replayed from captured HIP graphs (n / 8 launches of an 8-generation graph,
 * then one graph of the n mod 8 remaining generations; graphs are captured on
 * first use, see game_advance_prepare); no stop test.
 */
game_status game_advance(game_ctx* ctx, int32_t n_generations);

/*
 * Capture, without running anything, the HIP graphs game_advance(ctx, n)
 * replays (a graph of 8 generations when n >= 8 and one of the n mod 8
 * remaining generations), so that a later game_advance(ctx, n) only launches
 * them: a caller with a latency-critical loop pays the capture beforehand.
 * Blocking (host-side capture; may wait for the context's stream when it
 * replaces a remainder graph of another length).  Only the last remainder
 * length is kept.
 */
game_status game_advance_prepare(game_ctx* ctx, int32_t n_generations);

/*
 * Train until best MSE <= mse_threshold or max_generations generations have
 * been evaluated (Sec. 4).  Blocking.  Evaluation happens first in every
 * generation; no evolution follows the generation that stops the run.
 */
game_status game_run(game_ctx* ctx, game_result* out);

/*
 * Float32 re-score (the precision forms' check of their elites): MSE and
 * misclassification rate of n <= 8 chromosomes with float32 basis values
 * (recomputed from the patterns) and float32 arithmetic, async.
 *   genes_dev: n x L floats (device), or NULL for the current population's n
 *              best by the last ranking (GAME_E_STATE if none).
 *   mse_dev, miscls_dev: n doubles (device) or NULL.
 * GAME_E_UNSUPPORTED for F64 contexts; n * L must be <= 16384.
 */
game_status game_rescore(game_ctx* ctx, const float* genes_dev, int32_t n, double* mse_dev,
                         double* miscls_dev);

/*
 * For callers that cannot allocate device memory and hold no context: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The float32 re-score of game_rescore computed straight from the
 * patterns, async on `stream`; it allocates nothing (no hipMalloc, no
 * workspace) and needs no game_init.
 *   cfg:        a configuration as for game_init (validated as by game_query);
 *               F32, BF16 or F16 (F64: GAME_E_UNSUPPORTED).  The basis, degree,
 *               bias, shared and task fields define the model.
 *   X_dev:      N x F float patterns, row-major (device); t_dev: N float targets.
 *   genes_dev:  n x L float chromosomes (device), required.
 *   n:          1 <= n <= 8 (GAME_E_INVALID beyond: the scratch below holds the
 *               partial sums of at most 8 chromosomes), and n * L <= 16384.
 *   mse_dev, miscls_dev: n doubles each (device) or NULL.
 * Scratch: one fixed array of 131 328 bytes inside the library per GPU (1024
 * workgroup partials of 16 doubles and an arrival counter), held until the
 * process ends.  Every call on a GPU shares it, so calls that overlap on one
 * GPU (several streams or host threads) race: the caller serialises them.
 * The first call on a device also enqueues a one-thread kernel that clears
 * the counter.  Results equal game_rescore's bit for bit on a context built
 * from the same cfg, X and t.
 */
game_status game_rescore_noalloc(const game_config* cfg, const void* X_dev, const void* t_dev,
                                 const float* genes_dev, int32_t n, double* mse_dev,
                                 double* miscls_dev, void* stream);

/*
 * Offspring form, per generation, blocking: the Spearman rank correlation of
 * the surrogate's scores with the exact log MSE on the audit sample
 * (rho_audit) and on the children evaluated exactly (rho_selected), and the
 * last training loss.  Fills up to n_max records of the most recent
 * generations (oldest first, at most 4096 kept) into the host array
 * log_host (4 floats each: rho_audit, rho_selected, loss, 1) and returns the
 * number written in *n_out.
 */
game_status game_surrogate_log(game_ctx* ctx, float* log_host, int32_t n_max, int32_t* n_out);

/*
 * The surrogate's replay buffer (MLP prescreen contexts), for inspection:
 * genes_dev (surrogate_buffer x L floats) and y_dev (surrogate_buffer floats,
 * the stored natural-log MSEs) are device copies, async, either may be NULL;
 * count_head_host (2 ints: pairs stored, next slot) and mu_sigma_host (2
 * floats: mean and standard deviation the training targets are standardised
 * with) are host copies, and when either is non-NULL the call blocks.
 * Generations append their exact evaluations at the next slots of the ring
 * in evaluation order (prescreen choices, then the audit sample).
 */
game_status game_surrogate_buffer(game_ctx* ctx, float* genes_dev, float* y_dev,
                                  int32_t* count_head_host, float* mu_sigma_host);

/*
 * The surrogate MLP itself (MLP prescreen contexts), async; for checks
 * against a reference implementation.  Parameters are one float32 array in
 * the order W1 (H x L, row-major), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1).
 *   game_mlp_params: dir 0 copies the parameters out to params_dev, dir 1 in.
 *   game_mlp_forward: y_dev[i] = score of row i of X_dev (n x L),
 *     1 <= n <= max(n_offspring, surrogate_batch, P).
 *   game_mlp_grads: gradients (same layout) of the mean squared error of the
 *     scores against target_dev over the n rows (n <= surrogate_batch), and
 *     the loss in *loss_dev (device float) when non-NULL.
 *   game_mlp_adam: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the
 *     given gradients and the configured learning rate.
 */
game_status game_mlp_params(game_ctx* ctx, float* params_dev, int32_t dir);
game_status game_mlp_forward(game_ctx* ctx, const float* X_dev, int32_t n, float* y_dev);
game_status game_mlp_grads(game_ctx* ctx, const float* X_dev, const float* target_dev, int32_t n,
                           float* grads_dev, float* loss_dev);
game_status game_mlp_adam(game_ctx* ctx, const float* grads_dev);

/* Copy the population out / in: P x L floats, device pointers, async. */
game_status game_get_population(game_ctx* ctx, float* genes_dev);
game_status game_set_population(game_ctx* ctx, const float* genes_dev);

/*
 * Test and validation use (Sec. 4: the trained model applied to patterns).
 * genes_dev: one chromosome (L floats, device), or NULL for the best so far
 * (GAME_E_STATE before any population evaluation).  X_dev: n x F patterns,
 * t_dev: n targets (double for F64 contexts, else float; the basis is that of
 * the context).  Every pattern is computed in double.
 *   game_predict: out_dev[i] = z_i (regression) or sigmoid(z_i)
 *     (classification), n values of the input type; async.
 *   game_evaluate: blocking; fills *out: MSE (eq. 3) and RMSE over the n
 *     patterns and, for classification, the confusion counts with class 1
 *     positive (predicted 1 iff z >= 0, label t >= 0.5) and the rates the
 *     paper reports (Sec. 5): accuracy = (TP + TN) / n, completeness =
 *     TP / (TP + FN), contamination = FP / (TP + FP); rates are NaN when
 *     undefined (regression, or a zero denominator).
 */
typedef struct {
  int64_t n;
  double  mse, rmse, accuracy, completeness, contamination;
  int64_t tp, fp, tn, fn;
} game_metrics;
game_status game_predict(game_ctx* ctx, const float* genes_dev, const void* X_dev, int64_t n,
                         void* out_dev);
game_status game_evaluate(game_ctx* ctx, const float* genes_dev, const void* X_dev,
                          const void* t_dev, int64_t n, game_metrics* out_host);

/*
 * Checkpoint and resume.  game_save writes everything a context carries from
 * one generation to the next into a host buffer: the run state, both
 * population buffers, the last fitness values, elites and best genes, and in
 * the offspring form the surrogate's parameters, Adam moments and step, its
 * replay ring and statistics and the log.  The random draws are counter
 * based, so a context that loads the checkpoint continues bit for bit as the
 * saving one would.  Blocking.
 *   game_save: host_buf NULL -> *bytes = size needed; otherwise *bytes (in)
 *              is the buffer size (GAME_E_INVALID if too small) and (out)
 *              the size written.
 *   game_load: into a context created with the same configuration (only
 *              max_generations and mse_threshold may differ) and the same
 *              patterns; GAME_E_INVALID for a foreign or mismatched buffer.
 */
game_status game_save(game_ctx* ctx, void* host_buf, size_t* bytes);
game_status game_load(game_ctx* ctx, const void* host_buf, size_t bytes);

/* Blocking snapshot of the run state; best genes optional (host, L floats). */
game_status game_get_state(game_ctx* ctx, game_state* out, float* best_genes_host);

/*
 * Measurement: launch only the fitness kernel for the current population
 * `reps` times on the context's stream, bracketed by two HIP events, and
 * report the mean duration of one launch in *ms.  Blocking.  Each launch is
 * the one a generation runs (contraction, reduction, ranking and best
 * tracking), so the state is updated as by an evaluation of the current
 * population (game_eval_fitness with genes NULL).
 * The population's gene tile is packed once before the timed launches.
 */
game_status game_time_fitness(game_ctx* ctx, int32_t reps, float* ms);

/* Release the context (host memory only; the workspace stays the caller's). */
void game_destroy(game_ctx* ctx);

/*
 * Batched form: many independent GA runs (each one context with its own
 * configuration, patterns, population and stop rule) advanced together by
 * one persistent scheduler launch per up to 128 generations.  Each run moves
 * through its own phases (fitness items of chromosome tile x row range, the
 * wheel or rank order for roulette / ranking selection, the breed) as soon
 * as its previous phase ends, so runs progress independently: a small run's
 * generation takes about its own work, not the largest run's.  Workgroups
 * take open items from the runs in order of increasing generation cost.
 * Requirements: 1..4096 runs, one dtype for all (F32, BF16 or F16), the
 * generational GA (no offspring form, no re-score), gene counts whose tiles
 * fit the LDS-staged kernel.  Each run computes exactly what game_run would
 * on a context created with the same configuration and the tile_p /
 * row_groups the batch uses (game_batch_tiles).  A workgroup that finds no
 * open item for far longer than any phase takes (20x one generation of every
 * run at 50 TFLOP/s, at least 2 s; the environment variable
 * GAME_FLOW_IDLE_US, read when the batch's tiles are set, overrides it in
 * microseconds) ends the launch with GAME_E_DEVICE, naming the stuck run's
 * phase state, and poisons the batch.
 */
typedef struct game_batch game_batch;

/* Workspace bytes for the batch (the runs' workspaces plus the batch's tables). */
game_status game_batch_workspace_size(const game_config* cfgs, int32_t n_runs, size_t* bytes);

/*
 * Create the runs (as game_init: basis, targets, initial population) in one
 * workspace, then pick each run's tile width and row ranges: configurations
 * with tile_p and row_groups both set keep them when every run sets them;
 * otherwise the tuner times candidate assignments with evaluation-only
 * scheduler launches on the device and keeps the fastest: a sweep of LDS
 * budget x item size (each run the widest tile within the budget), then one
 * tile width narrower per class of runs (task x gene count), kept where
 * faster.  Each run's choice is cached for the process by its shape (dtype,
 * task, padded gene count, population, log2 patterns); a batch whose runs
 * all have a cached choice starts from those without a sweep.  Blocking.
 *   X_devs[i], t_devs[i]: run i's patterns and targets, as for game_init.
 */
game_status game_batch_init(const game_config* cfgs, int32_t n_runs, const void* const* X_devs,
                            const void* const* t_devs, void* workspace_dev, size_t ws_bytes,
                            void* stream, game_batch** out);

/* Tile width and row ranges each run uses (host arrays of n_runs, either may be NULL). */
game_status game_batch_tiles(game_batch* batch, int32_t* tile_p_host, int32_t* row_groups_host);

/* Run i's context, for inspection (population, state, fitness); owned by the batch. */
game_status game_batch_context(game_batch* batch, int32_t i, game_ctx** out);

/* Mean duration (ms) of one scheduler launch that evaluates every run's current
 * population once (fitness phase only, each run's ranking and best tracking
 * included); blocking. */
game_status game_batch_time_fitness(game_batch* batch, int32_t reps, float* ms);

/*
 * Run every run until its own stop rule holds (as game_run), blocking.
 *   results: n_runs records (best_genes may be NULL or L_i host floats).
 *   latency_us: NULL, or n_runs x G doubles (G = largest max_generations):
 *     entry [i][g] = microseconds from the opening of run i's g-th
 *     generation of this call (its fitness phase) to the end of its breed,
 *     -1 where run i did not breed a g-th generation.
 */
game_status game_batch_run(game_batch* batch, game_result* results, double* latency_us);

void game_batch_destroy(game_batch* batch);

/* game_batch_init + game_batch_run + game_batch_destroy. */
game_status game_run_batched(const game_config* cfgs, int32_t n_runs, const void* const* X_devs,
                             const void* const* t_devs, void* workspace_dev, size_t ws_bytes,
                             void* stream, game_result* results, double* latency_us);

const char* game_status_str(game_status s);
const char* game_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GAME_H */

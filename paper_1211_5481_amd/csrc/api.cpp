// C ABI of libgame (declared in include/game.h): validation, workspace
// carve-up, the per-generation launch sequence and its HIP-graph replay.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "game.h"
#include "game_internal.hpp"

namespace game {
}

using namespace game;

namespace {

thread_local char g_err[512] = "";

game_status fail(game_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

constexpr int kChunk = 8;  // generations per replayed graph in game_run / game_advance

}  // namespace

struct game_ctx {
  game_config cfg;
  Plan plan;
  hipStream_t stream = nullptr;      // caller's stream
  hipStream_t cap = nullptr;         // private stream used only for graph capture
  hipGraphExec_t execR = nullptr, execC = nullptr;
  hipGraph_t graphR = nullptr, graphC = nullptr;
  int nR = 0;                        // generations in graphR (game_advance's remainder)
  unsigned char* ws = nullptr;
  void *phi, *tvec, *tile, *biasv;
  float *pop0, *pop1, *best;  // generation g lives in pop[g & 1]
  double *psse, *mse, *miscls, *fit;
  uint32_t *pmiss, *counters;
  float* xf;      // float32 patterns (16-bit and float32 forms)
  double* rpart;  // re-score partials
  int* elite;
  uint64_t* wheel;  // selection wheel or ranking of the current population
  double* mpart;    // metric partials, then the 5 result values
  bool evaluated = false;  // a population evaluation has been enqueued (best genes exist)
  DevState* state;
  uint64_t thr_c, thr_m;
  bool poisoned = false;
  bool have_eval = false;   // elites/fitness of the current population are known
  bool tile_fresh = false;  // the gene tile holds the current population
  bool sur_warm = false;    // offspring form: initial population stored (and learned)
  // offspring form buffers
  float *O = nullptr, *evg = nullptr, *yhat = nullptr, *rho = nullptr, *loss = nullptr;
  uint64_t* keys = nullptr;
  int* rank_ws = nullptr;
  int *sel = nullptr, *aud = nullptr, *surv = nullptr;
  double *emse = nullptr, *emis = nullptr, *efit = nullptr, *snap = nullptr;
  float *prm = nullptr, *am = nullptr, *av = nullptr;
  int32_t* step = nullptr;
  float *WT = nullptr, *mscr = nullptr;
  float *buf = nullptr, *bufy = nullptr, *log = nullptr;
  SurState* sst = nullptr;
};

namespace game {

game_status make_plan(const game_config* c, Plan* p, char* err, size_t errlen) {
  auto bad = [&](const char* msg) {
    std::snprintf(err, errlen, "%s", msg);
    return GAME_E_INVALID;
  };
  if (!c) return bad("config is NULL");
  if (c->struct_size != sizeof(game_config)) return bad("config struct_size mismatch (ABI version)");
  if (c->basis < GAME_BASIS_POWER || c->basis > GAME_BASIS_TRIG) return bad("unknown basis");
  if (c->task != GAME_REGRESSION && c->task != GAME_CLASSIFICATION) return bad("unknown task");
  if (c->dtype < GAME_F64 || c->dtype > GAME_F16) return bad("unknown dtype");
  if (c->n_patterns < 1) return bad("n_patterns must be >= 1");
  if (c->n_patterns > (int64_t(1) << 40)) return bad("n_patterns too large");
  if (c->n_features < 1 || c->degree < 1) return bad("n_features and degree must be >= 1");
  if (c->bias != 0 && c->bias != 1) return bad("bias must be 0 or 1");
  if (c->selection < GAME_SEL_TOURNAMENT || c->selection > GAME_SEL_RANKING) return bad("unknown selection");
  if (c->shared != 0 && c->shared != 1) return bad("shared must be 0 or 1");
  if (c->tournament_k < 1 || c->tournament_k > kMaxTournament) return bad("tournament_k must be in [1, 16]");
  auto prob_ok = [](double v) { return std::isfinite(v) && v >= 0.0 && v <= 1.0; };
  if (!prob_ok(c->p_crossover) || !prob_ok(c->p_mutation)) return bad("probabilities must be in [0, 1]");
  if (!std::isfinite(c->mutation_sigma) || c->mutation_sigma < 0) return bad("mutation_sigma must be finite and >= 0");
  if (c->max_generations < 1) return bad("max_generations must be >= 1");
  if (std::isnan(c->mse_threshold)) return bad("mse_threshold is NaN");
  if (c->rescore_top < 0 || c->rescore_top > kMaxRescore) return bad("rescore_top must be in [0, 8]");
  const int64_t B = c->basis == GAME_BASIS_TRIG ? 2 : 1;
  const int64_t K = B * c->degree;
  const int64_t M = c->shared ? K : (int64_t)c->n_features * K;
  const int64_t L = M + c->bias;
  if (L > kMaxGenes) return bad("too many genes (M + bias must be <= 4096)");
  int64_t P = c->pop_size;
  if (P == 0) P = B * c->n_features + 1;  // eq. (4)
  if (P < 1 || P > (1 << 24)) return bad("pop_size out of range");
  if (c->elitism < 0 || c->elitism > P || c->elitism > kMaxElite) return bad("elitism must be in [0, min(P, 64)]");
  int64_t n_off = c->n_offspring == 0 ? P - c->elitism : c->n_offspring;
  if (c->rescore_top > 0 && c->dtype == GAME_F64) {
    std::snprintf(err, errlen, "rescore_top is not available with F64");
    return GAME_E_UNSUPPORTED;
  }
  if (c->rescore_top > P) return bad("rescore_top must not exceed the population size");
  if (c->selection == GAME_SEL_RANKING && P > 8192) return bad("ranking selection needs pop_size <= 8192");
  if (c->n_immigrants < 0 || c->n_immigrants > n_off) return bad("n_immigrants must be in [0, n_offspring]");
  if (c->surrogate < GAME_SURROGATE_NONE || c->surrogate > GAME_SURROGATE_RANDOM) return bad("unknown surrogate mode");
  const bool offspring = c->surrogate != GAME_SURROGATE_NONE || n_off != P - c->elitism;
  p->offspring = offspring;
  p->n_off = (int)n_off;
  p->sur = c->surrogate;
  if (offspring) {
    if (n_off < 2 || n_off > 8192) return bad("n_offspring must be in [2, 8192] in the offspring form");
    if (c->rescore_top > 0) {
      std::snprintf(err, errlen, "rescore_top is not available in the offspring form");
      return GAME_E_UNSUPPORTED;
    }
    if (c->surrogate != GAME_SURROGATE_NONE) {
      if (!(c->prescreen_frac > 0.0 && c->prescreen_frac <= 1.0)) return bad("prescreen_frac must be in (0, 1]");
      p->k_sel = (int)std::llround(c->prescreen_frac * (double)n_off);
      if (p->k_sel < 1) p->k_sel = 1;
      if (p->k_sel > 4096) return bad("prescreen_frac * n_offspring must be <= 4096");
      if (c->audit < 0 || c->audit > 4096) return bad("audit must be in [0, 4096]");
      // the audit sample measures the MLP's ranking; it is capped at n_offspring
      p->audit = c->surrogate == GAME_SURROGATE_MLP ? (int)std::min<int64_t>(c->audit, n_off) : 0;
    } else {
      p->k_sel = (int)n_off;
      p->audit = 0;
    }
    if (p->k_sel < P - c->elitism) return bad("the offspring evaluated exactly must cover P - elitism");
    p->P_eval = p->k_sel + p->audit;
    if (c->surrogate == GAME_SURROGATE_MLP) {
      if (c->surrogate_hidden < 16 || c->surrogate_hidden > 1024) return bad("surrogate_hidden must be in [16, 1024]");
      if (c->surrogate_batch < 1 || c->surrogate_batch > 8192) return bad("surrogate_batch must be in [1, 8192]");
      if (c->surrogate_buffer < c->surrogate_batch) return bad("surrogate_buffer must be >= surrogate_batch");
      if (c->surrogate_buffer > (1 << 24)) return bad("surrogate_buffer too large");
      if (c->surrogate_buffer < std::max<int64_t>(P, p->k_sel + p->audit))
        return bad("surrogate_buffer must hold one generation's exact evaluations (and the population)");
      if (c->surrogate_steps < 0 || c->surrogate_steps > 1024) return bad("surrogate_steps must be in [0, 1024]");
      if (!(std::isfinite(c->surrogate_lr) && c->surrogate_lr > 0.0)) return bad("surrogate_lr must be > 0");
      if (!(c->surrogate_recent >= 0.0 && c->surrogate_recent <= 1.0)) return bad("surrogate_recent must be in [0, 1]");
      p->n_recent = (int)std::floor(c->surrogate_recent * c->surrogate_batch + 0.5);
      p->H = c->surrogate_hidden;
      p->cap = c->surrogate_buffer;
      p->steps = c->surrogate_steps;
      p->batch = c->surrogate_batch;
    }
  }
  p->K = (int)K;
  p->M = (int)M;
  p->L = (int)L;
  p->M_pad = (int)round_up(M, (c->dtype == GAME_BF16 || c->dtype == GAME_F16) ? 32 : 8);
  p->P = (int)P;
  p->n_off = (int)n_off;
  p->E = c->elitism;
  p->k = c->tournament_k;
  p->P_max = (int)(offspring ? std::max<int64_t>(P, p->P_eval) : std::max<int64_t>(P, n_off));
  // fitness tile: tile_n patterns x tile_p chromosomes; buffers are sized for
  // every tile width, so a context can switch tile_p without a new workspace
  if (c->row_groups < 0) return bad("row_groups must be >= 0");
  p->row_groups = c->row_groups;
  if (c->dtype == GAME_F64) {
    if (c->tile_p != 0 && c->tile_p != 64) return bad("tile_p must be 0 or 64 with F64");
    p->tile_n = 64;
    p->tile_p = 64;
    p->lds = false;
  } else {
    p->tile_n = 128;
    if (c->tile_p == 0) {
      p->tile_p = fitness_lds_fits(c->dtype, p->M_pad, 128) ? 128 : 64;
      p->lds = fitness_lds_fits(c->dtype, p->M_pad, p->tile_p) != 0;
      if (!p->lds) p->tile_p = 128;  // streaming kernel, 128 x 128 tiles
    } else {
      if (c->tile_p != 32 && c->tile_p != 64 && c->tile_p != 128) return bad("tile_p must be 0, 32, 64 or 128");
      if (!fitness_lds_fits(c->dtype, p->M_pad, c->tile_p)) return bad("a tile of tile_p chromosomes does not fit in LDS at this gene count");
      p->tile_p = c->tile_p;
      p->lds = true;
    }
  }
  p->N = c->n_patterns;
  p->N_pad = round_up(p->N, p->tile_n);
  p->n_rt = p->N_pad / p->tile_n;
  p->P_max_pad = (int)round_up(p->P_max, 128);
  p->n_rg_max = p->n_rt < 8193 ? p->n_rt : 8193;
  p->rt_per_wg_max = (int)((p->n_rt + p->n_rg_max - 1) / p->n_rg_max);
  p->elt = c->dtype == GAME_F64 ? 8 : c->dtype == GAME_F32 ? 4 : 2;
  p->acc = c->dtype == GAME_F64 ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  p->off_phi = take((size_t)p->N_pad * p->M_pad * p->elt);
  p->off_t = take((size_t)p->N_pad * p->acc);
  p->off_tile = take((size_t)p->P_max_pad * p->M_pad * p->elt);
  p->off_bias = take((size_t)p->P_max_pad * p->acc);
  p->off_pop0 = take((size_t)P * L * 4);
  p->off_pop1 = take((size_t)P * L * 4);
  p->off_psse = take((size_t)p->n_rg_max * p->P_max_pad * 8);
  p->off_pmiss = take((size_t)p->n_rg_max * p->P_max_pad * 4);
  p->off_mse = take((size_t)p->P_max * 8);
  p->off_miscls = take((size_t)p->P_max * 8);
  p->off_fit = take((size_t)p->P_max * 8);
  p->off_elite = take(kMaxElite * 4);
  p->off_state = take(sizeof(DevState));
  p->off_best = take((size_t)L * 4);
  p->n_pt_cap = (int)round_up(p->P_max, 32) / 32;  // tiles at the narrowest width
  p->n_counters = p->n_pt_cap + 3;
  p->off_cnt = take((size_t)p->n_counters * 4);
  // float32 copy of the patterns and re-score partials (not kept for F64)
  const bool f32x = c->dtype != GAME_F64;
  p->off_x = take(f32x ? (size_t)p->N * c->n_features * 4 : 0);
  p->off_rpart = take(f32x ? (size_t)rescore_grid() * 2 * kMaxRescore * 8 : 0);
  p->off_wheel = take((size_t)P * 8);
  p->off_mpart = take((size_t)(kPredictParts + 1) * 5 * 8);
  if (offspring) {
    const size_t Lz = (size_t)L;
    const int evrows = std::max<int>((int)P, p->P_eval);
    p->off_O = take((size_t)n_off * Lz * 4);
    p->off_keys = take((size_t)n_off * 8);
    p->off_rank = take((size_t)sur_rank_ints((int)n_off) * 4);
    p->off_sel = take((size_t)p->k_sel * 4);
    p->off_aud = take((size_t)std::max(p->audit, 1) * 4);
    p->off_surv = take((size_t)P * 4);
    p->off_evg = take((size_t)evrows * Lz * 4);
    p->off_emse = take((size_t)evrows * 8);
    p->off_emis = take((size_t)evrows * 8);
    p->off_efit = take((size_t)evrows * 8);
    p->off_snap = take((size_t)kMaxElite * 3 * 8);
    p->off_yhat = take((size_t)n_off * 4);
    p->off_rho = take(16);
    p->off_loss = take(16);
    p->off_sst = take(sizeof(SurState));
    p->off_log = take((size_t)kLogCap * 4 * 4);
    if (c->surrogate == GAME_SURROGATE_MLP) {
      const size_t np = (size_t)mlp_layout((int)L, p->H, p->H).total;
      p->rows_max = std::max<int>((int)n_off, std::max<int>(p->batch, (int)P));
      const MlpDims md{(int)L, p->H, p->H};
      p->off_prm = take(np * 4);
      p->off_am = take(np * 4);
      p->off_av = take(np * 4);
      p->off_step = take(16);
      p->off_WT = take((size_t)p->H * p->H * 4);
      p->mlp_scratch = mlp_scratch_floats(md, p->batch, p->rows_max);
      p->off_mscr = take((size_t)p->mlp_scratch * 4);
      p->off_buf = take((size_t)p->cap * Lz * 4);
      p->off_bufy = take((size_t)p->cap * 4);
    }
  }
  p->total = off;
  return GAME_OK;
}

FitnessGeom fitness_geometry(const Plan& p, int task, int dtype, int P_eval) {
  FitnessGeom g;
  g.n_pt = (P_eval + p.tile_p - 1) / p.tile_p;
  const int slots = fitness_persistent_slots(p, task, dtype);
  if (slots > 0) {
    // persistent: one workgroup per (row range, chromosome tile), as many as are resident
    int64_t R = p.row_groups > 0 ? p.row_groups : slots / g.n_pt;
    if (R < 1) R = 1;
    if (R > p.n_rt) R = p.n_rt;
    if (R > p.n_rg_max) R = p.n_rg_max;
    g.rt_per_wg = 0;
    g.n_rg = R;
    g.n_items = R * g.n_pt;
    g.grid = (g.n_items + 7) / 8 * 8;
    // 32-row range blocks where they balance the SIMDs better; FP32 tiles
    // only: the 16-bit classification kernels, bound by the VALU epilogue,
    // measured no faster with them at 100 000 x 1000 (FP32 1.7 % faster)
    g.ub = dtype == GAME_F32 ? fitness_range_block(p.N, R, g.n_pt, slots) : 4;
    return g;
  }
  // Enough workgroups to fill 256 CUs many times over, few enough that the
  // partial sums stay small next to the Phi traffic.
  const int64_t target = 8192;
  int64_t rpw = p.row_groups > 0 ? (p.n_rt + p.row_groups - 1) / p.row_groups
                                 : (p.n_rt * g.n_pt + target - 1) / target;
  if (rpw < 1) rpw = 1;
  if ((p.n_rt + rpw - 1) / rpw > p.n_rg_max) rpw = (p.n_rt + p.n_rg_max - 1) / p.n_rg_max;
  g.rt_per_wg = (int)rpw;
  g.n_rg = (p.n_rt + rpw - 1) / rpw;
  g.n_items = g.n_rg * g.n_pt;
  g.grid = (g.n_items + 7) / 8 * 8;
  g.ub = 4;
  return g;
}

}  // namespace game

namespace {

game_status check_ctx(game_ctx* ctx) {
  if (!ctx) return fail(GAME_E_INVALID, "context is NULL");
  if (ctx->poisoned) return fail(GAME_E_STATE, "context poisoned by an earlier device error");
  return GAME_OK;
}

game_status dev(game_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return GAME_OK;
  if (ctx) ctx->poisoned = true;
  return fail(GAME_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define GAME_TRY(expr)                   \
  do {                                   \
    const game_status _s = (expr);       \
    if (_s != GAME_OK) return _s;        \
  } while (0)

FitTail make_tail(game_ctx* c, int P_eval, bool population, double* mse2, double* miscls2,
                  double* fit2) {
  const Plan& p = c->plan;
  FitTail t{};
  t.counters = c->counters;
  t.n_pt_cap = p.n_pt_cap;
  t.P = P_eval;
  t.invN = 1.0 / (double)p.N;
  t.mse2 = mse2;
  t.miscls2 = miscls2;
  t.fit2 = fit2;
  if (population) {
    t.mse = c->mse;
    t.miscls = c->miscls;
    t.fit = c->fit;
    t.n_top = std::max(p.E > 0 ? p.E : 1, c->cfg.rescore_top);
    t.track = c->cfg.rescore_top > 0 ? 0 : 1;
    t.top = c->elite;
    t.st = c->state;
    t.pop0 = c->pop0;
    t.pop1 = c->pop1;
    t.L = p.L;
    t.best = c->best;
  }
  return t;
}

game_status enqueue_pack_population(game_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  GAME_TRY(dev(c,
               launch_pack(c->cfg.dtype, c->pop0, c->pop1, c->state, p.P, p.L, p.M, c->cfg.bias,
                           p.M_pad, p.P_max_pad, c->tile, c->biasv, s),
               "pack"));
  c->tile_fresh = true;
  return GAME_OK;
}

// Fitness of P_eval chromosomes (the gene tile must already hold them); the
// kernel's tail reduces, and for the population also ranks and tracks.
game_status enqueue_fitness(game_ctx* c, int P_eval, const FitTail& tail, hipStream_t s) {
  const Plan& p = c->plan;
  const FitnessGeom g = fitness_geometry(p, c->cfg.task, c->cfg.dtype, P_eval);
  return dev(c,
             launch_fitness(p, c->cfg.task, c->cfg.dtype, g, c->phi, c->tile,
                            c->cfg.bias ? c->biasv : nullptr, c->tvec, c->psse, c->pmiss,
                            c->state, tail, s),
             "fitness");
}

game_status enqueue_rescore(game_ctx* c, const float* genes, int n, double* mse, double* miscls,
                            bool population, hipStream_t s) {
  const Plan& p = c->plan;
  return dev(c,
             launch_rescore(c->xf, reinterpret_cast<const float*>(c->tvec), p.N,
                            c->cfg.n_features, c->cfg.degree, p.K, c->cfg.basis, p.M, p.L,
                            c->cfg.bias, c->cfg.task, genes, n, c->pop0, c->pop1, c->elite,
                            c->rpart, c->counters + p.n_pt_cap + 2, mse, miscls, c->state,
                            population ? c->state : nullptr, c->best, s),
             "rescore");
}

// Evaluate the current population, rank it and track the best chromosome
// (by the float32 re-score of the top-k when rescore_top > 0).
game_status enqueue_eval_population(game_ctx* c, double* mse, double* miscls, double* fit,
                                    hipStream_t s) {
  if (!c->tile_fresh) GAME_TRY(enqueue_pack_population(c, s));
  c->evaluated = true;
  GAME_TRY(enqueue_fitness(c, c->plan.P, make_tail(c, c->plan.P, true, mse, miscls, fit), s));
  if (c->cfg.rescore_top > 0)
    GAME_TRY(enqueue_rescore(c, nullptr, c->cfg.rescore_top, nullptr, nullptr, true, s));
  return GAME_OK;
}

// Parent selection and immigrants of a breed (the wheel buffer holds the
// cumulative roulette weights or the ranking, written by launch_select_prep).
void set_selection(game_ctx* c, BreedArgs& a) {
  a.sel = c->cfg.selection;
  a.wheel = c->wheel;
  a.order = reinterpret_cast<const int*>(c->wheel);
  a.n_imm = c->cfg.n_immigrants;
}

game_status enqueue_select_prep(game_ctx* c, const double* fit, hipStream_t s) {
  return dev(c,
             launch_select_prep(c->cfg.selection, fit, c->plan.P, c->wheel,
                                reinterpret_cast<int*>(c->wheel), c->state, s),
             "selection");
}

// Breed arguments of the generational form: E elites and P - E children
// written to the next population buffer and the gene tile.
BreedArgs evolve_args(game_ctx* c, const double* fit) {
  const Plan& p = c->plan;
  BreedArgs a{};
  a.pop0 = c->pop0;
  a.pop1 = c->pop1;
  a.fit = fit;
  a.elite = c->elite;
  a.P = p.P;
  a.L = p.L;
  a.E = p.E;
  a.n_children = p.n_off;
  a.k = p.k;
  a.thr_c = c->thr_c;
  a.thr_m = c->thr_m;
  a.sigma = (float)c->cfg.mutation_sigma;
  a.k0 = (uint32_t)c->cfg.seed;
  a.k1 = (uint32_t)(c->cfg.seed >> 32);
  a.tile = c->tile;
  a.biasv = c->biasv;
  a.M = p.M;
  a.M_pad = p.M_pad;
  a.bias = c->cfg.bias;
  a.counter = c->counters + p.n_pt_cap + 1;
  set_selection(c, a);
  return a;
}

game_status enqueue_evolve(game_ctx* c, const double* fit, hipStream_t s) {
  const BreedArgs a = evolve_args(c, fit);
  GAME_TRY(enqueue_select_prep(c, fit, s));
  GAME_TRY(dev(c, launch_breed(c->cfg.dtype, a, c->state, s), "breed"));
  c->tile_fresh = true;  // breed writes the new population into the tile
  return GAME_OK;
}

MlpDims mlp_dims(const game_ctx* c) { return MlpDims{c->plan.L, c->plan.H, c->plan.H}; }

// S Adam steps on minibatches drawn from the replay buffer.
game_status enqueue_train(game_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  const MlpDims d = mlp_dims(c);
  for (int i = 0; i < p.steps; ++i)
    GAME_TRY(dev(c,
                 mlp_train_step(d, c->prm, c->WT, c->am, c->av, c->step, (float)c->cfg.surrogate_lr,
                                c->buf, c->bufy, c->sst, c->cfg.seed, p.batch, p.n_recent, p.cap,
                                c->mscr, c->loss, c->state, s),
                 "mlp train"));
  return GAME_OK;
}

// Offspring form, first use: the population is evaluated exactly (and, with
// the MLP prescreen, stored in the replay buffer and learned from).
game_status enqueue_offspring_warmup(game_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  if (!c->have_eval) GAME_TRY(enqueue_eval_population(c, nullptr, nullptr, nullptr, s));
  if (p.sur == GAME_SURROGATE_MLP) {
    GAME_TRY(dev(c, launch_pop_copy(c->pop0, c->pop1, c->state, c->evg, (int64_t)p.P * p.L, 0, s),
                 "population copy"));
    GAME_TRY(dev(c, sur_append(c->evg, c->mse, p.P, p.L, c->buf, c->bufy, p.cap, c->sst, c->state, s),
                 "replay append"));
    GAME_TRY(enqueue_train(c, s));
  }
  c->have_eval = true;
  c->sur_warm = true;
  return GAME_OK;
}

// Offspring form, one generation (see surrogate.hip for the order of steps).
game_status enqueue_offspring_generation(game_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  DevState* st = c->state;
  const int k = p.k_sel, A = p.audit;
  // children of the current population
  BreedArgs a{};
  a.pop0 = c->pop0;
  a.pop1 = c->pop1;
  a.fit = c->fit;
  a.elite = c->elite;
  a.P = p.P;
  a.L = p.L;
  a.E = 0;
  a.n_children = p.n_off;
  a.k = p.k;
  a.thr_c = c->thr_c;
  a.thr_m = c->thr_m;
  a.sigma = (float)c->cfg.mutation_sigma;
  a.k0 = (uint32_t)c->cfg.seed;
  a.k1 = (uint32_t)(c->cfg.seed >> 32);
  a.M = p.M;
  a.M_pad = p.M_pad;
  a.bias = c->cfg.bias;
  a.out = c->O;
  set_selection(c, a);
  GAME_TRY(enqueue_select_prep(c, c->fit, s));
  GAME_TRY(dev(c, launch_breed(c->cfg.dtype, a, st, s), "breed offspring"));
  // prescreen: which children are evaluated exactly
  const int* sel = nullptr;
  if (p.sur == GAME_SURROGATE_MLP) {
    GAME_TRY(dev(c,
                 mlp_forward(mlp_dims(c), c->prm, c->WT, c->O, p.n_off, c->yhat, c->mscr, st, s),
                 "mlp forward"));
    GAME_TRY(dev(c, sur_keys(0, c->yhat, nullptr, p.n_off, 0, st, c->cfg.seed, c->keys, s), "keys"));
    GAME_TRY(dev(c, sur_select(c->keys, p.n_off, k, c->sel, c->rank_ws, st, s), "prescreen"));
    sel = c->sel;
  } else if (p.sur == GAME_SURROGATE_RANDOM) {
    GAME_TRY(dev(c, sur_keys(1, nullptr, nullptr, p.n_off, kTagPrescreen, st, c->cfg.seed, c->keys, s), "keys"));
    GAME_TRY(dev(c, sur_select(c->keys, p.n_off, k, c->sel, c->rank_ws, st, s), "prescreen"));
    sel = c->sel;
  }
  if (A > 0) {
    GAME_TRY(dev(c, sur_keys(1, nullptr, nullptr, p.n_off, kTagAudit, st, c->cfg.seed, c->keys, s), "keys"));
    GAME_TRY(dev(c, sur_select(c->keys, p.n_off, A, c->aud, c->rank_ws, st, s), "audit"));
  }
  // exact fitness of the selected children and the audit sample
  GAME_TRY(dev(c, sur_gather(c->O, sel, k, p.L, c->evg, st, s), "gather"));
  if (A > 0) GAME_TRY(dev(c, sur_gather(c->O, c->aud, A, p.L, c->evg + (size_t)k * p.L, st, s), "gather"));
  const int Ppad = (p.P_eval + p.tile_p - 1) / p.tile_p * p.tile_p;
  GAME_TRY(dev(c,
               launch_pack(c->cfg.dtype, c->evg, nullptr, nullptr, p.P_eval, p.L, p.M, c->cfg.bias,
                           p.M_pad, Ppad, c->tile, c->biasv, s),
               "pack"));
  c->tile_fresh = false;
  FitTail t = make_tail(c, p.P_eval, false, c->emse, c->emis, c->efit);
  GAME_TRY(enqueue_fitness(c, p.P_eval, t, s));
  if (p.sur == GAME_SURROGATE_MLP) {
    if (A > 0)
      GAME_TRY(dev(c, sur_spearman(c->yhat, c->aud, c->emse + k, A, c->rho, c->rank_ws, st, s), "spearman"));
    GAME_TRY(dev(c, sur_spearman(c->yhat, c->sel, c->emse, k, c->rho + 1, c->rank_ws, st, s), "spearman"));
    GAME_TRY(dev(c, sur_append(c->evg, c->emse, p.P_eval, p.L, c->buf, c->bufy, p.cap, c->sst, st, s),
                 "replay append"));
  }
  // next population: elites + best P - E of the selected children
  GAME_TRY(dev(c, sur_keys(2, nullptr, c->efit, k, 0, st, c->cfg.seed, c->keys, s), "keys"));
  GAME_TRY(dev(c, sur_select(c->keys, k, p.P - p.E, c->surv, c->rank_ws, st, s), "survivors"));
  GAME_TRY(dev(c, sur_snapshot(c->elite, p.E, c->fit, c->mse, c->miscls, c->snap, st, s), "snapshot"));
  GAME_TRY(dev(c,
               sur_merge(c->pop0, c->pop1, c->elite, c->snap, p.E, c->evg, c->surv, c->efit, c->emse,
                         c->emis, p.P, p.L, c->fit, c->mse, c->miscls, st, s),
               "merge"));
  if (p.sur == GAME_SURROGATE_MLP) GAME_TRY(enqueue_train(c, s));
  GAME_TRY(dev(c, sur_log(c->rho, p.sur == GAME_SURROGATE_MLP ? c->loss : nullptr, c->log, kLogCap,
                          c->sst, st, s),
               "log"));
  GAME_TRY(dev(c,
               sur_rank_track(c->fit, c->mse, c->miscls, p.P, p.E > 0 ? p.E : 1, c->elite, c->pop0,
                              c->pop1, p.L, c->best, st, 1, s),
               "rank"));
  return GAME_OK;
}

game_status enqueue_generation(game_ctx* c, hipStream_t s) {
  if (c->plan.offspring) return enqueue_offspring_generation(c, s);
  GAME_TRY(enqueue_eval_population(c, nullptr, nullptr, nullptr, s));
  GAME_TRY(enqueue_evolve(c, c->fit, s));
  return GAME_OK;
}

game_status build_graph(game_ctx* c, int n_gen, hipGraph_t* graph, hipGraphExec_t* exec) {
  if (*exec) return GAME_OK;
  if (!c->cap) GAME_TRY(dev(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "stream create"));
  GAME_TRY(dev(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "begin capture"));
  game_status st = GAME_OK;
  // The captured generations never pack (the breed writes the next tile);
  // callers pack the population before the first replay when the tile is
  // stale, so the flag is restored after the capture.
  // (The offspring form leaves the tile holding the evaluated children.)
  const bool fresh = c->tile_fresh;
  if (!c->plan.offspring) c->tile_fresh = true;
  for (int i = 0; i < n_gen && st == GAME_OK; ++i) st = enqueue_generation(c, c->cap);
  c->tile_fresh = c->plan.offspring ? false : fresh;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (st != GAME_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  GAME_TRY(dev(c, e, "end capture"));
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return dev(c, ei, "graph instantiate");
  }
  *graph = g;
  *exec = x;
  return GAME_OK;
}

uint64_t threshold(double p) { return (uint64_t)std::floor(p * 4294967296.0); }

}  // namespace

extern "C" {

void game_config_default(game_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->struct_size = sizeof(game_config);
  c->basis = GAME_BASIS_CHEBYSHEV;
  c->n_patterns = 0;
  c->n_features = 0;
  c->degree = 4;
  c->task = GAME_REGRESSION;
  c->dtype = GAME_F32;
  c->bias = 0;
  c->pop_size = 0;
  c->n_offspring = 0;
  c->elitism = 2;
  c->selection = GAME_SEL_TOURNAMENT;
  c->tournament_k = 3;
  c->max_generations = 100;
  c->p_crossover = 0.9;
  c->p_mutation = 0.05;
  c->mutation_sigma = 0.1;
  c->mse_threshold = 0.0;
  c->seed = 0;
  c->rescore_top = 0;
  c->surrogate = GAME_SURROGATE_NONE;
  c->surrogate_hidden = 256;
  c->surrogate_buffer = 50000;
  c->surrogate_steps = 16;
  c->surrogate_batch = 2048;
  c->audit = 256;
  c->prescreen_frac = 0.25;
  c->surrogate_lr = 3e-4;
  c->surrogate_recent = 0.75;
}

game_status game_query(const game_config* cfg, game_dims* d) {
  if (!d) return fail(GAME_E_INVALID, "dims is NULL");
  Plan p;
  char err[256];
  const game_status s = make_plan(cfg, &p, err, sizeof(err));
  if (s != GAME_OK) return fail(s, "%s", err);
  d->K = p.K;
  d->M = p.M;
  d->L = p.L;
  d->M_pad = p.M_pad;
  d->P = p.P;
  d->n_offspring = p.n_off;
  d->N_pad = p.N_pad;
  d->workspace_bytes = p.total;
  return GAME_OK;
}

game_status game_workspace_size(const game_config* cfg, size_t* bytes) {
  if (!bytes) return fail(GAME_E_INVALID, "bytes is NULL");
  game_dims d;
  GAME_TRY(game_query(cfg, &d));
  *bytes = d.workspace_bytes;
  return GAME_OK;
}

game_status game_build_basis(const game_config* cfg, const void* X, void* phi, int64_t ld, void* stream) {
  Plan p;
  char err[256];
  const game_status s = make_plan(cfg, &p, err, sizeof(err));
  if (s != GAME_OK) return fail(s, "%s", err);
  if (!X || !phi) return fail(GAME_E_INVALID, "X and phi must be device pointers");
  if (ld < p.M || ld * (int64_t)p.elt > 65536) return fail(GAME_E_INVALID, "ld must be in [M, 64 KiB / element size]");
  const hipError_t e = launch_basis(cfg, X, p.N, p.N, phi, ld, (hipStream_t)stream);
  if (e != hipSuccess) return fail(GAME_E_DEVICE, "basis: %s", hipGetErrorString(e));
  return GAME_OK;
}

game_status game_init(const game_config* cfg, const void* X, const void* t, void* ws,
                      size_t ws_bytes, void* stream, game_ctx** out) {
  if (!out) return fail(GAME_E_INVALID, "out is NULL");
  *out = nullptr;
  Plan p;
  char err[256];
  const game_status s = make_plan(cfg, &p, err, sizeof(err));
  if (s != GAME_OK) return fail(s, "%s", err);
  if (!X || !t || !ws) return fail(GAME_E_INVALID, "X, t and workspace must be device pointers");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(GAME_E_INVALID, "workspace must be 256-byte aligned");
  if (ws_bytes < p.total)
    return fail(GAME_E_OOM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, p.total);
  game_ctx* c = new (std::nothrow) game_ctx();
  if (!c) return fail(GAME_E_OOM, "host allocation of the context failed");
  c->cfg = *cfg;
  c->plan = p;
  c->stream = (hipStream_t)stream;
  c->ws = static_cast<unsigned char*>(ws);
  c->phi = c->ws + p.off_phi;
  c->tvec = c->ws + p.off_t;
  c->tile = c->ws + p.off_tile;
  c->biasv = c->ws + p.off_bias;
  c->pop0 = reinterpret_cast<float*>(c->ws + p.off_pop0);
  c->pop1 = reinterpret_cast<float*>(c->ws + p.off_pop1);
  c->counters = reinterpret_cast<uint32_t*>(c->ws + p.off_cnt);
  c->xf = reinterpret_cast<float*>(c->ws + p.off_x);
  c->rpart = reinterpret_cast<double*>(c->ws + p.off_rpart);
  c->wheel = reinterpret_cast<uint64_t*>(c->ws + p.off_wheel);
  c->mpart = reinterpret_cast<double*>(c->ws + p.off_mpart);
  if (p.offspring) {
    auto F = [&](size_t o) { return reinterpret_cast<float*>(c->ws + o); };
    auto D = [&](size_t o) { return reinterpret_cast<double*>(c->ws + o); };
    auto I = [&](size_t o) { return reinterpret_cast<int*>(c->ws + o); };
    c->O = F(p.off_O);
    c->keys = reinterpret_cast<uint64_t*>(c->ws + p.off_keys);
    c->rank_ws = I(p.off_rank);
    c->sel = I(p.off_sel);
    c->aud = I(p.off_aud);
    c->surv = I(p.off_surv);
    c->evg = F(p.off_evg);
    c->emse = D(p.off_emse);
    c->emis = D(p.off_emis);
    c->efit = D(p.off_efit);
    c->snap = D(p.off_snap);
    c->yhat = F(p.off_yhat);
    c->rho = F(p.off_rho);
    c->loss = F(p.off_loss);
    c->sst = reinterpret_cast<SurState*>(c->ws + p.off_sst);
    c->log = F(p.off_log);
    if (p.sur == GAME_SURROGATE_MLP) {
      c->prm = F(p.off_prm);
      c->am = F(p.off_am);
      c->av = F(p.off_av);
      c->step = reinterpret_cast<int32_t*>(c->ws + p.off_step);
      c->WT = F(p.off_WT);
      c->mscr = F(p.off_mscr);
      c->buf = F(p.off_buf);
      c->bufy = F(p.off_bufy);
    }
  }
  c->psse = reinterpret_cast<double*>(c->ws + p.off_psse);
  c->pmiss = reinterpret_cast<uint32_t*>(c->ws + p.off_pmiss);
  c->mse = reinterpret_cast<double*>(c->ws + p.off_mse);
  c->miscls = reinterpret_cast<double*>(c->ws + p.off_miscls);
  c->fit = reinterpret_cast<double*>(c->ws + p.off_fit);
  c->elite = reinterpret_cast<int*>(c->ws + p.off_elite);
  c->state = reinterpret_cast<DevState*>(c->ws + p.off_state);
  c->best = reinterpret_cast<float*>(c->ws + p.off_best);
  c->thr_c = threshold(cfg->p_crossover);
  c->thr_m = threshold(cfg->p_mutation);
  hipStream_t st = c->stream;
  game_status r = GAME_OK;
  if (r == GAME_OK) r = dev(c, launch_basis(cfg, X, p.N, p.N_pad, c->phi, p.M_pad, st), "basis");
  if (r == GAME_OK) r = dev(c, launch_copy_targets(cfg->dtype, t, p.N, p.N_pad, c->tvec, st), "targets");
  if (r == GAME_OK) r = dev(c, launch_init_population(c->pop0, p.P, p.L, cfg->seed, st), "init population");
  if (r == GAME_OK) r = dev(c, launch_state_init(c->state, c->counters, p.n_counters, st), "state init");
  if (r == GAME_OK && cfg->dtype != GAME_F64)
    r = dev(c, hipMemcpyAsync(c->xf, X, (size_t)p.N * cfg->n_features * 4, hipMemcpyDeviceToDevice, st),
            "pattern copy");
  if (r == GAME_OK) r = enqueue_pack_population(c, st);
  if (r == GAME_OK) {  // prime per-kernel attributes outside any graph capture
    (void)fitness_geometry(p, cfg->task, cfg->dtype, p.P_max);
    r = dev(c, select_prepare(cfg->selection), "prepare");
  }
  if (r == GAME_OK && p.offspring) {
    r = dev(c, hipMemsetAsync(c->sst, 0, sizeof(SurState), st), "surrogate state");
    if (r == GAME_OK) r = dev(c, hipMemsetAsync(c->rho, 0, 16, st), "surrogate state");
    if (r == GAME_OK) r = dev(c, hipMemsetAsync(c->loss, 0, 16, st), "surrogate state");
    if (r == GAME_OK && p.sur == GAME_SURROGATE_MLP) {
      r = dev(c, mlp_init(MlpDims{p.L, p.H, p.H}, c->prm, c->am, c->av, c->WT, cfg->seed, st), "mlp init");
      if (r == GAME_OK) r = dev(c, mlp_scratch_init(MlpDims{p.L, p.H, p.H}, c->mscr, st), "mlp init");
      if (r == GAME_OK) r = dev(c, hipMemsetAsync(c->step, 0, 16, st), "mlp init");
    }
  }
  if (r != GAME_OK) {
    delete c;
    return r;
  }
  *out = c;
  return GAME_OK;
}

game_status game_eval_fitness(game_ctx* c, const float* genes, int32_t P, double* mse,
                              double* miscls, double* fit) {
  GAME_TRY(check_ctx(c));
  if (genes == nullptr) {
    if (P != c->plan.P) return fail(GAME_E_INVALID, "P must equal the population size when genes is NULL");
    GAME_TRY(enqueue_eval_population(c, mse, miscls, fit, c->stream));
    c->have_eval = true;
    return GAME_OK;
  }
  if (P < 1 || P > c->plan.P_max) return fail(GAME_E_INVALID, "P must be in [1, %d]", c->plan.P_max);
  const Plan& p = c->plan;
  const int P_pad = (P + p.tile_p - 1) / p.tile_p * p.tile_p;
  c->tile_fresh = false;
  GAME_TRY(dev(c,
               launch_pack(c->cfg.dtype, genes, nullptr, nullptr, P, p.L, p.M, c->cfg.bias, p.M_pad,
                           P_pad, c->tile, c->biasv, c->stream),
               "pack"));
  return enqueue_fitness(c, P, make_tail(c, P, false, mse, miscls, fit), c->stream);
}

game_status game_step(game_ctx* c, const double* fit) {
  GAME_TRY(check_ctx(c));
  const Plan& p = c->plan;
  if (p.offspring) {
    if (fit) return fail(GAME_E_UNSUPPORTED, "the offspring form keeps its own exact fitness: pass NULL");
    if (!c->sur_warm) GAME_TRY(enqueue_offspring_warmup(c, c->stream));
    GAME_TRY(enqueue_offspring_generation(c, c->stream));
    c->have_eval = true;
    return GAME_OK;
  }
  if (fit == nullptr) {
    if (!c->have_eval) return fail(GAME_E_STATE, "game_step(NULL) needs game_eval_fitness(NULL) on the current population first");
    GAME_TRY(enqueue_evolve(c, c->fit, c->stream));
  } else {
    const int n_top = p.E > 0 ? p.E : 1;
    GAME_TRY(dev(c, launch_rank(fit, p.P, n_top, c->elite, nullptr, c->stream), "rank"));
    GAME_TRY(enqueue_evolve(c, fit, c->stream));
  }
  c->have_eval = false;
  return GAME_OK;
}

// The graphs game_advance(n) replays: chunks of kChunk generations and one
// graph of the n mod kChunk remaining ones (kept until another remainder is
// asked for).
static game_status prepare_advance(game_ctx* c, int32_t n) {
  if (n >= kChunk) GAME_TRY(build_graph(c, kChunk, &c->graphC, &c->execC));
  const int rem = n % kChunk;
  if (rem && c->nR != rem) {
    if (c->execR) {
      // the old remainder graph may still be running on the stream
      GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
      (void)hipGraphExecDestroy(c->execR);
      c->execR = nullptr;
    }
    if (c->graphR) (void)hipGraphDestroy(c->graphR);
    c->graphR = nullptr;
    c->nR = 0;
    GAME_TRY(build_graph(c, rem, &c->graphR, &c->execR));
    c->nR = rem;
  }
  return GAME_OK;
}

game_status game_advance_prepare(game_ctx* c, int32_t n) {
  GAME_TRY(check_ctx(c));
  if (n < 0) return fail(GAME_E_INVALID, "n_generations must be >= 0");
  return prepare_advance(c, n);
}

game_status game_advance(game_ctx* c, int32_t n) {
  GAME_TRY(check_ctx(c));
  if (n < 0) return fail(GAME_E_INVALID, "n_generations must be >= 0");
  if (n == 0) return GAME_OK;
  if (c->plan.offspring && !c->sur_warm) GAME_TRY(enqueue_offspring_warmup(c, c->stream));
  GAME_TRY(prepare_advance(c, n));
  if (!c->plan.offspring) GAME_TRY(enqueue_pack_population(c, c->stream));
  for (int i = 0; i + kChunk <= n; i += kChunk)
    GAME_TRY(dev(c, hipGraphLaunch(c->execC, c->stream), "graph launch"));
  if (n % kChunk) GAME_TRY(dev(c, hipGraphLaunch(c->execR, c->stream), "graph launch"));
  c->have_eval = c->plan.offspring;
  return GAME_OK;
}

game_status game_get_state(game_ctx* c, game_state* out, float* best_genes) {
  GAME_TRY(check_ctx(c));
  if (!out) return fail(GAME_E_INVALID, "out is NULL");
  DevState h;
  GAME_TRY(dev(c, hipMemcpyAsync(&h, c->state, sizeof(h), hipMemcpyDeviceToHost, c->stream), "state copy"));
  if (best_genes)
    GAME_TRY(dev(c, hipMemcpyAsync(best_genes, c->best, (size_t)c->plan.L * 4, hipMemcpyDeviceToHost, c->stream), "best copy"));
  GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
  out->generation = h.generation;
  out->stopped = h.stopped;
  out->best_index = h.best_index;
  out->stop_reason = h.stop_reason;
  out->best_mse = h.best_mse;
  out->best_fitness = h.best_fitness;
  out->best_miscls = h.best_miscls;
  return GAME_OK;
}

game_status game_run(game_ctx* c, game_result* res) {
  GAME_TRY(check_ctx(c));
  if (!res) return fail(GAME_E_INVALID, "result is NULL");
  const int G = c->cfg.max_generations;
  if (c->plan.offspring && !c->sur_warm) GAME_TRY(enqueue_offspring_warmup(c, c->stream));
  GAME_TRY(build_graph(c, kChunk, &c->graphC, &c->execC));
  if (!c->plan.offspring && !c->tile_fresh) GAME_TRY(enqueue_pack_population(c, c->stream));
  game_state s0;
  GAME_TRY(game_get_state(c, &s0, nullptr));
  GAME_TRY(dev(c, launch_run_arm(c->state, G, c->cfg.mse_threshold, c->stream), "arm"));
  game_state s = s0;
  // each chunk evaluates up to kChunk generations; kernels after the stop are no-ops
  for (int launched = 0; launched < G + kChunk; launched += kChunk) {
    GAME_TRY(dev(c, hipGraphLaunch(c->execC, c->stream), "graph launch"));
    GAME_TRY(game_get_state(c, &s, nullptr));
    if (s.stopped) break;
  }
  GAME_TRY(dev(c, launch_run_disarm(c->state, c->stream), "disarm"));
  GAME_TRY(game_get_state(c, &s, res->best_genes));
  if (!s.stopped) return fail(GAME_E_STATE, "run did not reach a stop condition");
  res->best_mse = s.best_mse;
  res->best_fitness = s.best_fitness;
  res->best_miscls = s.best_miscls;
  // classic form: generations evaluated (the stopping one is not bred from);
  // offspring form: offspring generations produced
  res->generations = s.generation - s0.generation + (c->plan.offspring ? 0 : 1);
  res->stop_reason = s.stop_reason;
  c->have_eval = true;  // the population is the last evaluated generation
  return GAME_OK;
}

game_status game_rescore(game_ctx* c, const float* genes, int32_t n, double* mse, double* miscls) {
  GAME_TRY(check_ctx(c));
  if (c->cfg.dtype == GAME_F64) return fail(GAME_E_UNSUPPORTED, "game_rescore is not available with F64");
  if (n < 1 || n > kMaxRescore || n > c->plan.P) return fail(GAME_E_INVALID, "n must be in [1, min(8, P)]");
  if ((int64_t)n * c->plan.L > 16384) return fail(GAME_E_INVALID, "n * L must be <= 16384");
  if (!genes && !c->have_eval)
    return fail(GAME_E_STATE, "game_rescore(NULL) needs a ranking of the current population");
  const int ranked = std::max(c->plan.E > 0 ? c->plan.E : 1, c->cfg.rescore_top);
  if (!genes && n > ranked) return fail(GAME_E_INVALID, "n exceeds the ranked elites (%d)", ranked);
  return enqueue_rescore(c, genes, n, mse, miscls, false, c->stream);
}

game_status game_rescore_noalloc(const game_config* cfg, const void* X, const void* t,
                                 const float* genes, int32_t n, double* mse, double* miscls,
                                 void* stream) {
  Plan p{};
  char err[256] = "";
  const game_status st = make_plan(cfg, &p, err, sizeof(err));
  if (st != GAME_OK) return fail(st, "%s", err);
  if (cfg->dtype == GAME_F64)
    return fail(GAME_E_UNSUPPORTED, "game_rescore_noalloc scores in float32: F64 configurations are not accepted");
  if (!X || !t || !genes) return fail(GAME_E_INVALID, "X, t and genes are required");
  if (n < 1 || n > kMaxRescore)
    return fail(GAME_E_INVALID, "n must be in [1, %d]: the fixed scratch holds the partial sums of at most %d "
                "chromosomes", kMaxRescore, kMaxRescore);
  if ((int64_t)n * p.L > 16384) return fail(GAME_E_INVALID, "n * L must be <= 16384");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = nullptr;
  uint32_t* counter = nullptr;
  hipError_t e = rescore_scratch(s, &part, &counter);
  if (e != hipSuccess) return fail(GAME_E_DEVICE, "re-score scratch: %s", hipGetErrorString(e));
  e = launch_rescore(static_cast<const float*>(X), static_cast<const float*>(t), p.N, cfg->n_features,
                     cfg->degree, p.K, cfg->basis, p.M, p.L, cfg->bias, cfg->task, genes, n, nullptr,
                     nullptr, nullptr, part, counter, mse, miscls, nullptr, nullptr, nullptr, s);
  if (e != hipSuccess) return fail(GAME_E_DEVICE, "rescore: %s", hipGetErrorString(e));
  return GAME_OK;
}

game_status game_surrogate_log(game_ctx* c, float* out, int32_t n_max, int32_t* n_out) {
  GAME_TRY(check_ctx(c));
  if (!out || !n_out || n_max < 0) return fail(GAME_E_INVALID, "log buffer and count are required");
  if (!c->plan.offspring) return fail(GAME_E_UNSUPPORTED, "no offspring form in this context");
  SurState h;
  std::vector<float> all((size_t)kLogCap * 4);
  GAME_TRY(dev(c, hipMemcpyAsync(&h, c->sst, sizeof(h), hipMemcpyDeviceToHost, c->stream), "log copy"));
  GAME_TRY(dev(c, hipMemcpyAsync(all.data(), c->log, all.size() * 4, hipMemcpyDeviceToHost, c->stream), "log copy"));
  GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
  const int n = std::min(std::min(h.n_logged, kLogCap), n_max);
  const int start = h.n_logged - n;
  for (int i = 0; i < n; ++i) {
    const int slot = (start + i) % kLogCap;
    for (int q = 0; q < 4; ++q) out[4 * i + q] = all[4 * slot + q];
  }
  *n_out = n;
  return GAME_OK;
}

game_status game_surrogate_buffer(game_ctx* c, float* genes, float* y, int32_t* count_head,
                                  float* mu_sigma) {
  GAME_TRY(check_ctx(c));
  if (c->plan.sur != GAME_SURROGATE_MLP) return fail(GAME_E_UNSUPPORTED, "no surrogate MLP in this context");
  const Plan& p = c->plan;
  if (genes)
    GAME_TRY(dev(c, hipMemcpyAsync(genes, c->buf, (size_t)p.cap * p.L * 4, hipMemcpyDeviceToDevice, c->stream), "buffer copy"));
  if (y) GAME_TRY(dev(c, hipMemcpyAsync(y, c->bufy, (size_t)p.cap * 4, hipMemcpyDeviceToDevice, c->stream), "buffer copy"));
  if (count_head || mu_sigma) {
    SurState h;
    GAME_TRY(dev(c, hipMemcpyAsync(&h, c->sst, sizeof(h), hipMemcpyDeviceToHost, c->stream), "buffer copy"));
    GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
    if (count_head) {
      count_head[0] = h.count;
      count_head[1] = h.head;
    }
    if (mu_sigma) {
      mu_sigma[0] = h.mu;
      mu_sigma[1] = h.sigma;
    }
  }
  return GAME_OK;
}

static game_status need_mlp(game_ctx* c) {
  GAME_TRY(check_ctx(c));
  if (c->plan.sur != GAME_SURROGATE_MLP) return fail(GAME_E_UNSUPPORTED, "no surrogate MLP in this context");
  return GAME_OK;
}

game_status game_mlp_params(game_ctx* c, float* params, int32_t dir) {
  GAME_TRY(need_mlp(c));
  if (!params || (dir != 0 && dir != 1)) return fail(GAME_E_INVALID, "params and dir 0|1 required");
  const size_t bytes = (size_t)mlp_layout(c->plan.L, c->plan.H, c->plan.H).total * 4;
  if (dir == 0) return dev(c, hipMemcpyAsync(params, c->prm, bytes, hipMemcpyDeviceToDevice, c->stream), "params");
  GAME_TRY(dev(c, hipMemcpyAsync(c->prm, params, bytes, hipMemcpyDeviceToDevice, c->stream), "params"));
  return dev(c, mlp_transpose(mlp_dims(c), c->prm, c->WT, c->stream), "params");
}

game_status game_mlp_forward(game_ctx* c, const float* X, int32_t n, float* y) {
  GAME_TRY(need_mlp(c));
  if (!X || !y || n < 1 || n > c->plan.rows_max) return fail(GAME_E_INVALID, "n must be in [1, %d]", c->plan.rows_max);
  return dev(c, mlp_forward(mlp_dims(c), c->prm, c->WT, X, n, y, c->mscr, nullptr, c->stream),
             "mlp forward");
}

game_status game_mlp_grads(game_ctx* c, const float* X, const float* target, int32_t n, float* grads,
                           float* loss) {
  GAME_TRY(need_mlp(c));
  if (!X || !target || !grads || n < 1 || n > c->plan.batch)
    return fail(GAME_E_INVALID, "n must be in [1, %d]", c->plan.batch);
  return dev(c,
             mlp_grads(mlp_dims(c), c->prm, c->WT, X, target, n, c->mscr, grads, loss, nullptr,
                       c->stream),
             "mlp grads");
}

game_status game_mlp_adam(game_ctx* c, const float* grads) {
  GAME_TRY(need_mlp(c));
  if (!grads) return fail(GAME_E_INVALID, "grads is NULL");
  return dev(c,
             mlp_adam(mlp_dims(c), c->prm, c->WT, grads, c->am, c->av, c->step,
                      (float)c->cfg.surrogate_lr, nullptr, c->stream),
             "mlp adam");
}

game_status game_get_population(game_ctx* c, float* genes) {
  GAME_TRY(check_ctx(c));
  if (!genes) return fail(GAME_E_INVALID, "genes is NULL");
  return dev(c, launch_pop_copy(c->pop0, c->pop1, c->state, genes, (int64_t)c->plan.P * c->plan.L, 0, c->stream), "population copy");
}

game_status game_set_population(game_ctx* c, const float* genes) {
  GAME_TRY(check_ctx(c));
  if (!genes) return fail(GAME_E_INVALID, "genes is NULL");
  c->have_eval = false;
  c->tile_fresh = false;
  c->sur_warm = false;
  return dev(c, launch_pop_copy(c->pop0, c->pop1, c->state, const_cast<float*>(genes), (int64_t)c->plan.P * c->plan.L, 1, c->stream), "population copy");
}

static PredictArgs predict_args(game_ctx* c, const float* genes, const void* X, const void* t,
                                int64_t n) {
  PredictArgs a{};
  a.X = X;
  a.t = t;
  a.n = n;
  a.F = c->cfg.n_features;
  a.D = c->cfg.degree;
  a.K = c->plan.K;
  a.basis = c->cfg.basis;
  a.M = c->plan.M;
  a.L = c->plan.L;
  a.bias = c->cfg.bias;
  a.task = c->cfg.task;
  a.genes = genes ? genes : c->best;
  a.part = c->mpart;
  return a;
}

game_status game_predict(game_ctx* c, const float* genes, const void* X, int64_t n, void* out) {
  GAME_TRY(check_ctx(c));
  if (!X || !out || n < 1) return fail(GAME_E_INVALID, "X, out and n >= 1 are required");
  if (!genes && !c->evaluated) return fail(GAME_E_STATE, "no best chromosome yet: evaluate or pass genes");
  PredictArgs a = predict_args(c, genes, X, nullptr, n);
  a.out = out;
  return dev(c, launch_predict(c->cfg.dtype == GAME_F64, a, c->stream), "predict");
}

game_status game_evaluate(game_ctx* c, const float* genes, const void* X, const void* t, int64_t n,
                          game_metrics* out) {
  GAME_TRY(check_ctx(c));
  if (!X || !t || !out || n < 1) return fail(GAME_E_INVALID, "X, t, out and n >= 1 are required");
  if (!genes && !c->evaluated) return fail(GAME_E_STATE, "no best chromosome yet: evaluate or pass genes");
  const PredictArgs a = predict_args(c, genes, X, t, n);
  double* res = c->mpart + (size_t)kPredictParts * 5;
  double h[5];
  GAME_TRY(dev(c, launch_metrics(c->cfg.dtype == GAME_F64, a, res, c->stream), "metrics"));
  GAME_TRY(dev(c, hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, c->stream), "metrics"));
  GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
  out->n = n;
  out->mse = h[0] / (double)n;
  out->rmse = std::sqrt(out->mse);
  out->tp = (int64_t)h[1];
  out->fp = (int64_t)h[2];
  out->tn = (int64_t)h[3];
  out->fn = (int64_t)h[4];
  const bool cls = c->cfg.task == GAME_CLASSIFICATION;
  const double nan = std::nan("");
  out->accuracy = cls ? (double)(out->tp + out->tn) / (double)n : nan;
  out->completeness = cls && out->tp + out->fn ? (double)out->tp / (double)(out->tp + out->fn) : nan;
  out->contamination = cls && out->tp + out->fp ? (double)out->fp / (double)(out->tp + out->fp) : nan;
  return GAME_OK;
}

// Checkpoint sections: every device buffer that carries state from one
// generation to the next (the basis, targets, gene tile and scratch are
// rebuilt or rewritten).
struct Section {
  void* dev;
  size_t bytes;
};

static std::vector<Section> checkpoint_sections(game_ctx* c) {
  const Plan& p = c->plan;
  std::vector<Section> v = {
      {c->state, sizeof(DevState)},
      {c->pop0, (size_t)p.P * p.L * 4},
      {c->pop1, (size_t)p.P * p.L * 4},
      {c->mse, (size_t)p.P_max * 8},
      {c->miscls, (size_t)p.P_max * 8},
      {c->fit, (size_t)p.P_max * 8},
      {c->elite, (size_t)kMaxElite * 4},
      {c->best, (size_t)p.L * 4},
  };
  if (p.offspring) {
    v.push_back({c->sst, sizeof(SurState)});
    v.push_back({c->log, (size_t)kLogCap * 4 * 4});
    v.push_back({c->rho, 16});
    v.push_back({c->loss, 16});
    if (p.sur == GAME_SURROGATE_MLP) {
      const size_t np = (size_t)mlp_layout(p.L, p.H, p.H).total * 4;
      v.push_back({c->prm, np});
      v.push_back({c->am, np});
      v.push_back({c->av, np});
      v.push_back({c->step, 16});
      v.push_back({c->buf, (size_t)p.cap * p.L * 4});
      v.push_back({c->bufy, (size_t)p.cap * 4});
    }
  }
  return v;
}

struct CheckpointHeader {
  char magic[8];
  uint32_t version, config_bytes;
  uint64_t total_bytes;
  int32_t have_eval, sur_warm;
  game_config cfg;
};

// The configuration a checkpoint must match: all but the run limits.
static game_config comparable(game_config c) {
  c.max_generations = 0;
  c.mse_threshold = 0.0;
  return c;
}

game_status game_save(game_ctx* c, void* host, size_t* bytes) {
  GAME_TRY(check_ctx(c));
  if (!bytes) return fail(GAME_E_INVALID, "bytes is NULL");
  const std::vector<Section> secs = checkpoint_sections(c);
  size_t need = sizeof(CheckpointHeader);
  for (const Section& x : secs) need += x.bytes;
  if (!host) {
    *bytes = need;
    return GAME_OK;
  }
  if (*bytes < need) return fail(GAME_E_INVALID, "buffer of %zu bytes, %zu needed", *bytes, need);
  CheckpointHeader h{};
  std::memcpy(h.magic, "GAMECKPT", 8);
  h.version = 1;
  h.config_bytes = sizeof(game_config);
  h.total_bytes = need;
  h.have_eval = c->have_eval;
  h.sur_warm = c->sur_warm;
  h.cfg = c->cfg;
  unsigned char* out = static_cast<unsigned char*>(host);
  std::memcpy(out, &h, sizeof(h));
  size_t off = sizeof(h);
  for (const Section& x : secs) {
    GAME_TRY(dev(c, hipMemcpyAsync(out + off, x.dev, x.bytes, hipMemcpyDeviceToHost, c->stream), "save"));
    off += x.bytes;
  }
  GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
  *bytes = need;
  return GAME_OK;
}

game_status game_load(game_ctx* c, const void* host, size_t bytes) {
  GAME_TRY(check_ctx(c));
  if (!host || bytes < sizeof(CheckpointHeader)) return fail(GAME_E_INVALID, "not a checkpoint");
  CheckpointHeader h;
  std::memcpy(&h, host, sizeof(h));
  if (std::memcmp(h.magic, "GAMECKPT", 8) != 0 || h.version != 1 || h.config_bytes != sizeof(game_config))
    return fail(GAME_E_INVALID, "not a checkpoint of this library version");
  const game_config a = comparable(h.cfg), b = comparable(c->cfg);
  if (std::memcmp(&a, &b, sizeof(a)) != 0)
    return fail(GAME_E_INVALID, "the checkpoint was taken with another configuration");
  const std::vector<Section> secs = checkpoint_sections(c);
  size_t need = sizeof(CheckpointHeader);
  for (const Section& x : secs) need += x.bytes;
  if (h.total_bytes != need || bytes < need) return fail(GAME_E_INVALID, "checkpoint size mismatch");
  const unsigned char* in = static_cast<const unsigned char*>(host);
  size_t off = sizeof(h);
  for (const Section& x : secs) {
    GAME_TRY(dev(c, hipMemcpyAsync(x.dev, in + off, x.bytes, hipMemcpyHostToDevice, c->stream), "load"));
    off += x.bytes;
  }
  if (c->plan.sur == GAME_SURROGATE_MLP)
    GAME_TRY(dev(c, mlp_transpose(mlp_dims(c), c->prm, c->WT, c->stream), "load"));
  GAME_TRY(dev(c, hipStreamSynchronize(c->stream), "synchronize"));
  c->have_eval = h.have_eval != 0;
  c->sur_warm = h.sur_warm != 0;
  c->evaluated = true;
  c->tile_fresh = false;
  return GAME_OK;
}

game_status game_time_fitness(game_ctx* c, int32_t reps, float* ms) {
  GAME_TRY(check_ctx(c));
  if (reps < 1 || !ms) return fail(GAME_E_INVALID, "reps must be >= 1 and ms non-NULL");
  const Plan& p = c->plan;
  if (!c->tile_fresh) GAME_TRY(enqueue_pack_population(c, c->stream));
  // the population tail (ranking, best tracking) as in a generation
  const FitTail tail = make_tail(c, p.P, true, nullptr, nullptr, nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GAME_TRY(dev(c, hipEventCreate(&e0), "event create"));
  game_status s = dev(c, hipEventCreate(&e1), "event create");
  if (s == GAME_OK) s = dev(c, hipEventRecord(e0, c->stream), "event record");
  for (int r = 0; r < reps && s == GAME_OK; ++r) s = enqueue_fitness(c, p.P, tail, c->stream);
  if (s == GAME_OK) s = dev(c, hipEventRecord(e1, c->stream), "event record");
  if (s == GAME_OK) s = dev(c, hipEventSynchronize(e1), "event synchronize");
  float total = 0.f;
  if (s == GAME_OK) s = dev(c, hipEventElapsedTime(&total, e0, e1), "elapsed time");
  if (s == GAME_OK) *ms = total / (float)reps;
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return s;
}

void game_destroy(game_ctx* c) {
  if (!c) return;
  if (c->execR) (void)hipGraphExecDestroy(c->execR);
  if (c->execC) (void)hipGraphExecDestroy(c->execC);
  if (c->graphR) (void)hipGraphDestroy(c->graphR);
  if (c->graphC) (void)hipGraphDestroy(c->graphC);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

const char* game_status_str(game_status s) {
  switch (s) {
    case GAME_OK: return "GAME_OK";
    case GAME_E_INVALID: return "GAME_E_INVALID";
    case GAME_E_OOM: return "GAME_E_OOM";
    case GAME_E_DEVICE: return "GAME_E_DEVICE";
    case GAME_E_STATE: return "GAME_E_STATE";
    case GAME_E_UNSUPPORTED: return "GAME_E_UNSUPPORTED";
  }
  return "unknown game_status";
}

const char* game_last_error(void) { return g_err; }

}  // extern "C"

// ====================================================== batched form
// Many independent contexts advanced by one persistent scheduler launch
// (flow_kernel): each run moves through its own fitness, wheel / ranking and
// breed phases, so a run's generation takes about its own work.  Each
// context keeps its own workspace, state and stop rule.
struct game_batch {
  std::vector<game_ctx*> ctx;
  std::vector<size_t> ws_off;
  int n = 0, dtype = 0;
  hipStream_t stream = nullptr;
  FlowRun* druns = nullptr;  // device table, cheapest generation first
  FlowCtl* ctl = nullptr;
  FlowQueue* q = nullptr;
  uint64_t *t_start = nullptr, *t_done = nullptr;  // per context: G slots each
  int G = 0;  // timestamp slots per context
  int grid = 0;
  size_t lds = 0;
  uint64_t idle_ticks = 0;
  double gen_flop = 0.0;  // one generation of every run (2 N M P summed)
  bool poisoned = false;
  std::vector<int> tile_p, row_groups;  // per context, as tuned
  float tune_ms = 0.0f;
};

namespace {

// Generations each run may breed per scheduler launch: a launch of the
// workload of 64 runs of up to 5e5 patterns lasts about 2.5 s at this size.
constexpr int kFlowChunk = 128;
// FP32 contraction rate (flop/s) the fair-share deadlines assume; only the
// runs' relative shares depend on it.
constexpr double kFlowRate = 80e12;

struct BatchLayout {
  std::vector<size_t> ws_off;
  size_t tab_off, runs_off, ctl_off, q_off, ts_off, td_off, total;
  int G;
};

game_status batch_layout(const game_config* cfgs, int n, BatchLayout* L, int* dtype) {
  if (!cfgs || n < 1 || n > 4096) return fail(GAME_E_INVALID, "n_runs must be in [1, 4096]");
  size_t off = 0;
  int G = 1;
  L->ws_off.resize(n);
  for (int i = 0; i < n; ++i) {
    Plan p;
    char err[256];
    const game_status s = game::make_plan(&cfgs[i], &p, err, sizeof(err));
    if (s != GAME_OK) return fail(s, "run %d: %s", i, err);
    if (i == 0) *dtype = cfgs[i].dtype;
    if (cfgs[i].dtype != *dtype) return fail(GAME_E_INVALID, "all runs of a batch share one dtype");
    if (cfgs[i].dtype == GAME_F64) return fail(GAME_E_UNSUPPORTED, "the batched form runs F32, BF16 or F16");
    if (p.offspring || cfgs[i].rescore_top > 0)
      return fail(GAME_E_UNSUPPORTED, "run %d: the batched form runs the generational GA only", i);
    if (!p.lds) return fail(GAME_E_UNSUPPORTED, "run %d: too many genes for the LDS-staged kernel", i);
    L->ws_off[i] = off;
    off = align256(off + p.total);
    G = std::max(G, cfgs[i].max_generations);
  }
  L->G = G;
  L->tab_off = off;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L->runs_off = take(sizeof(FlowRun) * n);
  L->ctl_off = take(sizeof(FlowCtl) * n);
  L->q_off = take(sizeof(FlowQueue));
  L->ts_off = take(sizeof(uint64_t) * (size_t)G * n);
  L->td_off = take(sizeof(uint64_t) * (size_t)G * n);
  L->total = off;
  return GAME_OK;
}

game_status bdev(game_batch* b, hipError_t e, const char* what) {
  if (e == hipSuccess) return GAME_OK;
  b->poisoned = true;
  return fail(GAME_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// The scheduler's table for the contexts' current tile widths and row
// ranges, with each run's fair-share generation span, its dynamic LDS (the widest gene tile, or a ranking's sort) and
// the resident grid.
game_status batch_tables(game_batch* b) {
  std::vector<FlowRun> runs(b->n);
  std::vector<double> cost(b->n);
  std::vector<int> order(b->n);
  b->lds = 0;
  b->gen_flop = 0.0;
  int dev_id = 0, rate_khz = 0;
  GAME_TRY(bdev(b, hipGetDevice(&dev_id), "device"));
  GAME_TRY(bdev(b, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev_id), "clock rate"));
  const double ticks_per_s = 1e3 * (rate_khz > 0 ? rate_khz : 100000);
  for (int i = 0; i < b->n; ++i) {
    game_ctx* c = b->ctx[i];
    const Plan& p = c->plan;
    const FitnessGeom g = fitness_geometry(p, c->cfg.task, c->cfg.dtype, p.P);
    FlowRun& f = runs[i];
    f.phi = c->phi;
    f.tile = c->tile;
    f.biasv = c->cfg.bias ? c->biasv : nullptr;
    f.tvec = c->tvec;
    f.psse = c->psse;
    f.pmiss = c->pmiss;
    f.st = c->state;
    f.tail = make_tail(c, p.P, true, nullptr, nullptr, nullptr);
    f.breed = evolve_args(c, c->fit);
    f.breed.counter = nullptr;
    f.wheel = c->wheel;
    f.t_start = b->t_start + (size_t)i * b->G;
    f.t_done = b->t_done + (size_t)i * b->G;
    f.t_cap = b->G;
    f.N = p.N;
    f.M_pad = p.M_pad;
    f.ldsw = fitness_lds_stride(c->cfg.dtype, p.M_pad);
    f.n_pt = g.n_pt;
    f.n_ranges = (int)g.n_rg;
    f.part_ld = p.P_max_pad;
    f.task = c->cfg.task;
    f.tile_p = p.tile_p;
    f.ub = g.ub;
    f.n_fit = g.n_pt * (int)g.n_rg;
    f.n_breed = breed_blocks(f.breed);
    f.sel = c->cfg.selection;
    f.rank_pow2 = 1;
    while (f.rank_pow2 < p.P) f.rank_pow2 <<= 1;
    cost[i] = (double)p.N * p.M_pad * p.P;
    b->gen_flop += 2.0 * (double)p.N * p.M * p.P;
    // fair share: the generation (its contraction at kFlowRate, plus about
    // 20 us of tail and breed) with 1/n of the device
    f.span = (uint64_t)(b->n * (2.0 * cost[i] / kFlowRate + 20e-6) * ticks_per_s);
    order[i] = i;
    b->lds = std::max(b->lds, fitness_lds_bytes(c->cfg.dtype, p.M_pad, p.tile_p));
    if (f.sel == GAME_SEL_RANKING) b->lds = std::max(b->lds, (size_t)f.rank_pow2 * 12);
  }
  // the table lists the cheapest generation first: of runs with equal
  // deadlines the cheaper one is served first
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] < cost[y]; });
  std::vector<FlowRun> sorted(b->n);
  for (int k = 0; k < b->n; ++k) sorted[k] = runs[order[k]];
  const int slots = flow_slots(b->dtype, b->lds);
  if (slots <= 0) return fail(GAME_E_DEVICE, "batched scheduler cannot be resident");
  b->grid = slots;
  // a workgroup that finds no open item for this long gives up (a phase of
  // one run never takes nearly this long: 20x one generation of every run
  // at 50 TFLOP/s, at least 2 s)
  // (GAME_FLOW_IDLE_US overrides it, in microseconds)
  double idle_s = std::max(2.0, 20.0 * b->gen_flop / 50e12);
  if (const char* env = std::getenv("GAME_FLOW_IDLE_US")) {
    char* end = nullptr;
    const double us = std::strtod(env, &end);
    if (end != env && us > 0.0) idle_s = us * 1e-6;
  }
  b->idle_ticks = std::max<uint64_t>(1, (uint64_t)(idle_s * ticks_per_s));
  GAME_TRY(bdev(b, hipMemcpyAsync(b->druns, sorted.data(), sizeof(FlowRun) * b->n, hipMemcpyHostToDevice, b->stream), "batch tables"));
  GAME_TRY(bdev(b, hipStreamSynchronize(b->stream), "synchronize"));
  return GAME_OK;
}

// A workgroup of the scheduler found no open item for too long: poison the
// batch and name the first run that had not parked, with its phase state.
game_status batch_stall(game_batch* b) {
  b->poisoned = true;
  std::vector<FlowCtl> c(b->n);
  std::vector<FlowRun> r(b->n);
  char what[512] = "";
  if (hipMemcpy(c.data(), b->ctl, sizeof(FlowCtl) * b->n, hipMemcpyDeviceToHost) == hipSuccess &&
      hipMemcpy(r.data(), b->druns, sizeof(FlowRun) * b->n, hipMemcpyDeviceToHost) == hipSuccess) {
    for (int i = 0; i < b->n; ++i) {
      const uint32_t e = (uint32_t)(c[i].word >> 32);
      if (e == 0xFFFFFFFFu) continue;
      int n = snprintf(what, sizeof(what),
                       "; table run %d: epoch %u (phase %u), word claims %u, done %u, items %d/1/%d "
                       "(fitness/wheel/breed), ranges %d, gen %d, slices",
                       i, e, e % 3u, (uint32_t)c[i].word, c[i].done, r[i].n_fit, r[i].n_breed, r[i].n_ranges,
                       c[i].gen);
      for (int x = 0; x < kXcds && n > 0 && n < (int)sizeof(what); ++x)
        n += snprintf(what + n, sizeof(what) - n, " %u:%u", (uint32_t)(c[i].xw[x] >> 32), (uint32_t)c[i].xw[x]);
      break;
    }
  }
  return fail(GAME_E_DEVICE, "batched scheduler: a workgroup found no open item for too long%s", what);
}

// One scheduler launch (arm, scheduler, status) and its queue afterwards.
game_status batch_launch(game_batch* b, int chunk, int first, int eval_only, FlowQueue* hq) {
  GAME_TRY(bdev(b,
                launch_flow(b->dtype, b->druns, b->n, b->ctl, b->q, b->grid, b->lds, chunk, first,
                            eval_only, b->idle_ticks, b->stream),
                "batched scheduler"));
  if (!hq) return GAME_OK;
  GAME_TRY(bdev(b, hipMemcpyAsync(hq, b->q, sizeof(FlowQueue), hipMemcpyDeviceToHost, b->stream), "status copy"));
  GAME_TRY(bdev(b, hipStreamSynchronize(b->stream), "synchronize"));
  if (hq->error) return batch_stall(b);
  return GAME_OK;
}

// Apply per-context tile widths and row ranges (each must fit), rebuild tables.
game_status batch_apply(game_batch* b, const std::vector<int>& tp, const std::vector<int>& rg) {
  for (int i = 0; i < b->n; ++i) {
    Plan& p = b->ctx[i]->plan;
    if (!fitness_lds_fits(b->dtype, p.M_pad, tp[i])) return fail(GAME_E_INVALID, "tile does not fit");
    p.tile_p = tp[i];
    p.row_groups = rg[i];
  }
  b->tile_p = tp;
  b->row_groups = rg;
  return batch_tables(b);
}

// Mean duration (ms) of one scheduler launch that evaluates every run's
// current population once (the fitness phase only).
game_status batch_time(game_batch* b, int reps, float* ms) {
  for (game_ctx* c : b->ctx)
    if (!c->tile_fresh) GAME_TRY(enqueue_pack_population(c, b->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GAME_TRY(bdev(b, hipEventCreate(&e0), "event"));
  game_status st = bdev(b, hipEventCreate(&e1), "event");
  if (st == GAME_OK) st = batch_launch(b, 0, 0, 1, nullptr);  // warm
  if (st == GAME_OK) st = bdev(b, hipEventRecord(e0, b->stream), "event");
  for (int r = 0; r < reps && st == GAME_OK; ++r) st = batch_launch(b, 0, 0, 1, nullptr);
  if (st == GAME_OK) st = bdev(b, hipEventRecord(e1, b->stream), "event");
  if (st == GAME_OK) st = bdev(b, hipEventSynchronize(e1), "event");
  float t = 0.0f;
  if (st == GAME_OK) st = bdev(b, hipEventElapsedTime(&t, e0, e1), "event");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  FlowQueue hq{};
  if (st == GAME_OK) st = bdev(b, hipMemcpy(&hq, b->q, sizeof(hq), hipMemcpyDeviceToHost), "status copy");
  if (st == GAME_OK && hq.error) st = batch_stall(b);
  if (st == GAME_OK) *ms = t / (float)reps;
  for (game_ctx* c : b->ctx) c->evaluated = true;
  return st;
}

// Per-run results of the batched tuner, kept for the process and keyed by a
// run's shape (dtype, task, padded genes, population in 32s, log2 of the
// patterns): the tile width and the row-range rule (item size) the run had
// in the fastest batch it was tuned in.  A batch whose runs all have a
// cached choice starts from it instead of sweeping.
struct ShapeKey {
  int dtype, task, M_pad, P32, logN;
  bool operator<(const ShapeKey& o) const {
    return std::tie(dtype, task, M_pad, P32, logN) < std::tie(o.dtype, o.task, o.M_pad, o.P32, o.logN);
  }
};
struct ShapeChoice {
  int tile_p;
  double work;  // row-tile x chromosome x gene units per item
};
std::mutex g_tune_mu;
std::map<ShapeKey, ShapeChoice>& tune_cache() {
  static std::map<ShapeKey, ShapeChoice> m;
  return m;
}
ShapeKey shape_key(const game_ctx* c) {
  const Plan& p = c->plan;
  int logN = 0;
  while ((int64_t(1) << (logN + 1)) <= p.N) ++logN;
  return ShapeKey{c->cfg.dtype, c->cfg.task, p.M_pad, (p.P + 31) / 32, logN};
}

// Row ranges giving items of about W row-tile x chromosome x gene units.
int ranges_for(const Plan& p, int tp, double W) {
  const double per_rt = (double)tp * p.M_pad;
  const int64_t rts = std::max<int64_t>(1, (int64_t)std::llround(W / per_rt));
  return (int)std::min<int64_t>(std::max<int64_t>((p.n_rt + rts - 1) / rts, 1), p.n_rg_max);
}

// Widest tile within an LDS budget that a population of P fills.
int widest_tile(int dtype, const Plan& p, size_t budget) {
  for (int cand : {128, 64})
    if (cand <= round_up(p.P, 32) && fitness_lds_bytes(dtype, p.M_pad, cand) <= budget) return cand;
  return fitness_lds_fits(dtype, p.M_pad, 32) ? 32 : p.tile_p;
}

// The tuner, on evaluation-only scheduler launches over the runs' current
// populations (a configured tile_p / row_groups is always kept):
//   1. sweep: an LDS budget (the scheduler's dynamic LDS is its widest
//      tile; above 80 KiB one workgroup fits a CU instead of two) x an item
//      size W; every run takes the widest tile within the budget and ranges
//      of about W units per item;
//   2. refinement per class of runs (task x padded gene count up to 64, 128,
//      256, more): the class's runs one tile width narrower, each run's
//      item size kept; kept where the launch is faster;
//   3. the per-run choices go to the shape cache.
// With a cached choice for every run, the batch starts from those and
// steps 1-2 are skipped.
game_status batch_tune(game_batch* b) {
  const int n = b->n;
  std::vector<int> tp(n), rg(n);
  std::vector<double> wk(n, 0.0);
  auto fixed_tp = [&](int i) { return b->ctx[i]->cfg.tile_p; };
  auto fixed_rg = [&](int i) { return b->ctx[i]->cfg.row_groups; };
  auto build = [&](int i, int t, double W) {
    const Plan& p = b->ctx[i]->plan;
    tp[i] = fixed_tp(i) > 0 ? fixed_tp(i) : t;
    rg[i] = fixed_rg(i) > 0 ? fixed_rg(i) : ranges_for(p, tp[i], W);
    wk[i] = W;
  };
  bool all_cached = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < n; ++i) {
      auto it = tune_cache().find(shape_key(b->ctx[i]));
      if (it == tune_cache().end()) {
        all_cached = false;
        break;
      }
      build(i, it->second.tile_p, it->second.work);
    }
  }
  float best = 0.0f;
  if (all_cached) {
    GAME_TRY(batch_apply(b, tp, rg));
    GAME_TRY(batch_time(b, 3, &best));
  } else {
    const size_t budgets[] = {98304, 49152};
    // the small sizes are for batches of few runs, whose items must still
    // outnumber the scheduler's workgroups
    const double works[] = {0.25 * (1 << 20), 0.5 * (1 << 20), 1.0 * (1 << 20), 2.0 * (1 << 20),
                            4.0 * (1 << 20), 8.0 * (1 << 20), 16.0 * (1 << 20)};
    std::vector<int> btp, brg;
    std::vector<double> bwk;
    for (size_t budget : budgets)
      for (double W : works) {
        for (int i = 0; i < n; ++i) build(i, widest_tile(b->dtype, b->ctx[i]->plan, budget), W);
        GAME_TRY(batch_apply(b, tp, rg));
        float ms = 0.0f;
        GAME_TRY(batch_time(b, 3, &ms));
        if (btp.empty() || ms < best) {
          best = ms;
          btp = tp;
          brg = rg;
          bwk = wk;
        }
      }
    tp = btp;
    rg = brg;
    wk = bwk;
    auto cls = [&](int i) {
      const int M = b->ctx[i]->plan.M_pad;
      return 4 * b->ctx[i]->cfg.task + (M <= 64 ? 0 : M <= 128 ? 1 : M <= 256 ? 2 : 3);
    };
    for (int k = 0; k < 8; ++k) {
      std::vector<int> ctp = tp, crg = rg;
      bool any = false;
      for (int i = 0; i < n; ++i) {
        if (cls(i) != k || fixed_tp(i) > 0 || tp[i] <= 32) continue;
        ctp[i] = tp[i] / 2;
        if (fixed_rg(i) == 0) crg[i] = ranges_for(b->ctx[i]->plan, ctp[i], wk[i]);
        any = true;
      }
      if (!any) continue;
      GAME_TRY(batch_apply(b, ctp, crg));
      float ms = 0.0f;
      GAME_TRY(batch_time(b, 3, &ms));
      if (ms < best) {
        best = ms;
        tp = ctp;
        rg = crg;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < n; ++i) tune_cache()[shape_key(b->ctx[i])] = ShapeChoice{tp[i], wk[i]};
  }
  b->tune_ms = best;
  return batch_apply(b, tp, rg);
}

game_status check_batch(game_batch* b) {
  if (!b) return fail(GAME_E_INVALID, "batch is NULL");
  if (b->poisoned) return fail(GAME_E_STATE, "batch poisoned by an earlier device error");
  for (game_ctx* c : b->ctx)
    if (c->poisoned) return fail(GAME_E_STATE, "batch poisoned by an earlier device error");
  return GAME_OK;
}

}  // namespace

extern "C" {

game_status game_batch_workspace_size(const game_config* cfgs, int32_t n_runs, size_t* bytes) {
  if (!bytes) return fail(GAME_E_INVALID, "bytes is NULL");
  BatchLayout L;
  int dtype = 0;
  GAME_TRY(batch_layout(cfgs, n_runs, &L, &dtype));
  *bytes = L.total;
  return GAME_OK;
}

void game_batch_destroy(game_batch* b) {
  if (!b) return;
  for (game_ctx* c : b->ctx) game_destroy(c);
  delete b;
}

game_status game_batch_init(const game_config* cfgs, int32_t n_runs, const void* const* X_devs,
                            const void* const* t_devs, void* ws, size_t ws_bytes, void* stream,
                            game_batch** out) {
  if (!out) return fail(GAME_E_INVALID, "out is NULL");
  *out = nullptr;
  BatchLayout L;
  int dtype = 0;
  GAME_TRY(batch_layout(cfgs, n_runs, &L, &dtype));
  if (!X_devs || !t_devs || !ws) return fail(GAME_E_INVALID, "X_devs, t_devs and workspace are required");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(GAME_E_INVALID, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(GAME_E_OOM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
  for (int i = 0; i < n_runs; ++i)
    if (!X_devs[i] || !t_devs[i]) return fail(GAME_E_INVALID, "run %d: X and t must be device pointers", i);
  game_batch* b = new (std::nothrow) game_batch();
  if (!b) return fail(GAME_E_OOM, "host allocation of the batch failed");
  b->n = n_runs;
  b->dtype = dtype;
  b->stream = (hipStream_t)stream;
  b->G = L.G;
  b->ws_off = L.ws_off;
  unsigned char* base = static_cast<unsigned char*>(ws);
  for (int i = 0; i < n_runs; ++i) {
    game_ctx* c = nullptr;
    const size_t next = i + 1 < n_runs ? L.ws_off[i + 1] : L.tab_off;
    const game_status s = game_init(&cfgs[i], X_devs[i], t_devs[i], base + L.ws_off[i],
                                    next - L.ws_off[i], stream, &c);
    if (s != GAME_OK) {
      game_batch_destroy(b);
      return s;
    }
    b->ctx.push_back(c);
  }
  b->druns = reinterpret_cast<FlowRun*>(base + L.runs_off);
  b->ctl = reinterpret_cast<FlowCtl*>(base + L.ctl_off);
  b->q = reinterpret_cast<FlowQueue*>(base + L.q_off);
  b->t_start = reinterpret_cast<uint64_t*>(base + L.ts_off);
  b->t_done = reinterpret_cast<uint64_t*>(base + L.td_off);
  game_status s = bdev(b, hipMemsetAsync(b->q, 0, sizeof(FlowQueue), b->stream), "batch init");
  if (s == GAME_OK) {
    bool fixed = true;
    for (int i = 0; i < n_runs; ++i) fixed = fixed && cfgs[i].tile_p > 0 && cfgs[i].row_groups > 0;
    if (fixed) {
      std::vector<int> tp(n_runs), rg(n_runs);
      for (int i = 0; i < n_runs; ++i) {
        tp[i] = cfgs[i].tile_p;
        rg[i] = cfgs[i].row_groups;
      }
      s = batch_apply(b, tp, rg);
    } else {
      s = batch_tune(b);
    }
  }
  if (s != GAME_OK) {
    game_batch_destroy(b);
    return s;
  }
  *out = b;
  return GAME_OK;
}

game_status game_batch_tiles(game_batch* b, int32_t* tile_p, int32_t* row_groups) {
  GAME_TRY(check_batch(b));
  for (int i = 0; i < b->n; ++i) {
    if (tile_p) tile_p[i] = b->tile_p[i];
    if (row_groups) row_groups[i] = b->row_groups[i];
  }
  return GAME_OK;
}

game_status game_batch_context(game_batch* b, int32_t i, game_ctx** out) {
  GAME_TRY(check_batch(b));
  if (!out || i < 0 || i >= b->n) return fail(GAME_E_INVALID, "run index out of range");
  *out = b->ctx[i];
  return GAME_OK;
}

game_status game_batch_time_fitness(game_batch* b, int32_t reps, float* ms) {
  GAME_TRY(check_batch(b));
  if (!ms || reps < 1) return fail(GAME_E_INVALID, "reps must be >= 1 and ms non-NULL");
  return batch_time(b, reps, ms);
}

game_status game_batch_run(game_batch* b, game_result* results, double* latency_us) {
  GAME_TRY(check_batch(b));
  if (!results) return fail(GAME_E_INVALID, "results is NULL");
  std::vector<game_state> s0(b->n);
  for (int i = 0; i < b->n; ++i) {
    game_ctx* c = b->ctx[i];
    if (!c->tile_fresh) GAME_TRY(enqueue_pack_population(c, b->stream));
    GAME_TRY(game_get_state(c, &s0[i], nullptr));
    GAME_TRY(dev(c, launch_run_arm(c->state, c->cfg.max_generations, c->cfg.mse_threshold, b->stream), "arm"));
  }
  // each launch breeds up to kFlowChunk generations of every run; the last
  // one finds every run stopped
  FlowQueue hq{};
  const int launches = b->G / kFlowChunk + 2;
  for (int k = 0;; ++k) {
    if (k == launches) return fail(GAME_E_STATE, "batch did not reach its stop conditions");
    GAME_TRY(batch_launch(b, kFlowChunk, k == 0, 0, &hq));
    if (hq.running == 0) break;
  }
  std::vector<uint64_t> ts, td;
  int dev_id = 0, rate_khz = 0;
  if (latency_us) {
    ts.resize((size_t)b->G * b->n);
    td.resize((size_t)b->G * b->n);
    GAME_TRY(bdev(b, hipMemcpyAsync(ts.data(), b->t_start, ts.size() * 8, hipMemcpyDeviceToHost, b->stream), "stamps"));
    GAME_TRY(bdev(b, hipMemcpyAsync(td.data(), b->t_done, td.size() * 8, hipMemcpyDeviceToHost, b->stream), "stamps"));
    GAME_TRY(bdev(b, hipStreamSynchronize(b->stream), "synchronize"));
    GAME_TRY(bdev(b, hipGetDevice(&dev_id), "device"));
    GAME_TRY(bdev(b, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev_id), "clock rate"));
  }
  for (int i = 0; i < b->n; ++i) {
    game_ctx* c = b->ctx[i];
    GAME_TRY(dev(c, launch_run_disarm(c->state, b->stream), "disarm"));
    game_state s;
    GAME_TRY(game_get_state(c, &s, results[i].best_genes));
    results[i].best_mse = s.best_mse;
    results[i].best_fitness = s.best_fitness;
    results[i].best_miscls = s.best_miscls;
    results[i].generations = s.generation - s0[i].generation + 1;
    results[i].stop_reason = s.stop_reason;
    c->have_eval = true;
    c->tile_fresh = true;
    c->evaluated = true;
    if (latency_us) {
      // generation g of run i: from the opening of its fitness phase to the
      // end of its breed (bred generations only)
      for (int g = 0; g < b->G; ++g) {
        double v = -1.0;
        const uint64_t a = ts[(size_t)i * b->G + g], e = td[(size_t)i * b->G + g];
        if (g + 1 < results[i].generations && e > a && rate_khz > 0) v = (double)(e - a) * 1e3 / rate_khz;
        latency_us[(size_t)i * b->G + g] = v;
      }
    }
  }
  return GAME_OK;
}

game_status game_run_batched(const game_config* cfgs, int32_t n_runs, const void* const* X_devs,
                             const void* const* t_devs, void* ws, size_t ws_bytes, void* stream,
                             game_result* results, double* latency_us) {
  game_batch* b = nullptr;
  GAME_TRY(game_batch_init(cfgs, n_runs, X_devs, t_devs, ws, ws_bytes, stream, &b));
  const game_status s = game_batch_run(b, results, latency_us);
  game_batch_destroy(b);
  return s;
}

}  // extern "C"

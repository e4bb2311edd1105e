// Internal declarations of libgame: device helpers, workspace plan, launchers.
// Not part of the public ABI (that is include/game.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "game.h"

namespace game {

// ---------------------------------------------------------------- constants
constexpr int kMaxElite = 64;      // elitism limit (top-E ranking in one workgroup)
constexpr int kMaxTournament = 16; // tournament draws addressable by the counter layout
constexpr int kMaxGenes = 4096;    // L limit (keeps every index well inside int32)
constexpr int kMaxRescore = 8;     // chromosomes one float32 re-score launch handles

// Philox stream tags: the fourth counter word of every draw.
enum : uint32_t {
  kTagInit = 1,
  kTagSel = 2,
  kTagMut = 3,
  kTagMut1 = 4,
  kTagMut2 = 5,
  kTagMut3 = 6,
  kTagMlpInit = 7,
  kTagMinibatch = 8,
  kTagAudit = 9,
  kTagPrescreen = 10,
  kTagRoulette = 11,
  kTagImmigrant = 12,
};

// ------------------------------------------------- Philox4x32-10 (device)
// Salmon et al., SC'11: ten rounds; each multiplies counter words 0 and 2 by
// the two round multipliers, exchanges high/low product halves across the
// counter and xors in the key; the key advances by the two Weyl increments
// between rounds.
struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint32_t hi0 = __umulhi(m0, c0), lo0 = m0 * c0;
    const uint32_t hi1 = __umulhi(m1, c2), lo1 = m1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t word_of(const u32x4& b, int i) {
  return i == 0 ? b.x : i == 1 ? b.y : i == 2 ? b.z : b.w;
}

// ---------------------------------------------------------- device state
// Lives in the workspace; read and written only by kernels (and copied out
// by game_get_state).
struct DevState {
  int32_t generation;      // generations completed (keys the GA draws)
  int32_t stopped;         // a run's stop condition held
  int32_t best_index;      // best chromosome of the last ranking
  int32_t stop_reason;
  int32_t run_active;      // kernels honour `stopped` only while a run is active
  int32_t end_generation;  // run stops after evaluating generation end_generation-1
  int32_t have_best;
  int32_t pad;
  double best_mse, best_fitness, best_miscls;
  double mse_threshold;
};

// Kernels that may be skipped once a run stopped test this.
__device__ __forceinline__ bool run_halted(const DevState* s) {
  return s != nullptr && s->run_active && s->stopped;
}

// Tail of the fitness kernels: the last workgroup of each chromosome tile
// reduces that tile's partial sums (fixed order) into mse / miscls / fitness;
// for a population evaluation the last tile to finish also ranks the
// population and tracks the best chromosome.
struct FitTail {
  uint32_t* counters;   // [n_pt_cap + 1], zero between launches
  int n_pt_cap;         // index of the "tiles done" counter
  int P;                // chromosomes evaluated
  double invN;
  double *mse, *miscls, *fit;     // internal results or null
  double *mse2, *miscls2, *fit2;  // caller results or null
  int n_top;            // > 0: rank the population (top n_top)
  int track;            // with n_top: track the best chromosome and test the stop rule
  int* top;
  DevState* st;
  const float* pop0;    // population buffers; generation g lives in pop[g & 1]
  const float* pop1;
  int L;
  float* best;
};

// ----------------------------------------------------------- plan
struct Plan {
  int K, M, L, M_pad, P, n_off, E, P_max, k;
  int64_t N, N_pad;
  int tile_n, tile_p;          // fitness workgroup tile (rows x chromosomes)
  bool lds;                    // LDS-staged fitness kernel (else the streaming one)
  int row_groups;              // fixed row ranges of the fitness sums (0: automatic)
  int64_t n_rt;                // row tiles
  int P_max_pad;               // P_max rounded up to tile_p
  int rt_per_wg_max;           // bounds the partial buffer
  int64_t n_rg_max;            // row groups at rt_per_wg_max... (partials rows)
  size_t elt;                  // bytes per Phi / tile element
  size_t acc;                  // bytes per t / bias element (8 for F64 else 4)
  // workspace offsets
  int n_pt_cap;                // chromosome tiles at P_max
  int n_counters;              // arrival counters: tiles, tiles done, breed, re-score
  size_t off_phi, off_t, off_tile, off_bias, off_pop0, off_pop1, off_psse, off_pmiss;
  size_t off_mse, off_miscls, off_fit, off_elite, off_state, off_best, off_cnt;
  size_t off_x, off_rpart;          // float32 patterns and re-score partials (16-bit forms)
  size_t off_wheel;                 // selection wheel / ranking (P_max x 8 bytes)
  size_t off_mpart;                 // metric partials and result
  // offspring form (n_offspring != P - E, or a prescreen)
  bool offspring;
  int k_sel, audit, P_eval, sur, H, cap, steps, batch, n_recent, rows_max;
  int64_t mlp_scratch;         // floats of MLP activation scratch
  size_t off_O, off_keys, off_sel, off_aud, off_surv, off_evg, off_emse, off_emis, off_efit;
  size_t off_snap, off_yhat, off_rho, off_loss, off_prm, off_am, off_av, off_step;
  size_t off_rank, off_WT, off_mscr, off_buf, off_bufy, off_sst, off_log;
  size_t total;
};
constexpr int kLogCap = 4096;  // generations of surrogate statistics kept

game_status make_plan(const game_config* cfg, Plan* p, char* err, size_t errlen);

// ----------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.
hipError_t launch_basis(const game_config* cfg, const void* X, int64_t rows_in, int64_t rows_out,
                        void* phi, int64_t ld, hipStream_t s);

hipError_t launch_copy_targets(int dtype, const void* t, int64_t N, int64_t N_pad, void* tvec,
                               hipStream_t s);

// genes = (sel && sel->generation is odd) ? genes1 : genes0
hipError_t launch_pack(int dtype, const float* genes0, const float* genes1, const DevState* sel,
                       int P, int L, int M, int bias, int M_pad, int P_pad, void* tile, void* biasv,
                       hipStream_t s);

struct FitnessGeom {
  int n_pt;        // chromosome tiles
  int rt_per_wg;   // row tiles per workgroup
  int64_t n_rg;    // row groups (= partial rows)
  int64_t n_items; // workgroups doing work
  int64_t grid;    // launched workgroups (multiple of 8)
  int ub;          // LDS kernels: 32-row units per range boundary block (1 or 4)
};
// Workgroups of the persistent (LDS) fitness kernel resident at once, or 0
// when the configuration uses the non-persistent kernel.
int fitness_persistent_slots(const Plan& p, int task, int dtype);
// LDS-staged kernel: does a tile of tp chromosomes fit, and its dynamic LDS
int fitness_lds_fits(int dtype, int M_pad, int tp);
// Range boundary block (1 or 4 units of 32 rows) for n_rg row ranges of N
// patterns and n_pt chromosome tiles, given the resident workgroup count.
int fitness_range_block(int64_t N, int64_t n_rg, int n_pt, int slots);
size_t fitness_lds_bytes(int dtype, int M_pad, int tp);
int fitness_lds_stride(int dtype, int M_pad);  // LDS words per staged gene row
FitnessGeom fitness_geometry(const Plan& p, int task, int dtype, int P_eval);

hipError_t launch_fitness(const Plan& p, int task, int dtype, const FitnessGeom& g, const void* phi,
                          const void* tile, const void* biasv, const void* tvec, double* psse,
                          uint32_t* pmiss, const DevState* st, const FitTail& tail,
                          hipStream_t s);

hipError_t launch_init_population(float* pop, int P, int L, uint64_t seed, hipStream_t s);

hipError_t launch_rank(const double* fit, int P, int n_top, int* top_idx, const DevState* st,
                       hipStream_t s);

// One generation of the genetic operators: reads pop[g & 1], writes
// pop[(g + 1) & 1] and the gene tile (+ bias), then advances the generation.
struct BreedArgs {
  float* pop0;
  float* pop1;
  const double* fit;
  const int* elite;
  int P, L, E, n_children, k;
  uint64_t thr_c, thr_m;
  float sigma;
  uint32_t k0, k1;
  void* tile;
  void* biasv;
  int M, M_pad, bias;
  uint32_t* counter;  // zero between launches
  float* out;         // offspring form: children go here (no tile, no advance)
  int sel;            // game_selection
  const uint64_t* wheel;  // ROULETTE: cumulative integer weights (P)
  const int* order;       // RANKING: chromosome of each rank (P)
  int n_imm;          // the last n_imm children are random immigrants
};
// Per-generation input of the wheel selections: the cumulative roulette
// weights (ROULETTE) or the full ranking (RANKING) of fit[0..P); no-op for
// tournaments.
hipError_t launch_select_prep(int sel, const double* fit, int P, uint64_t* wheel, int* order,
                              const DevState* st, hipStream_t s);
hipError_t select_prepare(int sel);  // once per selection kind, outside graph capture
hipError_t launch_breed(int dtype, const BreedArgs& a, DevState* st, hipStream_t s);

// Population copies in and out of pop[g & 1] (dir 0: out to dst, 1: in from src).
hipError_t launch_pop_copy(float* pop0, float* pop1, const DevState* st, float* ext, int64_t n,
                           int dir, hipStream_t s);

int rescore_grid();
// The allocation-free re-score's scratch on the current device (block
// partials and arrival counter; set up on the first call per device).
size_t rescore_scratch_bytes();
hipError_t rescore_scratch(hipStream_t s, double** part, uint32_t** counter);
hipError_t launch_rescore(const float* X, const float* t, int64_t N, int F, int D, int K, int basis,
                          int M, int L, int bias, int task, const float* genes, int n,
                          const float* pop0, const float* pop1, const int* top, double* part,
                          uint32_t* counter, double* mse, double* miscls, const DevState* sel,
                          DevState* st, float* best, hipStream_t s);

// ------------------------------------------------------ offspring form
struct SurState {  // replay ring buffer, target statistics, log position
  int32_t head, count;
  float mu, sigma;
  int32_t n_logged;
  int32_t last;  // rows the latest append stored (they end at head - 1)
};
// rank_ws: sur_rank_ints(n) ints of per-slice rank counts (shared by the
// selections and statistics of one stream)
int64_t sur_rank_ints(int n);
hipError_t sur_keys(int mode, const float* fsrc, const double* dsrc, int n, uint32_t tag,
                    const DevState* st, uint64_t seed, uint64_t* keys, hipStream_t s);
hipError_t sur_select(const uint64_t* keys, int n, int k, int* out, int* rank_ws, const DevState* st,
                      hipStream_t s);
hipError_t sur_spearman(const float* x, const int* xi, const double* y, int n, float* out, int* rank_ws,
                        const DevState* st, hipStream_t s);
hipError_t sur_gather(const float* src, const int* idx, int n, int L, float* dst, const DevState* st,
                      hipStream_t s);
hipError_t sur_append(const float* genes, const double* mse, int n, int L, float* buf, float* buf_y,
                      int cap, SurState* ss, const DevState* st, hipStream_t s);
hipError_t sur_snapshot(const int* elite, int E, const double* fit, const double* mse,
                        const double* miscls, double* snap, const DevState* st, hipStream_t s);
hipError_t sur_merge(float* pop0, float* pop1, const int* elite, const double* snap, int E,
                     const float* cand, const int* surv, const double* cfit, const double* cmse,
                     const double* cmis, int P, int L, double* fit, double* mse, double* miscls,
                     const DevState* st, hipStream_t s);
hipError_t sur_rank_track(const double* fit, const double* mse, const double* miscls, int P, int n_top,
                          int* top, const float* pop0, const float* pop1, int L, float* best,
                          DevState* st, int advance, hipStream_t s);
hipError_t sur_log(const float* rho, const float* loss, float* log, int cap, SurState* ss,
                   const DevState* st, hipStream_t s);

// ------------------------------------------------------ surrogate MLP
struct MlpDims {
  int L, H1, H2;
};
struct MlpLayout {  // offsets into the flat parameter array
  int64_t W1, b1, W2, b2, w3, b3, total;
};
MlpLayout mlp_layout(int L, int H1, int H2);
// activation scratch (floats) for training steps of `batch` rows and forward
// passes of up to `rows_max` rows
int64_t mlp_scratch_floats(const MlpDims& d, int batch, int rows_max);
// Zero the gradient products' arrival counters in the scratch (once per context).
hipError_t mlp_scratch_init(const MlpDims& d, float* scratch, hipStream_t s);
// W2T: transposed copy of W2 (H1 x H2), kept in step with the parameters
hipError_t mlp_transpose(const MlpDims& d, const float* params, float* W2T, hipStream_t s);
hipError_t mlp_init(const MlpDims& d, float* params, float* m, float* v, float* W2T, uint64_t seed,
                    hipStream_t s);
// halt: kernels return at once once a run has stopped (may be null)
hipError_t mlp_forward(const MlpDims& d, const float* params, const float* W2T, const float* X, int B,
                       float* y, float* scratch, const DevState* halt, hipStream_t s);
hipError_t mlp_grads(const MlpDims& d, const float* params, const float* W2T, const float* X,
                     const float* target, int B, float* scratch, float* grads, float* loss,
                     const DevState* halt, hipStream_t s);
// one Adam step on a minibatch drawn from the replay ring (step[0]: steps
// taken, step[1]: arrival counter, zero between launches)
hipError_t mlp_train_step(const MlpDims& d, float* params, float* W2T, float* m, float* v,
                          int32_t* step, float lr, const float* buf, const float* bufy,
                          const SurState* ss, uint64_t seed, int B, int n_recent, int cap,
                          float* scratch, float* loss, const DevState* halt, hipStream_t s);
hipError_t mlp_adam(const MlpDims& d, float* params, float* W2T, const float* grads, float* m, float* v,
                    int32_t* step, float lr, const DevState* halt, hipStream_t s);

// ------------------------------------------------------ test / validation use
struct PredictArgs {
  const void* X;       // n x F patterns (double for F64, else float)
  const void* t;       // n targets (metrics)
  int64_t n;
  int F, D, K, basis, M, L, bias, task;
  const float* genes;  // one chromosome, L floats
  void* out;           // n outputs (prediction), same type as X
  double* part;        // kPredictParts x 5 metric partials
};
constexpr int kPredictParts = 1024;
hipError_t launch_predict(bool f64, const PredictArgs& a, hipStream_t s);
// result (device): {sum of squared errors, TP, FP, TN, FN}
hipError_t launch_metrics(bool f64, const PredictArgs& a, double* result, hipStream_t s);

// ------------------------------------------------------ batched form
// One run's entry in the batched scheduler's table (written by the host
// before a launch, read-only during it).  Phases per generation: fitness
// (n_fit items), the wheel or ranking (wheel selections), the breed
// (n_breed items).
struct FlowRun {
  const void* phi;
  const void* tile;
  const void* biasv;  // null without the bias gene
  const void* tvec;
  double* psse;
  uint32_t* pmiss;
  DevState* st;
  FitTail tail;
  BreedArgs breed;    // counter and out null: the scheduler advances the generation
  uint64_t* wheel;    // roulette wheel, or the ranking as int
  uint64_t* t_start;  // per generation of a batch run: its fitness phase opened
  uint64_t* t_done;   //   and its breed finished (wall clock)
  uint64_t span;      // wall-clock ticks a generation of the run would take with
                      // 1/n of the device (its fair share: deadline = opening + span)
  int64_t N;
  int M_pad, ldsw, n_pt, n_ranges, part_ld, task, tile_p, ub;
  int n_fit, n_breed, sel, rank_pow2, t_cap, pad;
};
constexpr int kXcds = 8;  // XCDs of the device (workgroup b runs on XCD b % 8)
struct FlowCtl {      // per run; read and written only at device scope
  uint64_t word;      // phase epoch << 32 | items claimed (wheel and breed phases)
  uint64_t xw[kXcds]; // fitness phase: epoch << 32 | items claimed in XCD slice x
  uint64_t deadline;  // of the run's current generation (wall clock)
  uint32_t done;      // items finished in the epoch
  int32_t gen;        // the run's generation
  int32_t rel;        // generations bred since the batch run began
  int32_t left;       // generations this launch may still breed
};
struct FlowQueue {
  uint32_t active;    // runs with work left in the launch
  uint32_t error;     // a workgroup found no open item for too long
  uint32_t running;   // runs not stopped after the launch
  uint32_t pad;
};
// Workgroups of the scheduler that are resident at once with `lds` bytes of
// dynamic LDS (0: cannot run).
int flow_slots(int dtype, size_t lds);
// arm (first: a batch run begins) -> scheduler -> status; chunk: generations
// each run may breed in this launch; eval_only: the fitness phase only.
hipError_t launch_flow(int dtype, const FlowRun* runs, int n_runs, FlowCtl* ctl, FlowQueue* q,
                       int grid, size_t lds, int chunk, int first, int eval_only, uint64_t idle_ticks,
                       hipStream_t s);
// a context's workgroups in a breed launch
int breed_blocks(const BreedArgs& a);

hipError_t launch_state_init(DevState* st, uint32_t* counters, int n_counters, hipStream_t s);
hipError_t launch_run_arm(DevState* st, int max_generations, double threshold, hipStream_t s);
hipError_t launch_run_disarm(DevState* st, hipStream_t s);

}  // namespace game

/*
 * vopp.h -- C ABI of the MI355X planner for Vectorized Online POMDP Planning
 * (VOPP: Hoerger, Sudrajat, Kurniawati).
 *
 * One call of vopp_plan() is one planning step of Alg. 1: K iterations, each
 * sampling n_p root states from the belief particles, running the
 * level-by-level forward search of Alg. 2 (softmax action draw of Eq. 6,
 * generative model G, AppendActions, FilterTerminals, AppendBeliefs) to the
 * iteration's depth, and the bottom-up preference backup of Alg. 3 (Q = C/N +
 * gamma W, Psi <- Psi - L_eta Psi + Q from Eq. 5, V = L_eta Psi from Eq. 3);
 * then the root action with the largest preference.  The tree holds the
 * tensors of Sec. III-C (belief rows, action-node rows, preference rows) in
 * HBM as one array per belief field, indexed by belief id: the preference
 * row, the visit counts, reward sums and child-value sums of the belief's
 * action nodes, and its value, visit count and parent.
 *
 * Conventions for every entry point:
 *   - Every function returns a vopp_status; nothing throws across the ABI.
 *     On failure vopp_last_error() returns a message (per thread, valid until
 *     the next call on that thread).
 *   - "host" pointers are read during the call and not retained; "device"
 *     pointers must point to memory of the current HIP device.
 *   - Inputs are validated before any device work.  HIP failures map to
 *     VOPP_E_DEVICE.  Handles are not thread-safe: use one stream per handle.
 *   - Random numbers are Philox4x32-10 streams keyed by the 64-bit seed with
 *     counter (episode, tag<<24 | level, iteration, real step), so the same
 *     inputs give the same tree on every run and in every batch.
 */
#ifndef VOPP_H
#define VOPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VOPP_OK = 0,
  VOPP_E_INVALID = -1,   /* bad argument; nothing was launched            */
  VOPP_E_NOMEM = -2,     /* footprint exceeds free HBM or a given budget  */
  VOPP_E_DEVICE = -3,    /* a HIP call failed                             */
  VOPP_E_BUSY = -4,      /* server: no slot or memory free right now      */
  VOPP_E_INTERNAL = -5   /* an internal consistency check failed          */
} vopp_status;

/* Message of the last failed call on this thread ("" if none). */
const char* vopp_last_error(void);

/* Library version string. */
const char* vopp_version(void);

/* ------------------------------------------------------------------------ */
/* POMDP models: the generative model G(s, a) -> (s', o, r) of Sec. III-B.   */
/* ------------------------------------------------------------------------ */

typedef struct vopp_pomdp vopp_pomdp;

/* Tabular POMDP <S, A, O, T, Z, R, gamma> (Sec. II-A).  All pointers are host
 * pointers, copied to the device at creation; the handle owns the copy.
 *   rowptr [nS*nA+1], col/tprob [rowptr[nS*nA]]: transition rows T(s, a, .) in
 *     CSR form, row index s*nA + a; probabilities fp32, non-negative, each row
 *     summing to 1 within 1e-5.
 *   zprob [nS*nA*nO]: observation rows Z(s', a, .) indexed [s'][a][o].
 *   reward [nS*nA]: R(s, a).   heur [nS] or NULL: leaf value heuristic.
 * Limits: 1 <= nA <= 4096, 1 <= nS < 2^31, 0 < gamma < 1, and 1 <= nO <=
 * 2^(26 - b) with b = max(6, ceil(log2 nA)) (belief keys hold the action and
 * observation in 26 bits): nO <= 2^20 up to 64 actions, 2^16 for 625, 2^14
 * for 3025.  Models with more than 64 actions keep preference rows in memory
 * (one wavefront per belief in the backup sweeps, half a wavefront per
 * episode in the forward search); batched and served plans take at most 16
 * actions.
 * Sampling uses integer thresholds rint(cum/total * 2^31) per row. */
typedef struct {
  int32_t nS, nA, nO;
  const int32_t* rowptr;
  const int32_t* col;
  const float* tprob;
  const float* zprob;
  const float* reward;
  const float* heur;
  double gamma;
} vopp_tabular_desc;

/* Continuous 2-D navigation POMDP (continuous spaces represented by a fixed
 * finite set chosen a priori, Sec. III-B): state (x, y) fp32 in [lo, hi]^2;
 * actions 0..3 move by +y, +x, -y, -x of length `step` with N(0, sigma_move^2)
 * noise per axis; observation = next position + N(0, sd^2) noise per axis with
 * sd = sigma_obs0 + sigma_obs_slope*|x' - obs_center_x|, keyed by its grid
 * cell floor(v*inv_bin) clamped to [key_lo, key_lo+key_n-1] per axis
 * (1 <= key_n <= 1024, key = cell_x * key_n + cell_y); reward
 * r_step, plus r_goal inside the goal disk (terminal), plus r_hit inside any
 * obstacle disk.  Noise comes from `gauss`, a host table of 4096 standard
 * normal quantiles indexed by 12 random bits.  disks [2*n_disks] holds the
 * centres.  heuristic: 0 = zero leaf value, 1 = -(|x-goal_x| + |y-goal_y|).
 * All arithmetic is single precision without contraction. */
typedef struct {
  float lo, hi, step, sigma_move, sigma_obs0, sigma_obs_slope, obs_center_x,
      inv_bin;
  int32_t key_lo, key_n;
  float goal_x, goal_y, goal_r2, disk_r2, r_step, r_goal, r_hit;
  int32_t heuristic;
  int32_t n_disks;
  const float* disks;
  const float* gauss;
  double gamma;
} vopp_nav2d_desc;

vopp_status vopp_pomdp_tabular(const vopp_tabular_desc* desc, vopp_pomdp** out);
vopp_status vopp_pomdp_nav2d(const vopp_nav2d_desc* desc, vopp_pomdp** out);
/* Number of actions |A| of a model (0 for NULL). */
int32_t vopp_pomdp_num_actions(const vopp_pomdp* pomdp);
/* Reference policy pi0 of the KL-regularised objective (Sec. III-A, Eq. 4): every
 * belief's preference row starts at ln pi0(a) / eta instead of the uniform
 * -ln|A| / eta, so the first softmax draws at a new belief follow pi0 and the
 * values are the pi0-weighted soft maxima.
 *   pi0  host array of |A| weights, each finite and > 0; they are normalised
 *        by their sum (a plain double sum in index order).  NULL restores the
 *        uniform policy.
 * Copied synchronously to the model's device memory; the model must live on
 * the current device.  Plans already enqueued may see either policy: do not
 * call it while a plan with this model is in flight.
 * Returns VOPP_E_INVALID (null model, bad entry, wrong device) with the model
 * unchanged, or VOPP_E_DEVICE. */
vopp_status vopp_pomdp_set_reference_policy(vopp_pomdp* pomdp, const double* pi0);
void vopp_pomdp_free(vopp_pomdp* pomdp);

/* ------------------------------------------------------------------------ */
/* Planning (Alg. 1-3).                                                      */
/* ------------------------------------------------------------------------ */

enum { VOPP_SCHEDULE_DEEPEN = 0, VOPP_SCHEDULE_FIXED = 1 };

/* n_particles: episodes per iteration (n_p of Alg. 1), 1 .. 2^24.
 * eta: the multiplier of the preferences in the softmax (Eq. 3, 6), > 0.
 * schedule: DEEPEN grows the search depth as D_k = min(k, depth) (D_max of
 *   Alg. 1 starts at 1 and grows by one per iteration); FIXED uses depth.
 * seed: Philox key.  step: real step index t (a counter word). */
typedef struct {
  int32_t n_particles;
  int32_t schedule;
  double eta;
  uint64_t seed;
  uint32_t step;
} vopp_params;

/* near_ties: action draws (Eq. 6) whose position t = u * P_last lies within
 * 2^-16 * P_last of a neighbouring boundary P_j of the running sums, in the
 * kernel's own arithmetic.  It counts draws from rows that a backup has
 * updated (the root from the second iteration on, rows of a belief whose
 * entries are not all equal); draws from the initial row are exact and
 * do not count.  A planner that keeps its preferences in another precision
 * may decide such a draw the other way. */
typedef struct {
  int64_t particle_steps;   /* generative-model calls made by the plan     */
  int64_t n_beliefs;        /* beliefs of the tree (root included)         */
  int64_t n_actions;        /* action nodes (b, a) visited at least once   */
  double device_ms;         /* device time of the plan, HIP events          */
  int64_t near_ties;        /* near-tie action draws (see above)           */
  /* Work of the depth sweeps of the backup (Alg. 3, the loop over d = D..2,
   * summed over every iteration; the leaf sweep is not included): belief
   * visits, the visits of beliefs with at least one action node (those
   * update their preference row), and action-node visits. */
  int64_t sweep_visits;
  int64_t sweep_internal;
  int64_t sweep_nodes;
  /* Inserts of new beliefs in the forward search whose slot another key
   * took first, so that the episode probed for its key again (its next
   * level's key formed again).  A count of insert races, not an error. */
  int64_t insert_reprobes;
} vopp_stats;

/* A workspace holds one plan's tree and per-episode trace in HBM, sized for
 * the worst case (beliefs <= 1 + n_p * sum_k D_k <= 2^28), so no plan can
 * overflow it.  Each belief owns a record of 24*ra + 32 bytes rounded up to a
 * multiple of 128 (ra = |A| rounded up to a multiple of 4), stored by level
 * step, and a 16-byte slot of an open-addressing table of
 * 2^ceil(log2(2*(1 + n_p*sum_k D_k))) slots (load <= 1/2). */
typedef struct vopp_workspace vopp_workspace;

/* Bytes of device memory a workspace for (pomdp, params, budget, depth) needs. */
size_t vopp_plan_footprint(const vopp_pomdp* pomdp, const vopp_params* params,
                           int32_t budget, int32_t depth);

vopp_status vopp_workspace_create(const vopp_pomdp* pomdp,
                                  const vopp_params* params, int32_t budget,
                                  int32_t depth, vopp_workspace** out);
void vopp_workspace_free(vopp_workspace* ws);

/* One planning step.
 *   pomdp: the model.  belief_particles: DEVICE pointer to n_belief particles
 *     (tabular: int32 states [n_belief]; navigation: fp32 x[n_belief] followed
 *     by fp32 y[n_belief]).  Root states are drawn with replacement, index =
 *     (x0 * n_belief) >> 32.
 *   budget: iterations K >= 1.  depth: maximum leaf depth, 1 .. 64.
 *   ws: a workspace created for at least these sizes, or NULL to use one
 *     owned by the pomdp handle (grown on demand).
 *   stream: hipStream_t (NULL = default stream).
 *   action (host, out): argmax_a Psi(root, a), lowest index on ties.
 *   values (host, out, may be NULL): the root preferences Psi(root, .) [nA],
 *     kept in double precision.  v_root (host, may be NULL): L_eta Psi(root).
 *   stats (host, may be NULL).
 * The call returns after the result has reached the host. */
vopp_status vopp_plan(const vopp_pomdp* pomdp, const void* belief_particles,
                      int32_t n_belief, int32_t budget, int32_t depth,
                      const vopp_params* params, vopp_workspace* ws,
                      void* stream, int32_t* action, double* values,
                      double* v_root, vopp_stats* stats);

/* vopp_plan that also exports every action draw of the forward search
 * (Alg. 2, one draw per live episode per level), for parity checks and
 * debugging.  draw_act and draw_obs are DEVICE arrays of trace_len entries,
 * at least n_steps * n_particles with n_steps = D_1 + ... + D_K (a re-rooted
 * plan's kept steps not counted).  Entry t * n_particles + ep, for level step
 * t = D_1 + ... + D_{k-1} + d (level d of iteration k) and episode ep, gets
 * the action the episode drew there and the observation key G returned for
 * it (also on the step that terminated it), or -1 in both once the episode
 * has terminated.  force_act (DEVICE, may be NULL), same indexing: an entry
 * in [0, nA) replaces the kernel's decision at that draw by that action; any
 * other entry (-1) leaves it.  draw_act always receives the kernel's own decision.
 * This is a test hook: a parity check forces the draws that a reference
 * planner in another precision reports as near ties to that planner's
 * decision, so the rest of the two trees can be compared bit for bit.
 * Other arguments and outputs as for vopp_plan; the export adds two stores
 * (and the force one load) per draw.  VOPP_E_INVALID for null output arrays
 * or a short trace_len. */
vopp_status vopp_plan_trace(const vopp_pomdp* pomdp, const void* belief_particles,
                            int32_t n_belief, int32_t budget, int32_t depth,
                            const vopp_params* params, vopp_workspace* ws, void* stream,
                            int32_t* action, double* values, double* v_root,
                            vopp_stats* stats, int16_t* draw_act, int32_t* draw_obs,
                            const int16_t* force_act, int64_t trace_len);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): vopp_plan
 * without a workspace.  The tree lives in a static device array of
 * VOPP_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends; the call allocates nothing (no hipMalloc, no pinned host
 * memory, no events) and copies nothing from or to the host, so it can be
 * captured in a graph.  It only enqueues the plan on `stream` and returns.
 *   pomdp, belief_particles (DEVICE), n_belief, budget, depth, params: as
 *     for vopp_plan; the plan's vopp_plan_footprint must not exceed
 *     VOPP_NOALLOC_SCRATCH_BYTES, else VOPP_E_INVALID before any launch.
 *   result (DEVICE, out): nA + 10 doubles, written when the stream reaches
 *     the end of the plan: [0] action, [1 .. nA] root preferences, [nA+1]
 *     V(root), [nA+2] particle steps, [nA+3] beliefs, [nA+4] action nodes,
 *     [nA+5] error flags (1: a belief particle outside [0, nS); 2: internal
 *     table overflow; 0 on success), [nA+6] near-tie draws, [nA+7 .. nA+9]
 *     the sweep counts of vopp_stats.
 * The result equals vopp_plan's bit for bit.  Every call on one GPU uses
 * that GPU's one array: calls that overlap on one GPU (other streams or
 * threads) race and give undefined results; calls in stream order do not.
 * Every plan clears what it reads of the array first. */
#define VOPP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vopp_status vopp_plan_noalloc(const vopp_pomdp* pomdp, const void* belief_particles,
                              int32_t n_belief, int32_t budget, int32_t depth,
                              const vopp_params* params, void* stream, double* result);

/* Anytime planning step: Alg. 1 with its wall-clock budget.  Iterations run
 * while the planning time is not used up: after each iteration the device
 * compares its wall clock with the start of the plan's first kernel, and the
 * next iteration runs only if less than time_ms has passed, so the plan ends
 * at most one iteration after the budget.  At least one and at most
 * max_budget iterations run.
 *   max_budget: the cap K (sizes the workspace like vopp_plan's budget).
 *   time_ms: the planning time, > 0 milliseconds of device time.
 *   iterations (host, out, may be NULL): the number K' of iterations run.
 * Other arguments and outputs as for vopp_plan.  The tree and result are
 * those of vopp_plan with budget K' (same draws, the same schedule D_k),
 * except that the fixed-point resolution of the sums is chosen for
 * max_budget, so values agree to that resolution.  The host enqueues
 * iterations at most two ahead of the device and stops once the device
 * reports the budget spent; kernels of iterations already enqueued then
 * return at once.  The workspace allocates a small pinned host word on its
 * first anytime plan.  The vopp_tree_dump and vopp_level_counts of the
 * workspace then describe the K'-iteration tree. */
vopp_status vopp_plan_anytime(const vopp_pomdp* pomdp, const void* belief_particles,
                              int32_t n_belief, int32_t max_budget, int32_t depth,
                              double time_ms, const vopp_params* params,
                              vopp_workspace* ws, void* stream, int32_t* action,
                              double* values, double* v_root, vopp_stats* stats,
                              int32_t* iterations);

/* Tree re-rooting between real steps (the outer loop of Alg. 1).  After the
 * plan in `src` chose an action, the environment executed `action` and
 * returned observation `obs`: the belief reached from the root by (action,
 * obs) becomes the root of the next plan, and its descendants are kept with
 * their statistics (preference rows, C, N, V, N_b), one level shallower.  The
 * paper's Alg. 1 starts every real step from a fresh tree; this keeps the
 * relevant subtree instead.
 *   src: a workspace whose last plan (vopp_plan or vopp_plan_anytime) holds
 *     the tree; it is only read.
 *   next, next_budget, next_depth: the parameters of the next plan, which
 *     runs in dst.  That plan must use next->n_particles and at most
 *     next_budget (<= 255) iterations.
 *   dst: receives the kept subtree; the next vopp_plan or vopp_plan_anytime
 *     on dst starts from it (its root preferences, visit counts and rewards
 *     included) instead of a fresh root.  dst is re-allocated (same handle)
 *     when it is too small for the subtree plus the next plan.  Its previous
 *     tree is discarded.
 *   kept (host, out, may be NULL): beliefs kept, the new root included; 0
 *     when the tree has no belief for (action, obs) -- dst then holds nothing
 *     and the next plan on it starts from a fresh root.
 * Kept beliefs are packed by depth into level steps ahead of the next plan's
 * own, and the next plan's sweeps visit them as every belief of their depth
 * (the backup of Alg. 3 covers the whole tree).  The call allocates and frees
 * temporary device memory (5 bytes per source belief slot) and synchronizes
 * the stream. */
vopp_status vopp_reroot(const vopp_pomdp* pomdp, vopp_workspace* src, int32_t action,
                        int32_t obs, const vopp_params* next, int32_t next_budget,
                        int32_t next_depth, vopp_workspace* dst, void* stream,
                        int64_t* kept);

/* Copy the tree of the last plan run in `ws` to host arrays (any may be
 * NULL).  Sizes come from vopp_stats.  Belief arrays [n_beliefs]: parent
 * action row (-1 for the root), observation key (-1 for the root), depth,
 * value V, visit count N_b; psi [n_beliefs*nA] (fp32; row 0 is the root,
 * whose double values are in vopp_plan's `values`).  Action arrays
 * [n_actions]: parent belief row, action, cumulative reward C, visits N.
 * Rows are in canonical order, which depends only on the tree: beliefs by
 * depth, then by (parent belief row, action, observation key); action nodes
 * by (parent belief row, action).  The root is belief row 0.  The dump
 * allocates temporary device memory and synchronizes the device. */
vopp_status vopp_tree_dump(vopp_workspace* ws, int32_t* b_parent, int32_t* b_obs,
                           int32_t* b_depth, float* psi, float* b_V,
                           int32_t* b_N, int32_t* a_parent, int32_t* a_act,
                           double* a_C, int32_t* a_N);

/* Beliefs created by each level step of the last plan run in `ws`.  Level
 * step t = D_1 + ... + D_{k-1} + d is level d of iteration k; it creates
 * beliefs of depth d + 1.  counts (host, out, may be NULL) receives the first
 * min(cap, n_steps) counts; n_steps (host, out) the number of level steps. */
vopp_status vopp_level_counts(const vopp_workspace* ws, int32_t* counts, int32_t cap,
                              int32_t* n_steps);

/* ------------------------------------------------------------------------ */
/* Between real steps: the true environment and the belief update.          */
/* ------------------------------------------------------------------------ */

/* One step of a simulated true environment (Alg. 1, "execute action a and
 * perceive o"): the generative model G with its own Philox stream, counter
 * (0, 4<<24, 0, step) under env_seed.  state: DEVICE pointer, in/out
 * (tabular: int32[1]; navigation: fp32 x, y).  obs, reward, terminal: host
 * outputs (any may be NULL).  Synchronous. */
vopp_status vopp_env_step(const vopp_pomdp* pomdp, void* state, int32_t action,
                          uint64_t env_seed, uint32_t step, void* stream,
                          int32_t* obs, float* reward, int32_t* terminal);

/* Sequential importance resampling belief update b <- tau(b, a, o) (Alg. 1,
 * belief update; SIR particle filter of Sec. III-B), in place on n DEVICE
 * particles (layout of vopp_plan's belief_particles).  Each particle moves
 * under a (transition part of G, Philox counter (i, 5<<24, 0, step)); its
 * weight is the exact integer likelihood of o (tabular: the observation
 * threshold difference; navigation: the count of noise indices per axis that
 * land in o's grid cell, multiplied); n new particles are drawn
 * multinomially (counter (j, 6<<24, 0, step)).  If every weight is zero the
 * moved particles are kept.  total_weight (host, may be NULL): the weight
 * sum (tabular in units of 2^-31, navigation in units of 2^-24).
 * Synchronous. */
vopp_status vopp_belief_update(const vopp_pomdp* pomdp, void* particles, int32_t n,
                               int32_t action, int32_t obs, uint64_t seed,
                               uint32_t step, void* stream, uint64_t* total_weight);

/* ------------------------------------------------------------------------ */
/* Batched planning: many independent instances (models of any kind, uneven */
/* n_p, budget and depth) advanced together.                                 */
/* ------------------------------------------------------------------------ */

/* One planning request: the arguments of vopp_plan.  belief_particles is a
 * DEVICE pointer in the layout vopp_plan documents. */
typedef struct {
  const vopp_pomdp* pomdp;
  const void* belief_particles;
  int32_t n_belief;
  int32_t budget;
  int32_t depth;
  vopp_params params;
} vopp_request;

#define VOPP_MAX_ACTIONS 64

/* Result of one request.  values[0 .. nA-1] are the root preferences. */
typedef struct {
  int32_t action;
  int32_t status;           /* vopp_status of this request */
  double v_root;
  int64_t particle_steps;
  int64_t n_beliefs;
  int64_t n_actions;
  double values[VOPP_MAX_ACTIONS];
} vopp_result;

/* Launch-shape knobs of a batch.  accum_cap: most tiles (blocks) of one
 * instance's accumulate sweep (a tile loops over its share of the trace);
 * backup_cap: most tiles of one backup sweep of one instance (both in the
 * per-phase launches).  The persistent launch sizes
 * its tiles by work instead: sweep_group chunks of 256 record positions (or
 * trace items, or table slots of the set-up) per sweep tile, forward_group
 * blocks of 256 episodes per forward tile (both >= 1), and runs blocks_per_cu
 * blocks per compute unit (0: as many as fit). */
typedef struct {
  int32_t accum_cap;
  int32_t backup_cap;
  int32_t blocks_per_cu;
  int32_t forward_group;
  int32_t sweep_group;
} vopp_tuning;

/* Modes of vopp_batch_run. */
enum {
  VOPP_BATCH_EAGER = 0,       /* per-phase launches issued one by one         */
  VOPP_BATCH_GRAPH = 1,       /* the per-phase launches as one hipGraph      */
  VOPP_BATCH_PERSISTENT = 2,  /* one persistent launch over a device queue   */
  VOPP_BATCH_AUTO = 3         /* the faster of GRAPH and PERSISTENT as the last
                                 vopp_batch_autotune measured it (PERSISTENT
                                 before any autotuning)                       */
};

typedef struct vopp_batch vopp_batch;

/* Create a batch of n requests: one workspace per request (owned by the
 * batch), and two ways to run it (Sec. III: the vectorised planner applied to
 * many instances at once):
 *   - the persistent launch: one kernel sized to the blocks the GPU holds at
 *     once, whose blocks take (instance, phase, tile) items from a device
 *     queue; each instance has its own phase counter, so every instance moves
 *     to its next phase as soon as its previous one is done; the queue reset
 *     and the kernel are captured in one hipGraph;
 *   - per-phase launches: launch g runs the g-th phase of every instance that
 *     has one, captured in a second hipGraph or issued eagerly.
 * All models must have |A| <= 16.  tuning may be NULL (defaults). */
vopp_status vopp_batch_create(const vopp_request* reqs, int32_t n,
                              const vopp_tuning* tuning, vopp_batch** out);
/* Bytes of device memory the batch's workspaces need. */
size_t vopp_batch_footprint(const vopp_request* reqs, int32_t n);
/* Replace request i's belief particles, seed and real step (same sizes). */
vopp_status vopp_batch_set_request(vopp_batch* b, int32_t i, const void* belief_particles,
                                   int32_t n_belief, uint64_t seed, uint32_t step);
/* Run every request once in the given mode (VOPP_BATCH_*; VOPP_E_INVALID
 * for another value).  The batch runs on its own stream, ordered after the
 * work already queued on `stream`.  results[n] (host, out); device_ms (host,
 * out, may be NULL): device time of the batch.  Every mode gives the same
 * results bit for bit. */
vopp_status vopp_batch_run(vopp_batch* b, void* stream, int32_t mode,
                           vopp_result* results, double* device_ms);
/* The autotuner (reps timed runs per shape, after one warm-up run): time the
 * persistent launch of this batch over its tile sizes (sweep_group in
 * {1, 2, 4, 8}, forward_group in {1, 4}) and blocks per CU (all that fit, or
 * one), then the per-phase graph over its block caps (accum_cap and
 * backup_cap 256 each, or the plain plan's caps); keep the fastest of each,
 * re-capture both graphs, report the tuning in chosen (may be NULL), and let
 * VOPP_BATCH_AUTO run the faster mode from then on.  Every tried shape must
 * give bit-identical results, else VOPP_E_INTERNAL. */
vopp_status vopp_batch_autotune(vopp_batch* b, void* stream, int32_t reps,
                                vopp_tuning* chosen);
/* Number of batched launches (phases of the longest instance). */
int32_t vopp_batch_num_launches(const vopp_batch* b);
/* The mode VOPP_BATCH_AUTO runs (VOPP_BATCH_GRAPH or VOPP_BATCH_PERSISTENT);
 * -1 for a null batch. */
int32_t vopp_batch_auto_mode(const vopp_batch* b);
void vopp_batch_free(vopp_batch* b);

/* One-shot form: create, run once, free. */
vopp_status vopp_plan_batch(const vopp_request* reqs, int32_t n, void* stream,
                            vopp_result* results);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of episodes' planning steps.                 */
/* ------------------------------------------------------------------------ */

/* hbm_budget_bytes: admission limit on the summed footprint (workspace and
 * particle buffers) of the active episodes.  max_active: most episodes
 * resident at once (<= 4096).  max_inflight: ticks queued ahead on the device
 * (1..8).  phases_per_tick: launches one tick queues back to back (0..64; 0
 * or 1: one), each advancing every active request by one phase; more per tick
 * means fewer host round trips per request, fewer means new requests join
 * sooner. */
typedef struct {
  uint64_t hbm_budget_bytes;
  int32_t max_active;
  int32_t max_inflight;
  int32_t phases_per_tick;
} vopp_server_config;

/* One episode: a model, its initial belief particles (HOST array, n_particles
 * of them, in vopp_plan's belief layout), the planner settings of every step,
 * the true initial state (HOST: tabular int32[1]; navigation fp32[2]), the
 * environment's seed and the number of real steps.  Every step plans with
 * params (step index t as the Philox counter word), executes the chosen
 * action in the simulated environment and updates the belief particles with
 * vopp_belief_update's filter -- all on the device.  Models need |A| <= 16. */
typedef struct {
  const vopp_pomdp* pomdp;
  const void* init_particles;
  int32_t n_particles;
  int32_t budget;
  int32_t depth;
  vopp_params params;
  const void* true_state;
  uint64_t env_seed;
  int32_t n_steps;
} vopp_episode_desc;

/* A finished planning request (one real step of one episode).  Times are
 * seconds on the server's steady clock: arrival = when the request was
 * issued (episode submission for step 0, completion of the previous step
 * otherwise), done = when the server saw its result. */
typedef struct {
  int32_t episode;
  int32_t step;
  int32_t action;
  int32_t status;
  double v_root;
  int64_t particle_steps;
  double arrival_s;
  double done_s;
} vopp_served;

typedef struct vopp_server vopp_server;

vopp_status vopp_server_create(const vopp_server_config* cfg, vopp_server** out);
/* Queue an episode for admission; its id is returned in *episode. */
vopp_status vopp_server_submit(vopp_server* s, const vopp_episode_desc* ep, int32_t* episode);
/* Admit what fits, issue up to phases_per_tick batched launches that each
 * advance every active request by one phase, and collect finished requests.  *pending
 * (may be NULL) = queued + active episodes after the call. */
vopp_status vopp_server_tick(vopp_server* s, int32_t* pending);
/* Move up to max finished requests into out; returns how many. */
int32_t vopp_server_poll(vopp_server* s, vopp_served* out, int32_t max);
/* Current true state (host out, as in vopp_episode_desc) and step of an
 * episode that is active or finished. */
vopp_status vopp_server_episode_state(vopp_server* s, int32_t episode, void* true_state,
                                      int32_t* steps_done);
void vopp_server_free(vopp_server* s);

/* ------------------------------------------------------------------------ */
/* Per-kernel timing (HIP events on the plan's stream).                      */
/* ------------------------------------------------------------------------ */

/* Kernel kinds of a plan, in the order of vopp_profile_read's arrays. */
enum {
  VOPP_KERNEL_FORWARD = 0,      /* all levels of one iteration's search      */
  VOPP_KERNEL_ACCUMULATE = 1,   /* shallow and shared visits from the trace  */
  VOPP_KERNEL_BACKUP_LEAF = 2,  /* leaf values (Alg. 3, leaves)              */
  VOPP_KERNEL_BACKUP_LEVEL = 3, /* one depth of the backup (Alg. 3 loop)     */
  VOPP_KERNEL_BACKUP_ROOT = 4,  /* root backup in double precision           */
  VOPP_KERNEL_SETUP = 5,        /* table clearing and root initialisation    */
  VOPP_KERNEL_SELECT = 6,       /* argmax of the root preferences            */
  VOPP_KERNEL_KINDS = 7
};

/* kind_mask != 0: every later vopp_plan in `ws` times each launch of the
 * kernel kinds whose bit (1 << kind) is set by the start and end timestamps
 * of its own dispatch (a pair of HIP events that hipExtLaunchKernel takes on
 * the plan's stream; the accumulate kind spans its claim pass too) and adds
 * the elapsed time to per-kind totals (-1 = all kinds).  kind_mask == 0 stops
 * it.  Totals are kept until vopp_profile_reset.  Timed launches are
 * dispatched with their events attached, which costs a little device time,
 * so time only the kinds being measured. */
vopp_status vopp_profile_enable(vopp_workspace* ws, int32_t kind_mask);
vopp_status vopp_profile_reset(vopp_workspace* ws);
/* ms[VOPP_KERNEL_KINDS] (host, out): summed kernel milliseconds per kind;
 * launches[VOPP_KERNEL_KINDS] (host, out, may be NULL): launch counts. */
vopp_status vopp_profile_read(const vopp_workspace* ws, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* VOPP_H */

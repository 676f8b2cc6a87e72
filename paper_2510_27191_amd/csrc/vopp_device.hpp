// vopp_device.hpp -- device-side data views and per-episode building blocks
// of the VOPP planning step on CDNA4 (gfx950).
//
// Everything here runs in registers: the Philox4x32-10 counter-based
// generator, the tabular and navigation generative models G (Sec. III-B)
// and the softmax action draw of Eq. (6).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vopp {

constexpr int kBlock = 256;                 // threads per block (4 wavefronts)
constexpr int kMaxA = 64;                   // actions held in registers
// Action field of parent links, trace words and aggregation keys.
constexpr int kActBits = 12;
constexpr unsigned long long kActMask = (1ull << kActBits) - 1;
constexpr int kMaxBudget = 256;             // iterations per plan
constexpr int kMaxDepth = 64;               // maximum leaf depth of a plan
// Level steps a sweep of one depth may visit: the plan's own (one per
// iteration) and up to as many again holding a kept subtree.
constexpr int kMaxRanges = 2 * kMaxBudget;
constexpr unsigned long long kEmptyKey = ~0ull;

// Belief keys of the open-addressing table (AppendBeliefs):
//   bits  0..19  observation key      bits 20..25  action
//   bits 26..55  parent's slot id     bits 56..63  iteration that inserted it
// A belief's slot id is its table slot + 1 (the root is 0): every episode that
// reaches a belief knows it as soon as its probe ends, without waiting for a
// numbering pass, so one launch can run every level.  The iteration stamp
// tells whether the belief was inserted by an earlier kernel (then its record
// exists and may be read) or by this one (then its preference row is psi0).
// Beliefs of a kept subtree carry the stamp 0xFF, which no iteration of a plan
// from a kept tree uses (such plans have at most 255 iterations).
// Records are stored by creation: the belief that episode ep inserts at level
// step t owns record 1 + t*n_p + ep (an episode inserts at most one belief per
// level step), so no episode allocates anything; the inserting episode stores
// the record index in the slot for later kernels.
constexpr int kObsBits = 20;                // observation field for |A| <= 64
constexpr int kKeyLowBits = 26;             // action and observation fields together
constexpr int kMaxAWide = 1 << 12;          // largest action set (rows in memory)
constexpr int kStampShift = 56;
constexpr unsigned long long kStampMask = 0xFFull << kStampShift;
constexpr unsigned long long kSidMask = (1ull << 30) - 1;
constexpr long long kMaxBeliefs = 1ll << 28;   // twice as many slots: ids <= 2^29
constexpr unsigned long long kCarryStamp = 0xFFull << kStampShift;
constexpr int kMaxCarryBudget = kMaxBudget - 1;

struct HSlot {
  unsigned long long key;
  int id;                    // record index (valid in later kernels)
  int pad;
};

// Trace words written by the forward kernel, one per (level, episode), for
// the visits it does not count itself (the two shallowest levels, which many
// episodes share, and beliefs another episode inserted in this iteration):
//   level d < D: (id << kActBits) | action;  leaf (d = D): id;
//   kTraceRec: id is a record index, else a slot id;  kEmptyKey: nothing.
constexpr unsigned long long kTraceRec = 1ull << 62;
constexpr int kDirectLevel = 2;             // levels >= this count in place

// Parent link of a record: (record << kActBits) | action, or kLinkSlot |
// (slot id << kActBits) | action while the parent's record is not known yet;
// ~0 for the root.
constexpr unsigned long long kLinkSlot = 1ull << 62;

enum : uint32_t { kTagRoot = 1, kTagStep = 2, kTagEnv = 4, kTagPF = 5, kTagResample = 6 };
enum : int { kTabular = 0, kNav = 1 };

struct NavParams {
  float lo, hi, step, sigma_move, sigma_obs0, sigma_obs_slope, obs_center_x,
      inv_bin;
  int key_lo, key_n;
  float goal_x, goal_y, goal_r2, disk_r2, r_step, r_goal, r_hit;
  int heuristic;
  int n_disks;
};

// Device copy of a model (owned by the pomdp handle).
struct ModelView {
  int kind;
  int nS, nA, nO, Apad;                    // Apad: row stride, multiple of 4
  const int* rowptr;                       // [nS*nA+1]
  const int* col;                          // [nnz]
  const uint32_t* thrT;                    // [nnz]
  const uint32_t* thrZ;                    // [nS*nA*nO]
  const float* R;                          // [nS*nA]
  const float* H;                          // [nS] or null
  NavParams nav;
  const float* disks;                      // [2*n_disks]
  const float* gauss;                      // [4096]
  int obs_bits;                            // observation field of belief keys; the
                                           // action field has 26 - obs_bits bits
  const double* logpi0;                    // [max(kMaxA, Apad)] ln pi0(a) of the reference
                                           // policy, normalised; -ln|A| if uniform
  float gamma;
  double gamma64;
};

// Per-belief fields besides the preference row and the action-node columns:
// the part every backup visit reads (hot) and the part only the leaf updates,
// the observation key and the tree dump use.
struct BeliefHot {
  float V;                   // L_eta Psi (internal) or mean heuristic (leaf)
  int Nb;                    // visit count N_b
  unsigned long long parent; // (parent id << kActBits) | action; ~0 for the root
};
struct BeliefLeaf {
  int leaf_cnt;              // this iteration's leaf visits (0 between iterations)
  int obs;                   // observation key (-1 for the root)
  unsigned long long leaf_h; // this iteration's heuristic sum (fixed point)
};

// The tree store in HBM: one array per field, indexed by belief id.  With
// ra = |A| rounded up to a multiple of 4, belief id owns
//   psi[id*ra ..] f32, n[id*ra ..] i32, c[id*ra ..] i64, w[id*ra ..] i64,
//   hot[id], leaf[id]
// where N, C (cumulative reward) and W (sum of V*N_b over the child beliefs)
// are the action nodes (b, a) of tensor A, stored with their parent belief.
// C, W and the leaf sums are 64-bit two's-complement fixed point.  Belief 0 is
// the root (its preference row is kept in double precision in psi_root); the
// beliefs created by level step t are ids 1 + t*n_p + [0, n_p), where
// list[t*n_p + ep] says which ids are used.  One depth of the tree is thus a
// few contiguous runs of ids, and a backup sweep that gives consecutive ids to
// consecutive lanes reads each field with full cache lines.
struct TreeView {
  float* psi;                    // [cap * ra]
  int* nv;                       // [cap * ra]
  unsigned long long* cv;        // [cap * ra]
  unsigned long long* wv;        // [cap * ra]
  BeliefHot* hot;                // [cap]
  BeliefLeaf* leaf;              // [cap]
  uint32_t* bits;                // [cap * bw] long rows only (see below)
  int ra;
  int bw;                        // bitmap words per belief (0 up to kMaxA actions)
  HSlot* h_slot;                 // [h_mask + 1] open-addressing table
  uint32_t h_mask;
  double* psi_root;              // [nA]
  float* psi0;                   // [ra] initial preference row ln pi0 / eta,
                                 // zero past |A|
  double* root_cdf;              // [nA] running sums of the root's softmax weights
  double* psi0_cdf64;            // [nA] running sums of the softmax weights of
                                 // the initial row (double precision; the draws
                                 // at beliefs created in the current iteration
                                 // read them)
  unsigned long long* root_acc;  // [3][ra][kStripes]: N, C and W of the root's
                                 // action nodes, striped over blocks (every
                                 // episode passes through one of them)
  double* v_root;                // [1]
  int* list;                     // [steps * n_p]: slot id of the belief that
                                 // episode ep inserted at level step t, or 0
  unsigned long long* counters;  // [1] error flags [2] beliefs of the last plan
                                 // [3] table dirty [5] last plan's level steps
                                 // [6] last plan's n_p
  unsigned long long* stats;     // [kStatRows][kStripes] particle steps, then two
                                 // banks of (action nodes, beliefs), near-tie
                                 // draws and the sweeps' work, striped over
                                 // blocks so that no address takes many atomics
  unsigned long long* gate;      // [4] plans with a time budget: [0] start on
                                 // the wall clock, [1] stop flag, [2] iterations run
  const int* carry_rng;          // [kMaxDepth + 1][2] level steps of a kept
                                 // subtree by depth: first step, step count
  const int* step_base;          // [K+1] first level step of each iteration
  unsigned long long* tr_key;    // [(depth + 1) * n_p] trace words
  float* tr_val;                 // reward (levels) or heuristic (leaf)
  // Optional per-draw export (null unless a traced plan): for the plan's own
  // level step t (0-based, kept-subtree steps not counted) and episode ep,
  // entry t * n_p + ep holds the drawn action and the observation key, or -1
  // where the episode drew nothing (it had terminated).
  short* dbg_act;
  int* dbg_obs;
  // Optional forced draws, same indexing: an entry in [0, nA) replaces the
  // kernel's decision at that draw (dbg_act still receives the kernel's own).
  const short* dbg_force;
  int dbg_step0;                 // level step of the plan's first own step
};

// Long rows (ra > kMaxA) add a bitmap of ra bits per belief, padded to
// 16-byte quads: for a belief other than the root, N[a], C[a] and W[a] hold
// values only where bit a is set (set, and the three cleared, by the first
// visit of (b, a)); elsewhere they are whatever the memory held.  A new belief
// then writes Psi, its tails and the bitmap, not three quarters of its bytes.
// The root's columns are all valid.
__host__ __device__ inline int rec_bitmap_quads(int ra) { return (ra + 127) / 128; }
__host__ __device__ inline int rec_bitmap_words(int ra) {
  return ra > kMaxA ? 4 * rec_bitmap_quads(ra) : 0;
}
// Bytes one belief owns across the field arrays.
__host__ __device__ inline int rec_bytes(int ra) {
  return 24 * ra + (int)(sizeof(BeliefHot) + sizeof(BeliefLeaf)) + 4 * rec_bitmap_words(ra);
}
__device__ __forceinline__ float* rec_psi(const TreeView& t, int id) {
  return t.psi + (size_t)id * (size_t)t.ra;
}
__device__ __forceinline__ int* rec_n(const TreeView& t, int id) {
  return t.nv + (size_t)id * (size_t)t.ra;
}
__device__ __forceinline__ unsigned long long* rec_c(const TreeView& t, int id) {
  return t.cv + (size_t)id * (size_t)t.ra;
}
__device__ __forceinline__ unsigned long long* rec_w(const TreeView& t, int id) {
  return t.wv + (size_t)id * (size_t)t.ra;
}
__device__ __forceinline__ BeliefHot* rec_hot(const TreeView& t, int id) { return t.hot + id; }
__device__ __forceinline__ BeliefLeaf* rec_leaf(const TreeView& t, int id) { return t.leaf + id; }
__device__ __forceinline__ uint32_t* rec_bits(const TreeView& t, int id) {
  return t.bits + (size_t)id * (size_t)t.bw;
}

// The tree dump's packed copy of one belief (gathered on the device, parsed
// on the host): Psi[ra] f32 | N[ra] i32 | C[ra] i64 | V f32 | N_b i32 | obs
// i32 | pad | parent u64 | bitmap (long rows).
__host__ __device__ inline int dump_n_off(int ra) { return 4 * ra; }
__host__ __device__ inline int dump_c_off(int ra) { return 8 * ra; }
__host__ __device__ inline int dump_tail_off(int ra) { return 16 * ra; }
__host__ __device__ inline int dump_bits_off(int ra) { return 16 * ra + 24; }
__host__ __device__ inline int dump_bytes(int ra) {
  return (dump_bits_off(ra) + 4 * rec_bitmap_words(ra) + 15) / 16 * 16;
}

// The root belief of a plan.
struct EpisodeView {
  const void* belief;      // root belief particles
  int n_belief;
};

constexpr int kBackupCap = 2048;            // default block cap of a backup sweep
constexpr int kStripes = 64;                // stripes of each tree statistic
constexpr int kStatRows = 9;                // rows of kStripes in TreeView::stats
constexpr int kStatNear = 5;                // row of the near-tie draw count
constexpr int kStatSweep = 6;               // rows 6, 7, 8: the level sweeps' belief
                                            // visits, internal-belief visits and
                                            // action-node visits over the plan
constexpr int kAccumCap = 4096;             // default block cap of the accumulate sweep

// Particle-filter belief and true-environment state of a served episode.
struct FilterView {
  void* part;              // M belief particles (the plan's root belief)
  void* prop;              // M propagated particles, same layout
  unsigned long long* w;   // [M] integer weights, then their inclusive sums
  int M;
  int* env;                // [0] state (tabular) or x bits, [1] y bits,
                           // [2] last observation, [3] last action,
                           // [4] last reward bits, [5] terminal flag
  uint32_t env_seed_lo, env_seed_hi;
};

struct PlanView {
  ModelView m;
  TreeView t;
  EpisodeView e;
  int n_p;
  float eta;
  double eta64;
  uint32_t seed_lo, seed_hi, step;
  float fix_scale;         // 2^S: fixed-point scale of the deterministic sums
  float fix_inv;           // 2^-S
  double fix_inv64;
  int K, depth, schedule;
  int steps;               // level steps of the plan (sum of D_k)
  double* out;             // max(kOutStride, ra + 12) doubles: the plan's result
  // Time budget (anytime plan): 0 = run all K iterations.  Otherwise the
  // iterations after the first run only while fewer than budget_ticks
  // wall-clock ticks have passed since set-up; K is then the cap.
  unsigned long long budget_ticks;
  unsigned long long* gate_host;  // pinned host word: iterations run | stop << 32
  int timed;
  // The plan starts from a kept subtree (tree re-rooting): its beliefs sit in
  // the level steps before the plan's own, listed by depth in t.carry_rng.
  int carry;
  // Plans without a workspace (the allocation-free entry point): set-up clears
  // the whole table (the memory holds whatever the last call left) and
  // writes the schedule t.step_base itself (the host copies nothing).
  int clear_all;
  FilterView f;            // served episodes only
};

// Tree statistics are counted by the backups of one iteration (the backup
// sweeps the whole tree): the last one, K.  Under a time budget the last
// iteration is not known in advance, so every iteration counts, into bank
// k & 1, and the root backup clears the other bank for the next iteration.
__device__ __forceinline__ bool counts_tree(const PlanView& P, int k) {
  return P.timed || k == P.K;
}
// Nodes stripes; the beliefs stripes follow at + kStripes.
__device__ __forceinline__ unsigned long long* stat_bank(const PlanView& P, int k) {
  return P.t.stats + (size_t)(1 + 2 * (P.timed ? (k & 1) : 0)) * kStripes;
}
// The time budget ran out at the end of an earlier iteration: the phases of
// later iterations return at once (uniform over the grid).
__device__ __forceinline__ bool budget_spent(const PlanView& P) {
  return P.timed && *reinterpret_cast<const volatile unsigned long long*>(&P.t.gate[1]) != 0ull;
}

// Result record written by the select phase (doubles): [0] action,
// [1..A] root preferences, [A+1] V(root), [A+2] particle steps, [A+3] beliefs,
// [A+4] action nodes, [A+5] input-error flags, [A+6] near-tie draws,
// [A+7 .. A+9] the level sweeps' belief, internal-belief and action-node visits.
constexpr int kOutStride = kMaxA + 12;

// Phase kinds (same numbering as the ABI's VOPP_KERNEL_* kinds).
enum : int {
  kPhaseForward = 0, kPhaseAccum = 1, kPhaseLeaf = 2, kPhaseLevel = 3,
  kPhaseRoot = 4, kPhaseSetup = 5, kPhaseSelect = 6,
  // Served episodes: true-environment step and SIR belief update.
  kPhaseEnv = 7, kPhasePFWeight = 8, kPhasePFScan = 9, kPhasePFResample = 10
};

// One phase of one instance inside a batched launch: blocks
// [blk0, blk0 + nblk) of the launch run phase `kind` of instance `inst`.
struct BatchItem {
  int inst, kind, a0, a1, blk0, nblk;
};

// The persistent batched launch: a work queue over every instance's phase
// list.  word[i] = (current phase << 32) | tiles of it taken; done[i] = tiles
// of the current phase finished; finished = instances past their last phase.
struct PersistView {
  unsigned long long* word;
  unsigned int* done;
  unsigned int* finished;
  const BatchItem* phases;     // every instance's phases, concatenated (a forward
                               // phase: blk0 = its blocks of episodes, nblk = tiles)
  const int* ph_off;           // [n + 1] first phase of each instance
  int n;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds; each multiplies words 0
// and 2 by the two round constants, mixes the high halves with the key and the
// other two words, and the key advances by the two Weyl constants.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo0 = c0 * 0xD2511F53u, hi0 = __umulhi(c0, 0xD2511F53u);
    const uint32_t lo1 = c2 * 0xCD9E8D57u, hi1 = __umulhi(c2, 0xCD9E8D57u);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(const PlanView& P, uint32_t ep, uint32_t tag,
                                   uint32_t level, uint32_t iter) {
  return philox(ep, (tag << 24) | level, iter, P.step, P.seed_lo, P.seed_hi);
}

// splitmix64 finaliser for the open-addressing table.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Count of thresholds <= u among n monotone thresholds = first j with u < thr_j.
// Rows are read as 16-byte vectors when 16-byte aligned, four vectors in
// flight at a time, so a row costs one memory round trip rather than one per
// vector.
__device__ __forceinline__ int count_le(const uint32_t* __restrict__ thr, int n,
                                        uint32_t u) {
  int c = 0;
  int j = 0;
  if ((((uintptr_t)thr) & 15) == 0) {
    for (; j + 16 <= n; j += 16) {
      const uint4* q = reinterpret_cast<const uint4*>(thr + j);
      const uint4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
      c += (q0.x <= u) + (q0.y <= u) + (q0.z <= u) + (q0.w <= u);
      c += (q1.x <= u) + (q1.y <= u) + (q1.z <= u) + (q1.w <= u);
      c += (q2.x <= u) + (q2.y <= u) + (q2.z <= u) + (q2.w <= u);
      c += (q3.x <= u) + (q3.y <= u) + (q3.z <= u) + (q3.w <= u);
    }
    for (; j + 4 <= n; j += 4) {
      const uint4 q = *reinterpret_cast<const uint4*>(thr + j);
      c += (q.x <= u) + (q.y <= u) + (q.z <= u) + (q.w <= u);
    }
  }
#pragma unroll 8
  for (; j < n; ++j) c += (thr[j] <= u) ? 1 : 0;
  return c;
}

// Tabular transition: successor of (s, a) from a 32-bit random word.
__device__ __forceinline__ int tabular_next(const ModelView& m, int s, int a, uint32_t word) {
  const int row = s * m.nA + a;
  const int lo = m.rowptr[row];
  const int n = m.rowptr[row + 1] - lo;
  int j = count_le(m.thrT + lo, n, word >> 1);
  j = j < n ? j : n - 1;
  return m.col[lo + j];
}

// Tabular G: successor from word y, observation from word z, R(s, a).
__device__ __forceinline__ void tabular_step(const ModelView& m, int s, int a,
                                             const U4& x, int& sn, int& obs,
                                             float& r) {
  r = m.R[s * m.nA + a];
  sn = tabular_next(m, s, a, x.y);
  const uint32_t* zr = m.thrZ + ((size_t)sn * m.nA + a) * m.nO;
  int o = count_le(zr, m.nO, x.z >> 1);
  obs = o < m.nO ? o : m.nO - 1;
}

__device__ __forceinline__ int nav_axis(const NavParams& p, float v) {
  float c = floorf(v * p.inv_bin);
  c = fmaxf(fminf(c, (float)(p.key_lo + p.key_n - 1)), (float)p.key_lo);
  return (int)c - p.key_lo;
}

// Navigation motion: next position of (x, y) under move a, noise from word y.
__device__ __forceinline__ void nav_move(const ModelView& m, float x, float y, int a,
                                         uint32_t word, float& nx, float& ny) {
  const NavParams& p = m.nav;
  float dx = 0.0f, dy = 0.0f;
  if (a == 0) dy = p.step;
  else if (a == 1) dx = p.step;
  else if (a == 2) dy = -p.step;
  else dx = -p.step;
  const float zx = m.gauss[word >> 20];
  const float zy = m.gauss[(word >> 8) & 4095u];
  const float mx = x + dx;
  const float my = y + dy;
  nx = fminf(fmaxf(mx + p.sigma_move * zx, p.lo), p.hi);
  ny = fminf(fmaxf(my + p.sigma_move * zy, p.lo), p.hi);
}

__device__ __forceinline__ float nav_obs_sd(const NavParams& p, float nx) {
  return p.sigma_obs0 + p.sigma_obs_slope * fabsf(nx - p.obs_center_x);
}

// Obstacle centres of the navigation model held in registers (uniform across
// the wavefront) when there are at most kDiskRegs of them; more are read from
// memory.  Reading them once per kernel keeps the obstacle test free of
// memory waits.
constexpr int kDiskRegs = 8;
struct DiskCache {
  float c[2 * kDiskRegs];
};
__device__ __forceinline__ DiskCache load_disks(const ModelView& m) {
  DiskCache d;
  const int n = m.nav.n_disks;
#pragma unroll
  for (int i = 0; i < 2 * kDiskRegs; ++i) d.c[i] = i < 2 * n ? m.disks[i] : 0.0f;
  return d;
}
__device__ __forceinline__ bool nav_hit(const ModelView& m, const DiskCache& dc, float nx,
                                        float ny) {
  const NavParams& p = m.nav;
  bool hit = false;
  if (p.n_disks <= kDiskRegs) {
#pragma unroll
    for (int i = 0; i < kDiskRegs; ++i) {
      const float ex = nx - dc.c[2 * i], ey = ny - dc.c[2 * i + 1];
      hit = hit || (i < p.n_disks && (ex * ex + ey * ey) <= p.disk_r2);
    }
  } else {
    for (int i = 0; i < p.n_disks; ++i) {
      const float ex = nx - m.disks[2 * i], ey = ny - m.disks[2 * i + 1];
      hit = hit || ((ex * ex + ey * ey) <= p.disk_r2);
    }
  }
  return hit;
}

// The four standard-normal quantiles one navigation step uses: motion noise
// from word y, observation noise from word z.
struct NavNoise {
  float mx, my, ox, oy;
};
__device__ __forceinline__ NavNoise nav_noise(const ModelView& m, const U4& w) {
  return NavNoise{m.gauss[w.y >> 20], m.gauss[(w.y >> 8) & 4095u], m.gauss[w.z >> 20],
                  m.gauss[(w.z >> 8) & 4095u]};
}

// Navigation G with its noise already read.  Built without contraction: each
// operation rounds once.
__device__ __forceinline__ void nav_step_z(const ModelView& m, const DiskCache& dc, float x,
                                           float y, int a, const NavNoise& z, float& nx,
                                           float& ny, int& key, float& r, bool& term) {
  const NavParams& p = m.nav;
  float dx = 0.0f, dy = 0.0f;
  if (a == 0) dy = p.step;
  else if (a == 1) dx = p.step;
  else if (a == 2) dy = -p.step;
  else dx = -p.step;
  const float mx = x + dx;
  const float my = y + dy;
  nx = fminf(fmaxf(mx + p.sigma_move * z.mx, p.lo), p.hi);
  ny = fminf(fmaxf(my + p.sigma_move * z.my, p.lo), p.hi);
  const float sd = nav_obs_sd(p, nx);
  const float ox = nx + sd * z.ox;
  const float oy = ny + sd * z.oy;
  key = nav_axis(p, ox) * p.key_n + nav_axis(p, oy);
  const float gx = nx - p.goal_x, gy = ny - p.goal_y;
  const bool goal = (gx * gx + gy * gy) <= p.goal_r2;
  const bool hit = nav_hit(m, dc, nx, ny);
  float rr = p.r_step;
  if (goal) rr = rr + p.r_goal;
  if (hit) rr = rr + p.r_hit;
  r = rr;
  term = goal;
}

// Navigation G (Sec. III-B generative model of the navigation workload).
__device__ __forceinline__ void nav_step(const ModelView& m, float x, float y,
                                         int a, const U4& w, float& nx,
                                         float& ny, int& key, float& r,
                                         bool& term) {
  nav_step_z(m, load_disks(m), x, y, a, nav_noise(m, w), nx, ny, key, r, term);
}

__device__ __forceinline__ float nav_heuristic(const NavParams& p, float x, float y) {
  if (p.heuristic == 0) return 0.0f;
  return -(fabsf(x - p.goal_x) + fabsf(y - p.goal_y));
}

// Near-tie screen of the kernel's own draws: a draw counts as a near tie when
// t lies within kTieRel * P_last of an interior boundary P_j next to it (the
// running sums just below and above t).  Rows whose entries are all equal are
// decided exactly and never count.
constexpr double kTieRel = 1.0 / 65536.0;

// Softmax draw of Eq. (6) over a row held in registers: single-precision
// weights exp(eta (psi_j - max)), their running sums P_j and t = u * P_last
// in double precision, action = first j with t < P_j.  The double sums of
// single-precision weights are exact to far below the weights' own rounding,
// and the product u * P_last is exact, so a row whose entries are all equal
// (weights exactly 1, P_j = j + 1) gives floor(u |A|) exactly.  AM >= A is a
// compile-time bound so the row stays in registers.
template <int AM>
__device__ __forceinline__ int draw_row32(float (&v)[AM], int A, float eta, uint32_t x0,
                                          bool& near) {
  float m = v[0];
  bool flat = true;
#pragma unroll
  for (int j = 1; j < AM; ++j)
    if (j < A) { m = fmaxf(m, v[j]); flat = flat && v[j] == v[0]; }
  double total = 0.0;
#pragma unroll
  for (int j = 0; j < AM; ++j)
    if (j < A) { v[j] = expf(eta * (v[j] - m)); total = total + (double)v[j]; }
  const double u = (double)(x0 >> 8) * (1.0 / 16777216.0);
  const double t = u * total;
  double run = 0.0, below = 0.0, above = total;
  int a = A - 1;
  bool found = false;
#pragma unroll
  for (int j = 0; j < AM; ++j) {
    if (j < A && !found) {
      below = run;
      run = run + (double)v[j];
      if (t < run) { a = j; found = true; above = run; }
    }
  }
  const double lim = kTieRel * total;
  near = !flat && ((a > 0 && t - below <= lim) || (a < A - 1 && above - t <= lim));
  return a;
}

// A preference row (padded to a multiple of 4) read into registers.
template <int AM>
__device__ __forceinline__ void load_row(const float* __restrict__ row, int A, float (&v)[AM]) {
#pragma unroll
  for (int j = 0; j < AM; j += 4) {
    float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (j < A) q = *reinterpret_cast<const float4*>(row + j);
    v[j] = q.x; v[j + 1] = q.y; v[j + 2] = q.z; v[j + 3] = q.w;
  }
}

// The running sums P_j of the weights exp(eta (psi_j - max)) of the root row
// (double precision), accumulated in action order; the root draw
// (draw_cdf64: t = u * P_last, the first j with t < P_j) reads them.  The
// root row changes once per iteration, so every episode's root draw reads
// these instead of evaluating 2|A| double exponentials.
__device__ __forceinline__ void root_cdf(const double* __restrict__ row, int A, double eta,
                                         double* __restrict__ cdf) {
  double m = row[0];
  for (int j = 1; j < A; ++j) m = fmax(m, row[j]);
  double run = 0.0;
  for (int j = 0; j < A; ++j) {
    run = run + exp(eta * (row[j] - m));
    cdf[j] = run;
  }
}

// draw_cdf64 by bisection: the first j with t < P_j in a non-decreasing row.
__device__ __forceinline__ int draw_cdf64_bisect(const double* __restrict__ cdf, int A,
                                                 uint32_t x0) {
  const double u = (double)(x0 >> 8) * (1.0 / 16777216.0);
  const double t = u * cdf[A - 1];
  int lo = 0, hi = A - 1;                     // the answer lies in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (t < cdf[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ int draw_cdf64(const double* __restrict__ cdf, int A, uint32_t x0) {
  const double u = (double)(x0 >> 8) * (1.0 / 16777216.0);
  const double t = u * cdf[A - 1];
  for (int j = 0; j < A; ++j)
    if (t < cdf[j]) return j;
  return A - 1;
}

// draw_cdf64 over running sums held in registers (AM >= A of them): the
// same comparisons in the same order.
template <int AM>
__device__ __forceinline__ int draw_cdf64_regs(const double (&cdf)[AM], int A, uint32_t x0) {
  double last = cdf[0];
#pragma unroll
  for (int j = 1; j < AM; ++j)
    if (j == A - 1) last = cdf[j];
  const double u = (double)(x0 >> 8) * (1.0 / 16777216.0);
  const double t = u * last;
  int a = A - 1;
  bool found = false;
#pragma unroll
  for (int j = 0; j < AM; ++j) {
    if (!found && j < A && t < cdf[j]) {
      a = j;
      found = true;
    }
  }
  return a;
}

// Whether the draw of action a from running sums cdf lies within kTieRel *
// P_last of one of its interior boundaries (cdf[a - 1] below, cdf[a] above).
// flat: the row's entries are all equal (then the draw is exact).
__device__ __forceinline__ bool near_tie64(const double* __restrict__ cdf, int A, uint32_t x0,
                                           int a) {
  const double u = (double)(x0 >> 8) * (1.0 / 16777216.0);
  const double tot = cdf[A - 1];
  const double t = u * tot;
  const double lim = kTieRel * tot;
  return (a > 0 && t - cdf[a - 1] <= lim) || (a < A - 1 && cdf[a] - t <= lim);
}

// Fixed-point conversion of a value for the order-independent sums.
__device__ __forceinline__ unsigned long long to_fix(float v, float scale) {
  return (unsigned long long)__float2ll_rn(v * scale);
}
__device__ __forceinline__ float from_fix(unsigned long long v, float inv) {
  return (float)(long long)v * inv;
}

}  // namespace vopp

// vopp_kernels.hip -- HIP kernels of one VOPP planning step for gfx950.
//
// One iteration of Alg. 1 is a short, fixed sequence of phases:
//
//   forward     one thread per episode runs every level of the vectorized
//               forward search (Alg. 2) with its state in registers: draw the
//               action from the softmax of the belief's preferences (Eq. 6),
//               call G, count the visit and reward into the action node
//               (AppendActions), and find or insert the child belief
//               (belief, action, observation) in the open-addressing table
//               (AppendBeliefs).  A belief is named by its table slot, so no
//               episode ever waits for another and one launch covers all D_k
//               levels; the inserting episode also takes the belief's record.
//               Visits it cannot count in place go to a trace.
//   accumulate  folds the trace into the records (LDS-aggregated atomics).
//   backup      Alg. 3, one phase per depth over every belief of that depth:
//               leaves take their mean heuristic, internal beliefs update their
//               preference row with Q = C/N + gamma W and V = L_eta Psi, and
//               each belief pushes V*N_b into its parent action's W
//               accumulator.  The root runs in double precision.
//
// All cross-episode sums (rewards, heuristics, V*N_b) are 64-bit fixed-point
// integer atomics, so the results do not depend on thread order; which slot
// and record a belief gets depends on the order of insertions, the tree and
// every value in it do not.
//
// Every phase is a __device__ function of (plan view, block index within the
// phase, block count of the phase).  The single-plan path launches one kernel
// per phase; the batched path launches k_batch, whose blocks each run one
// phase of one instance of a batch (BatchItem), so one launch advances every
// instance of the batch by one phase.
#include <hip/hip_ext.h>

#include <algorithm>

#include "vopp_device.hpp"
#include "vopp_launch.hpp"

namespace vopp {

// ---------------------------------------------------------------------------
// Open-addressing table of 16-byte slots, load <= 1/2.  Finds or inserts key;
// the inserting thread writes key | stamp.  Returns the slot, or ~0u if the
// table has no free slot left (an internal error, reported by the plan).
//
// A key hashes to a bucket, one 128-byte line of 8 slots, which the probe
// reads with one round of loads and scans in registers; a full bucket
// continues into the next line.  Within a line the key visits the slots in a
// rotated order that is a function of the key, so every thread that looks
// for one key meets the same first empty slot (linear probing over a fixed
// per-key sequence: one compare-and-swap there decides the insert), while
// different keys spread their inserts over the line.  A wavefront waits for
// its slowest lane, so reading whole lines and deciding in registers keeps
// most wavefronts at one read and at most one compare-and-swap per lane (a
// compare-and-swap is about twice as slow as a read).  Keys and record indices written by earlier kernels are
// visible to the plain loads; a key being inserted by this kernel may read
// as empty, and then the compare-and-swap returns it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t probe(const TreeView& t, unsigned long long key,
                                          unsigned long long stamp, bool& won,
                                          bool& fresh, int& id) {
  const unsigned long long hk = mix64(key);
  uint32_t base = (uint32_t)hk & t.h_mask & ~7u;
  const uint32_t rot = (uint32_t)(hk >> 40) & 7u;
  const uint32_t lines = (t.h_mask >> 3) + 1;
  for (uint32_t n = 0; n <= 2 * lines; ++n) {
    const uint4* ln = reinterpret_cast<const uint4*>(&t.h_slot[base]);
    uint4 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = ln[j];
    // The first slot in the key's order that holds the key or is empty.
    uint32_t best = 8;
    int at = -1;
    bool empty = false;
    int rid = -1;
    unsigned long long seen = kEmptyKey;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned long long cur = ((unsigned long long)v[j].y << 32) | v[j].x;
      const uint32_t pos = ((uint32_t)j - rot) & 7u;
      if ((cur == kEmptyKey || (cur & ~kStampMask) == key) && pos < best) {
        best = pos;
        at = j;
        empty = cur == kEmptyKey;
        seen = cur;
        rid = (int)v[j].z;
      }
    }
    if (at < 0) {                               // the bucket is full: next line
      base = (base + 8u) & t.h_mask;
      continue;
    }
    const uint32_t slot = base + (uint32_t)at;
    if (empty) {
      seen = atomicCAS(&t.h_slot[slot].key, kEmptyKey, key | stamp);
      if (seen == kEmptyKey) {
        won = true;
        fresh = true;
        id = -1;
        return slot;
      }
      if ((seen & ~kStampMask) != key) continue;  // another key took it: re-read
      rid = -1;                                 // inserted by this kernel: fresh
    }
    won = false;
    fresh = (seen & kStampMask) == stamp;
    id = fresh ? -1 : rid;
    return slot;
  }
  won = false;
  fresh = false;
  id = -1;
  return ~0u;
}

// The first line of a key's probe sequence (its 8 slots, one batch of
// loads) and the key's slot order in it.
struct Bucket {
  uint4 v[8];
  uint32_t base, rot;
};
__device__ __forceinline__ void bucket_read(const TreeView& t, unsigned long long key,
                                            Bucket& b) {
  const unsigned long long hk = mix64(key);
  b.base = (uint32_t)hk & t.h_mask & ~7u;
  b.rot = (uint32_t)(hk >> 40) & 7u;
  const uint4* ln = reinterpret_cast<const uint4*>(&t.h_slot[b.base]);
#pragma unroll
  for (int j = 0; j < 8; ++j) b.v[j] = ln[j];
}

// probe() split for the forward search, on the first line already read:
//   1: the key is there (won false; fresh and id as probe() sets them);
//   2: an empty slot comes first in the key's order; the insert's
//      compare-and-swap is issued and its old value returned in `seen`,
//      not waited for (the caller settles it later with settle_insert);
//   0: the line is full (the caller falls back to probe()).
__device__ __forceinline__ int probe_line(const TreeView& t, const Bucket& b,
                                          unsigned long long key, unsigned long long stamp,
                                          uint32_t& slot, bool& fresh, int& id,
                                          unsigned long long& seen) {
  uint32_t best = 8;
  int at = -1;
  bool empty = false;
  unsigned long long cur_at = kEmptyKey;
  int rid = -1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const unsigned long long cur = ((unsigned long long)b.v[j].y << 32) | b.v[j].x;
    const uint32_t pos = ((uint32_t)j - b.rot) & 7u;
    if ((cur == kEmptyKey || (cur & ~kStampMask) == key) && pos < best) {
      best = pos;
      at = j;
      empty = cur == kEmptyKey;
      cur_at = cur;
      rid = (int)b.v[j].z;
    }
  }
  if (at < 0) return 0;
  slot = b.base + (uint32_t)at;
  if (empty) {
    seen = atomicCAS(&t.h_slot[slot].key, kEmptyKey, key | stamp);
    fresh = true;
    id = -1;
    return 2;
  }
  fresh = (cur_at & kStampMask) == stamp;
  id = fresh ? -1 : rid;
  return 1;
}

// Key of belief (parent slot id b, action a, observation obs); the
// observation takes the low ob bits, the action the next 26 - ob.
__device__ __forceinline__ unsigned long long belief_key(int b, int a, int obs, int ob) {
  return ((unsigned long long)(uint32_t)b << kKeyLowBits) |
         ((unsigned long long)(uint32_t)a << ob) | (uint32_t)obs;
}

// ---------------------------------------------------------------------------
// Shared memory of every phase (one static allocation per kernel).
// ---------------------------------------------------------------------------

// Block-level pre-aggregation.  Shallow tree levels funnel many episodes into
// few nodes (every episode of an iteration passes through one of the |A| root
// action nodes), so same-address global atomics would serialise.  Each block
// first combines its contributions per key in an LDS hash table and then
// issues one global atomic per distinct key.  Integer adds are
// order-independent, so results stay bit-identical.
constexpr int kAggSlots = 2 * kBlock;      // at most kBlock keys per block

struct AggTable {
  unsigned long long key[kAggSlots];
  unsigned long long a[kAggSlots];
  unsigned long long b[kAggSlots];
};

// Level steps holding the beliefs of one depth: level dep-1 of every
// iteration that reached that depth created one run of n_p records.
struct Ranges {
  int n;
  int step[kMaxRanges];
};

struct Smem {
  AggTable agg;
  Ranges ranges;
  unsigned long long wave[kBlock / 64];
  float psi0[kMaxA];        // the forward search's copy of the initial row
};

__device__ __forceinline__ void agg_clear(AggTable& T) {
  for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
    T.key[i] = kEmptyKey;
    T.a[i] = 0ull;
    T.b[i] = 0ull;
  }
}

__device__ __forceinline__ int agg_slot(AggTable& T, unsigned long long key) {
  uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 55);   // 9 bits
  while (true) {
    const unsigned long long prev = atomicCAS(&T.key[h], kEmptyKey, key);
    if (prev == kEmptyKey || prev == key) return (int)h;
    h = (h + 1) & (kAggSlots - 1);
  }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; red holds kBlock / 64 words of LDS.  Called by every
// thread of the block (it contains barriers); thread 0 gets the total.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v,
                                                        unsigned long long* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Phase: set-up of a plan.  Clears the belief table (a full fill, or only the
// slots the previous plan used when that is cheaper), the list lengths and
// the root record.  The previous plan's sizes are read on the device, so the
// phase is identical on every replay of a captured launch sequence.
// ---------------------------------------------------------------------------
// LDS of the set-up of a plan with more than kMaxA actions (the root's draw
// table is built by the block).
struct SetupSmem {
  double buf[kBlock];
  double red[kBlock / 64];
  double bc;
  unsigned long long part[kBlock];
};
__device__ double block_max64(double v, double* red);
__device__ double block_ordered_sum(const double* x, int A, double m, double eta, double* cdf,
                                    double* buf, double* bc);

__device__ void dev_setup(const PlanView& P, int blk, int nblk, SetupSmem* ss) {
  const TreeView& T = P.t;
  const unsigned long long n_prev = T.counters[2];
  const size_t hcap = (size_t)T.h_mask + 1;
  const bool full = P.clear_all || T.counters[3] != 0ull ||
                    n_prev * 10ull >= (unsigned long long)hcap;
  const size_t tid = (size_t)blk * kBlock + threadIdx.x;
  const size_t stride = (size_t)nblk * kBlock;
  if (P.carry) {
    // The table and the kept records were written by the re-rooting.
  } else if (full) {
    uint4* hs = reinterpret_cast<uint4*>(T.h_slot);
    const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (size_t i = tid; i < hcap; i += stride) hs[i] = ones;
  } else {
    const size_t used = (size_t)T.counters[5] * (size_t)T.counters[6];
    for (size_t i = tid; i < used; i += stride) {
      const int sid = T.list[i];
      if (sid) T.h_slot[sid - 1].key = kEmptyKey;
    }
  }
  // Root action-node sums; with a kept root, stripe 0 of N and C starts from
  // its record (written below by block 0).
  for (size_t i = tid; i < (size_t)3 * T.ra * kStripes; i += stride)
    if (!(P.carry && i % kStripes == 0 && i < (size_t)2 * T.ra * kStripes)) T.root_acc[i] = 0ull;
  if (blk == 0) {
    if (!P.carry) {                             // a fresh root: every field of belief 0
      for (int i = threadIdx.x; i < T.ra; i += kBlock) {
        rec_psi(T, 0)[i] = 0.0f;
        rec_n(T, 0)[i] = 0;
        rec_c(T, 0)[i] = 0ull;
        rec_w(T, 0)[i] = 0ull;
      }
      for (int i = threadIdx.x; i < T.bw; i += kBlock) rec_bits(T, 0)[i] = 0u;
      if (threadIdx.x == 0) {
        *rec_hot(T, 0) = BeliefHot{0.0f, 0, kEmptyKey};
        *rec_leaf(T, 0) = BeliefLeaf{0, -1, 0ull};
      }
    }
    __syncthreads();
    const int j = threadIdx.x;
    for (int i = j; i < kStatRows * kStripes; i += kBlock) T.stats[i] = 0ull;
    if (j == 0 && P.clear_all) {
      // The schedule D_k (no kept subtree on this path): first level step of
      // each iteration.
      int* sb = const_cast<int*>(T.step_base);
      int run = 0;
      for (int k = 1; k <= P.K; ++k) {
        sb[k - 1] = run;
        run += P.schedule == 1 ? P.depth : min(k, P.depth);
      }
      sb[P.K] = run;
    }
    if (j == 0) {
      T.gate[0] = (unsigned long long)wall_clock64();   // start of the plan
      T.gate[1] = 0ull;
      T.gate[2] = 0ull;
    }
    for (int a = j; a < T.ra; a += kBlock) {
      // Initial preferences ln pi0 / eta: the root keeps them in double
      // precision, every other belief starts from their f32 rounding.
      const double v = a < P.m.nA ? P.m.logpi0[a] / P.eta64 : 0.0;
      T.psi0[a] = (float)v;
      if (a < P.m.nA) {
        if (P.carry) {                          // the kept root's own row and sums
          // (long rows: the kept belief's columns count where its bitmap says)
          const bool v = T.ra <= kMaxA || ((rec_bits(T, 0)[a >> 5] >> (a & 31)) & 1u);
          T.psi_root[a] = (double)rec_psi(T, 0)[a];
          T.root_acc[((size_t)0 * T.ra + a) * kStripes] =
              v ? (unsigned long long)(long long)rec_n(T, 0)[a] : 0ull;
          T.root_acc[((size_t)1 * T.ra + a) * kStripes] = v ? rec_c(T, 0)[a] : 0ull;
        } else {
          rec_psi(T, 0)[a] = (float)v;
          T.psi_root[a] = v;
        }
      } else if (P.carry) {
        T.root_acc[((size_t)0 * T.ra + a) * kStripes] = 0ull;
        T.root_acc[((size_t)1 * T.ra + a) * kStripes] = 0ull;
      }
    }
    __syncthreads();
    if (T.ra > kMaxA) {                         // long rows: the block builds the table
      double mloc = -INFINITY;
      for (int a = j; a < P.m.nA; a += kBlock) mloc = fmax(mloc, T.psi_root[a]);
      const double m = block_max64(mloc, ss->red);
      block_ordered_sum(T.psi_root, P.m.nA, m, P.eta64, T.root_cdf, ss->buf, &ss->bc);
      // The initial row's running sums: eta * psi0 = ln pi0.
      double m0 = -INFINITY;
      for (int a = j; a < P.m.nA; a += kBlock) m0 = fmax(m0, P.m.logpi0[a]);
      m0 = block_max64(m0, ss->red);
      block_ordered_sum(P.m.logpi0, P.m.nA, m0, 1.0, T.psi0_cdf64, ss->buf, &ss->bc);
    }
    if (j == 0) {
      if (T.ra <= kMaxA) {
        root_cdf(T.psi_root, P.m.nA, P.eta64, T.root_cdf);
        // The initial row ln pi0 / eta in double precision: its running sums
        // serve the draws at beliefs created in the current iteration.
        double m = P.m.logpi0[0] / P.eta64;
        for (int a = 1; a < P.m.nA; ++a) m = fmax(m, P.m.logpi0[a] / P.eta64);
        double run = 0.0;
        for (int a = 0; a < P.m.nA; ++a) {
          run = run + exp(P.eta64 * (P.m.logpi0[a] / P.eta64 - m));
          T.psi0_cdf64[a] = run;
        }
      }
      rec_leaf(T, 0)->obs = -1;
      rec_hot(T, 0)->parent = kEmptyKey;
      T.v_root[0] = P.carry ? (double)rec_hot(T, 0)->V : 0.0;
      T.counters[1] = 0ull;
      T.counters[4] = 0ull;
    }
  }
}

// ---------------------------------------------------------------------------
// Phase: the forward search of iteration k over D levels (Alg. 2).
// ---------------------------------------------------------------------------

// A new belief's record: Psi = ln pi0 / eta (the first term of Eq. 4; uniform
// unless a reference policy is set), N = C = W = 0, its observation key and its
// parent link.
// psi0s: the initial row staged in LDS (a copy from global memory would wait
// for every store issued before it).
__device__ __forceinline__ void init_record(const PlanView& P, const float* psi0s, int id,
                                            int obs, unsigned long long link) {
  const TreeView& T = P.t;
  const int ra = T.ra;
  float4* pq = reinterpret_cast<float4*>(rec_psi(T, id));
  int4* nq = reinterpret_cast<int4*>(rec_n(T, id));
  ulonglong2* cq = reinterpret_cast<ulonglong2*>(rec_c(T, id));
  ulonglong2* wq = reinterpret_cast<ulonglong2*>(rec_w(T, id));
  const float4* p0 = reinterpret_cast<const float4*>(psi0s);
  const ulonglong2 z2 = make_ulonglong2(0ull, 0ull);
  for (int j = 0; j < ra / 4; ++j) {
    pq[j] = p0[j];
    nq[j] = make_int4(0, 0, 0, 0);
    cq[2 * j] = z2;
    cq[2 * j + 1] = z2;
    wq[2 * j] = z2;
    wq[2 * j + 1] = z2;
  }
  *rec_hot(T, id) = BeliefHot{0.0f, 0, link};
  *rec_leaf(T, id) = BeliefLeaf{0, obs, 0ull};
}

template <int AM>
__device__ void dev_forward(const PlanView& P, int k, int D, int blk,
                            unsigned long long* red, float* psi0s) {
  const TreeView& T = P.t;
  // The initial row in LDS, copied into new records (every thread of the
  // block calls).
  for (int i = threadIdx.x; i < T.ra; i += kBlock) psi0s[i] = T.psi0[i];
  __syncthreads();
  const int t0 = T.step_base[k - 1];          // level step of level 0
  const int ep = blk * kBlock + threadIdx.x;
  const bool ep_ok = ep < P.n_p;
  const int A = P.m.nA;
  const bool nav = P.m.kind != kTabular;
  const size_t n_p = (size_t)P.n_p;
  const unsigned long long stamp = (unsigned long long)(k - 1) << kStampShift;
  int s = 0;
  float x = 0.0f, y = 0.0f;
  int sid = 0;                // current belief's slot id (0: root)
  int rid = 0;                // its record, -1 if another episode inserted it
                              // during this iteration
  bool fresh = false;         // inserted during this iteration (Psi initial)
  bool alive = false;
  if (ep_ok) {
    // Alg. 1: the episode starts at the root with a state drawn from the
    // belief particles.
    const U4 w = draw(P, (uint32_t)ep, kTagRoot, 0, (uint32_t)k);
    const uint32_t idx = __umulhi(w.x, (uint32_t)P.e.n_belief);
    if (!nav) {
      s = ((const int*)P.e.belief)[idx];
      if ((unsigned)s >= (unsigned)P.m.nS) {   // caller's particle out of range
        atomicOr((unsigned int*)&T.counters[1], 1u);
        s = 0;
      }
    } else {
      const float* bf = (const float*)P.e.belief;
      x = bf[idx];
      y = bf[P.e.n_belief + idx];
    }
    alive = true;
  }
  // Inputs of the next level, read ahead of the previous level's writes: a
  // wait for a load also waits for every memory operation issued before it.
  U4 w = draw(P, (uint32_t)ep, kTagStep, 0u, (uint32_t)k);
  float row[AM];
#pragma unroll
  for (int j = 0; j < AM; ++j) row[j] = 0.0f;
  NavNoise z{0.0f, 0.0f, 0.0f, 0.0f};
  if (alive && nav) z = nav_noise(P.m, w);
  DiskCache dc;
#pragma unroll
  for (int i = 0; i < 2 * kDiskRegs; ++i) dc.c[i] = 0.0f;
  if (nav) dc = load_disks(P.m);
  // The running sums of the initial row in registers for short rows, so that
  // a draw at a belief created in this iteration issues no memory access.
  constexpr int kCdfRegs = AM <= 8 ? AM : 1;
  double cdf0[kCdfRegs];
#pragma unroll
  for (int j = 0; j < kCdfRegs; ++j) cdf0[j] = (AM <= 8 && j < A) ? T.psi0_cdf64[j] : 0.0;
  unsigned long long g = 0;   // generative-model calls of this episode
  unsigned long long nt = 0;  // its near-tie draws
  // An insert whose compare-and-swap is still in flight: the episode goes on
  // as if it had won the slot (a belief created in this iteration, Psi
  // initial, whichever episode inserted it) and settles it at the next level
  // or after the last one.  Only if another key took the slot does the next
  // level's key change; it is then formed again.  The insert's writes (list
  // entry, slot's record index, the new record) wait for the settlement.
  bool pend = false;
  uint32_t pend_slot = 0;
  unsigned long long pend_key = 0, pend_seen = 0, pend_link = 0;
  int pend_t = 0, pend_obs = 0;
  // Settles the pending insert: sets sid and rid of the belief the episode
  // stands on; returns false if the table is full.
  auto settle = [&]() -> bool {
    pend = false;
    bool won = pend_seen == kEmptyKey;
    int rid_new = -1;
    uint32_t slot = pend_slot;
    if (!won && (pend_seen & ~kStampMask) != pend_key) {
      // Another key took the slot: find or insert the key again (a belief of
      // this iteration either way, so the draws made on it stand).
      atomicAdd(&T.counters[4], 1ull);
      bool fr;
      int id;
      slot = probe(T, pend_key, stamp, won, fr, id);
      if (slot == ~0u) {
        atomicOr((unsigned int*)&T.counters[1], 2u);
        if (ep_ok) T.list[(size_t)pend_t * n_p + ep] = 0;
        return false;
      }
    }
    if (won) rid_new = 1 + pend_t * P.n_p + ep;   // the inserter's own record
    sid = (int)slot + 1;
    rid = rid_new;
    fresh = true;
    T.list[(size_t)pend_t * n_p + ep] = won ? sid : 0;
    if (won) {
      T.h_slot[slot].id = rid_new;
      init_record(P, psi0s, rid_new, pend_obs, pend_link);
    }
    return true;
  };
  for (int d = 0; d < D; ++d) {
    unsigned long long tk = kEmptyKey;
    float r = 0.0f;
    bool direct = false, insert_now = false, won_now = false;
    int obs = 0, a = 0;
    uint32_t h = 0;
    unsigned long long link = kEmptyKey;
    const bool drew = alive;
    int own = 0;                // the kernel's own decision (before a forced draw)
    if (alive) {
      // Eq. (6): the root's running sums (double precision), those of the
      // initial row for a belief created in this iteration, else the row.
      bool tie = false;
      if (sid == 0) {
        a = draw_cdf64(T.root_cdf, A, w.x);
        tie = (k > 1 || P.carry) && near_tie64(T.root_cdf, A, w.x, a);
      } else if (fresh) {
        if constexpr (AM <= 8) a = draw_cdf64_regs<AM>(cdf0, A, w.x);
        else a = draw_cdf64(T.psi0_cdf64, A, w.x);
      } else {
        a = draw_row32<AM>(row, A, P.eta, w.x, tie);
      }
      nt += tie ? 1u : 0u;
      own = a;
      if (T.dbg_force) {
        const short f = T.dbg_force[(size_t)(t0 + d - T.dbg_step0) * n_p + ep];
        if (f >= 0 && f < A) a = f;
      }
      bool term = false;
      if (!nav) {
        int sn;
        tabular_step(P.m, s, a, w, sn, obs, r);
        s = sn;
      } else {
        float nx, ny;
        nav_step_z(P.m, dc, x, y, a, z, nx, ny, obs, r, term);
        x = nx;
        y = ny;
      }
      ++g;
      // The next level's noise, issued before this level's insert.
      const U4 wn = draw(P, (uint32_t)ep, kTagStep, (uint32_t)(d + 1), (uint32_t)k);
      if (nav && !term && d + 1 < D) z = nav_noise(P.m, wn);
      // AppendBeliefs, first line: read with the previous insert in flight.
      Bucket bk;
      unsigned long long key = 0;
      if (!term) {
        key = belief_key(sid, a, obs, P.m.obs_bits);
        bucket_read(T, key, bk);
      }
      bool full = false;
      if (pend) {
        const uint32_t sid_guess = (uint32_t)sid;
        if (!settle()) {
          full = true;                          // the table is full: stop
        } else if (!term && (uint32_t)sid != sid_guess) {
          key = belief_key(sid, a, obs, P.m.obs_bits);
          bucket_read(T, key, bk);
        }
      }
      // AppendActions: visit count and reward sum of (b, a), counted below
      // when b's record is known, else left to the accumulate pass.
      direct = !full && d >= kDirectLevel && rid >= 0;
      if (!direct && !full)
        tk = rid >= 0 ? (((unsigned long long)(uint32_t)rid << kActBits) | (uint32_t)a | kTraceRec)
                      : (((unsigned long long)(uint32_t)sid << kActBits) | (uint32_t)a);
      link = rid >= 0 ? (((unsigned long long)(uint32_t)rid << kActBits) | (uint32_t)a)
                      : (kLinkSlot | ((unsigned long long)(uint32_t)sid << kActBits) | (uint32_t)a);
      const int rid_b = rid;
      if (term || full) {
        alive = false;                          // FilterTerminals
      } else {
        // AppendBeliefs: find or insert (b, a, o).
        bool fr = false;
        int id = -1;
        unsigned long long seen = 0;
        const int got = probe_line(T, bk, key, stamp, h, fr, id, seen);
        if (got == 2) {
          pend = true;
          pend_slot = h;
          pend_key = key;
          pend_seen = seen;
          pend_link = link;
          pend_t = t0 + d;
          pend_obs = obs;
          sid = (int)h + 1;
          fresh = true;
          rid = -1;
        } else {
          bool won = false;
          if (got == 0) h = probe(T, key, stamp, won, fr, id);   // the line is full
          if (h == ~0u) {                       // table full: stop and report
            atomicOr((unsigned int*)&T.counters[1], 2u);
            alive = false;
          } else {
            sid = (int)h + 1;
            fresh = fr;
            rid = won ? 1 + (t0 + d) * P.n_p + ep : id;   // the inserter's own record
            won_now = won;
          }
        }
        insert_now = pend;
      }
      // The next level's row (an existing belief's; a new one's is Psi0).
      w = wn;
      if (alive && d + 1 < D && !fresh) load_row<AM>(rec_psi(T, rid), A, row);
      // Writes of level d.
      if (direct) {
        atomicAdd(&rec_n(T, rid_b)[a], 1);
        const unsigned long long fx = to_fix(r, P.fix_scale);
        if (fx) atomicAdd(&rec_c(T, rid_b)[a], fx);
      }
    }
    if (ep_ok) {
      const int t = t0 + d;
      T.tr_key[(size_t)d * n_p + ep] = tk;
      T.tr_val[(size_t)d * n_p + ep] = r;
      if (!insert_now) T.list[(size_t)t * n_p + ep] = won_now ? sid : 0;
      if (won_now) {
        T.h_slot[h].id = rid;
        init_record(P, psi0s, rid, obs, link);
      }
      if (T.dbg_act) {
        const size_t i = (size_t)(t - T.dbg_step0) * n_p + ep;
        T.dbg_act[i] = drew ? (short)own : (short)-1;
        T.dbg_obs[i] = drew ? obs : -1;
      }
    }
  }
  if (pend && !settle()) alive = false;
  if (ep_ok) {
    unsigned long long tk = kEmptyKey;
    float hv = 0.0f;                            // ValueHeuristic of the leaf state
    if (alive) {
      if (!nav) {
        if (P.m.H) hv = P.m.H[s];
      } else {
        hv = nav_heuristic(P.m.nav, x, y);
      }
      if (D >= kDirectLevel && rid >= 0) {
        BeliefLeaf* lf = rec_leaf(T, rid);
        atomicAdd(&lf->leaf_cnt, 1);
        const unsigned long long fx = to_fix(hv, P.fix_scale);
        if (fx) atomicAdd(&lf->leaf_h, fx);
      } else {
        tk = rid >= 0 ? ((unsigned long long)(uint32_t)rid | kTraceRec)
                      : (unsigned long long)(uint32_t)sid;
      }
    }
    T.tr_key[(size_t)D * n_p + ep] = tk;
    T.tr_val[(size_t)D * n_p + ep] = hv;
  }
  // Both counts in one word: a block makes fewer than 2^32 of each.
  g = block_sum(g | (nt << 32), red);
  if (threadIdx.x == 0 && (g & 0xffffffffull))
    atomicAdd(&T.stats[blk % kStripes], g & 0xffffffffull);
  if (threadIdx.x == 0 && (g >> 32)) atomicAdd(&T.stats[kStatNear * kStripes + blk % kStripes], g >> 32);
}

// The forward search of the batched kernels: the same decisions, draws and
// writes as dev_forward, with each insert settled before the next level.  A
// batched kernel holds the registers of its largest phase, and carrying an
// unsettled insert across levels (dev_forward) would cost it half its
// wavefronts per SIMD.
template <int AM>
__device__ void dev_forward_inorder(const PlanView& P, int k, int D, int blk,
                                    unsigned long long* red, float* psi0s) {
  const TreeView& T = P.t;
  // The initial row in LDS, copied into new records (every thread of the
  // block calls).
  for (int i = threadIdx.x; i < T.ra; i += kBlock) psi0s[i] = T.psi0[i];
  __syncthreads();
  const int t0 = T.step_base[k - 1];          // level step of level 0
  const int ep = blk * kBlock + threadIdx.x;
  const bool ep_ok = ep < P.n_p;
  const int A = P.m.nA;
  const bool nav = P.m.kind != kTabular;
  const size_t n_p = (size_t)P.n_p;
  const unsigned long long stamp = (unsigned long long)(k - 1) << kStampShift;
  int s = 0;
  float x = 0.0f, y = 0.0f;
  int sid = 0;                // current belief's slot id (0: root)
  int rid = 0;                // its record, -1 if another episode inserted it
                              // during this iteration
  bool fresh = false;         // inserted during this iteration (Psi initial)
  bool alive = false;
  if (ep_ok) {
    // Alg. 1: the episode starts at the root with a state drawn from the
    // belief particles.
    const U4 w = draw(P, (uint32_t)ep, kTagRoot, 0, (uint32_t)k);
    const uint32_t idx = __umulhi(w.x, (uint32_t)P.e.n_belief);
    if (!nav) {
      s = ((const int*)P.e.belief)[idx];
      if ((unsigned)s >= (unsigned)P.m.nS) {   // caller's particle out of range
        atomicOr((unsigned int*)&T.counters[1], 1u);
        s = 0;
      }
    } else {
      const float* bf = (const float*)P.e.belief;
      x = bf[idx];
      y = bf[P.e.n_belief + idx];
    }
    alive = true;
  }
  // Inputs of the next level, read ahead of the previous level's writes: a
  // wait for a load also waits for every memory operation issued before it.
  U4 w = draw(P, (uint32_t)ep, kTagStep, 0u, (uint32_t)k);
  float row[AM];
#pragma unroll
  for (int j = 0; j < AM; ++j) row[j] = 0.0f;
  NavNoise z{0.0f, 0.0f, 0.0f, 0.0f};
  if (alive && nav) z = nav_noise(P.m, w);
  DiskCache dc;
#pragma unroll
  for (int i = 0; i < 2 * kDiskRegs; ++i) dc.c[i] = 0.0f;
  if (nav) dc = load_disks(P.m);
  unsigned long long g = 0;   // generative-model calls of this episode
  unsigned long long nt = 0;  // its near-tie draws
  for (int d = 0; d < D; ++d) {
    unsigned long long tk = kEmptyKey;
    float r = 0.0f;
    bool won = false, direct = false;
    int obs = 0, a = 0;
    uint32_t h = 0;
    unsigned long long link = kEmptyKey;
    const int rid_b = rid;
    const bool drew = alive;
    int own = 0;                // the kernel's own decision (before a forced draw)
    if (alive) {
      // Eq. (6): the root's running sums (double precision), those of the
      // initial row for a belief created in this iteration, else the row.
      bool tie = false;
      if (sid == 0) {
        a = draw_cdf64(T.root_cdf, A, w.x);
        tie = (k > 1 || P.carry) && near_tie64(T.root_cdf, A, w.x, a);
      } else if (fresh) {
        a = draw_cdf64(T.psi0_cdf64, A, w.x);
      } else {
        a = draw_row32<AM>(row, A, P.eta, w.x, tie);
      }
      nt += tie ? 1u : 0u;
      own = a;
      if (T.dbg_force) {
        const short f = T.dbg_force[(size_t)(t0 + d - T.dbg_step0) * n_p + ep];
        if (f >= 0 && f < A) a = f;
      }
      bool term = false;
      if (!nav) {
        int sn;
        tabular_step(P.m, s, a, w, sn, obs, r);
        s = sn;
      } else {
        float nx, ny;
        nav_step_z(P.m, dc, x, y, a, z, nx, ny, obs, r, term);
        x = nx;
        y = ny;
      }
      ++g;
      // AppendActions: visit count and reward sum of (b, a), counted below
      // when b's record is known, else left to the accumulate pass.
      direct = d >= kDirectLevel && rid >= 0;
      if (!direct)
        tk = rid >= 0 ? (((unsigned long long)(uint32_t)rid << kActBits) | (uint32_t)a | kTraceRec)
                      : (((unsigned long long)(uint32_t)sid << kActBits) | (uint32_t)a);
      link = rid >= 0 ? (((unsigned long long)(uint32_t)rid << kActBits) | (uint32_t)a)
                      : (kLinkSlot | ((unsigned long long)(uint32_t)sid << kActBits) | (uint32_t)a);
      if (term) {
        alive = false;                          // FilterTerminals
      } else {
        // AppendBeliefs: find or insert (b, a, o).
        const unsigned long long key = belief_key(sid, a, obs, P.m.obs_bits);
        bool fr;
        int id;
        h = probe(T, key, stamp, won, fr, id);
        if (h == ~0u) {                         // table full: stop and report
          atomicOr((unsigned int*)&T.counters[1], 2u);
          alive = false;
        } else {
          sid = (int)h + 1;
          fresh = fr;
          rid = won ? 1 + (t0 + d) * P.n_p + ep : id;   // the inserter's own record
        }
      }
    }
    if (alive && d + 1 < D) {
      w = draw(P, (uint32_t)ep, kTagStep, (uint32_t)(d + 1), (uint32_t)k);
      if (!fresh) load_row<AM>(rec_psi(T, rid), A, row);
      if (nav) z = nav_noise(P.m, w);
    }
    // Writes of level d.
    if (direct) {
      atomicAdd(&rec_n(T, rid_b)[a], 1);
      const unsigned long long fx = to_fix(r, P.fix_scale);
      if (fx) atomicAdd(&rec_c(T, rid_b)[a], fx);
    }
    if (ep_ok) {
      const int t = t0 + d;
      T.tr_key[(size_t)d * n_p + ep] = tk;
      T.tr_val[(size_t)d * n_p + ep] = r;
      T.list[(size_t)t * n_p + ep] = won ? sid : 0;
      if (won) {
        T.h_slot[h].id = rid;
        init_record(P, psi0s, rid, obs, link);
      }
      if (T.dbg_act) {
        const size_t i = (size_t)(t - T.dbg_step0) * n_p + ep;
        T.dbg_act[i] = drew ? (short)own : (short)-1;
        T.dbg_obs[i] = drew ? obs : -1;
      }
    }
  }
  if (ep_ok) {
    unsigned long long tk = kEmptyKey;
    float hv = 0.0f;                            // ValueHeuristic of the leaf state
    if (alive) {
      if (!nav) {
        if (P.m.H) hv = P.m.H[s];
      } else {
        hv = nav_heuristic(P.m.nav, x, y);
      }
      if (D >= kDirectLevel && rid >= 0) {
        BeliefLeaf* lf = rec_leaf(T, rid);
        atomicAdd(&lf->leaf_cnt, 1);
        const unsigned long long fx = to_fix(hv, P.fix_scale);
        if (fx) atomicAdd(&lf->leaf_h, fx);
      } else {
        tk = rid >= 0 ? ((unsigned long long)(uint32_t)rid | kTraceRec)
                      : (unsigned long long)(uint32_t)sid;
      }
    }
    T.tr_key[(size_t)D * n_p + ep] = tk;
    T.tr_val[(size_t)D * n_p + ep] = hv;
  }
  // Both counts in one word: a block makes fewer than 2^32 of each.
  g = block_sum(g | (nt << 32), red);
  if (threadIdx.x == 0 && (g & 0xffffffffull))
    atomicAdd(&T.stats[blk % kStripes], g & 0xffffffffull);
  if (threadIdx.x == 0 && (g >> 32)) atomicAdd(&T.stats[kStatNear * kStripes + blk % kStripes], g >> 32);
}

// ---------------------------------------------------------------------------
// Phase: fold the trace of an iteration with D levels into the records.
// Aggregation keys: (record << (kActBits + 1)) | (a << 1) for action nodes,
// (record << (kActBits + 1)) | 1
// for leaves.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int record_of(const TreeView& T, int sid) {
  return sid == 0 ? 0 : T.h_slot[sid - 1].id;
}

// Stripe q (0: N, 1: C, 2: W) of root action a for the calling block.
__device__ __forceinline__ unsigned long long* root_stripe(const TreeView& T, int q, int a) {
  // Long rows spread the root's visits over many actions: no striping there.
  const int stripe = T.ra > kMaxA ? 0 : (int)(blockIdx.x % kStripes);
  return T.root_acc + ((size_t)q * T.ra + a) * kStripes + stripe;
}

// Long rows: the first visit of each (b, a) in the trace of an iteration
// sets bit a of b's bitmap and clears N[a], C[a] and W[a] (the root keeps its
// sums elsewhere).  It runs before the accumulate pass adds the visits.
__global__ __launch_bounds__(kBlock) void k_claim_wide(PlanView P, int D) {
  if (budget_spent(P)) return;
  const TreeView& T = P.t;
  const long long n = (long long)D * P.n_p;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const unsigned long long tk = T.tr_key[i];
    if (tk == kEmptyKey) continue;
    const unsigned long long body = tk & ~kTraceRec;
    const int id = (int)(body >> kActBits);
    const int rid = (tk & kTraceRec) ? id : record_of(T, id);
    if (rid == 0) continue;
    const int a = (int)(body & kActMask);
    const uint32_t bit = 1u << (a & 31);
    if (!(atomicOr(&rec_bits(T, rid)[a >> 5], bit) & bit)) {
      rec_n(T, rid)[a] = 0;
      rec_c(T, rid)[a] = 0ull;
      rec_w(T, rid)[a] = 0ull;
    }
  }
}

__device__ void dev_accum(const PlanView& P, int D, int blk, int nblk, Smem& sm) {
  const TreeView& T = P.t;
  AggTable& G = sm.agg;
  const size_t n_p = (size_t)P.n_p;
  const int per = (P.n_p + kBlock - 1) / kBlock;   // chunks of kBlock items per level
  for (int c = blk; c < (D + 1) * per; c += nblk) {
    const int lvl = c / per;
    const int ep = (c - lvl * per) * kBlock + threadIdx.x;
    const size_t i = (size_t)lvl * n_p + (size_t)ep;
    unsigned long long tk = kEmptyKey;
    float v = 0.0f;
    if (ep < P.n_p) tk = T.tr_key[i];
    const bool has = tk != kEmptyKey;
    const bool leaf = lvl == D;
    unsigned long long key = kEmptyKey;
    if (has) {
      v = T.tr_val[i];
      const unsigned long long body = tk & ~kTraceRec;
      const int id = (int)(leaf ? body : body >> kActBits);
      const int rid = (tk & kTraceRec) ? id : record_of(T, id);
      key = ((unsigned long long)(uint32_t)rid << (kActBits + 1)) |
            (leaf ? 1ull : ((body & kActMask) << 1));
    }
    if (__syncthreads_or(has)) {
      agg_clear(G);
      __syncthreads();
      if (has) {
        const int sl = agg_slot(G, key);
        atomicAdd(&G.a[sl], 1ull);
        const unsigned long long fx = to_fix(v, P.fix_scale);
        if (fx) atomicAdd(&G.b[sl], fx);
      }
      __syncthreads();
      for (int j = threadIdx.x; j < kAggSlots; j += kBlock) {
        const unsigned long long k2 = G.key[j];
        if (k2 == kEmptyKey) continue;
        const int rid = (int)(k2 >> (kActBits + 1));
        if (k2 & 1ull) {
          BeliefLeaf* lf = rec_leaf(T, rid);
          atomicAdd(&lf->leaf_cnt, (int)G.a[j]);
          if (G.b[j]) atomicAdd(&lf->leaf_h, G.b[j]);
        } else if (rid == 0) {
          const int a = (int)((k2 >> 1) & kActMask);
          atomicAdd(root_stripe(T, 0, a), G.a[j]);
          if (G.b[j]) atomicAdd(root_stripe(T, 1, a), G.b[j]);
        } else {
          const int a = (int)((k2 >> 1) & kActMask);
          atomicAdd(&rec_n(T, rid)[a], (int)G.a[j]);
          if (G.b[j]) atomicAdd(&rec_c(T, rid)[a], G.b[j]);
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Backup (Alg. 3).  Beliefs of depth `dep` were created by level dep-1 of
// every iteration k' <= k whose depth D_k' >= dep.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_ranges(const PlanView& P, int dep, int k, Ranges& R) {
  if (threadIdx.x == 0) {
    int n = 0;
    if (P.carry) {                              // a kept subtree's steps first
      const int f = P.t.carry_rng[2 * dep], c = P.t.carry_rng[2 * dep + 1];
      for (int i = 0; i < c; ++i) R.step[n++] = f + i;
    }
    for (int kk = 1; kk <= k; ++kk) {
      const int s0 = P.t.step_base[kk - 1];
      const int Dk = P.t.step_base[kk] - s0;
      if (Dk >= dep) R.step[n++] = s0 + dep - 1;
    }
    R.n = n;
  }
  __syncthreads();
}

// The parent link of a record, resolved to (record << kActBits) | a (written
// back); par is the stored link, read by the caller.
__device__ __forceinline__ unsigned long long resolve_link(const TreeView& T, BeliefHot* mt,
                                                          unsigned long long par) {
  if (par != kEmptyKey && (par & kLinkSlot)) {
    const int psid = (int)((par & ~kLinkSlot) >> kActBits);
    par = ((unsigned long long)(uint32_t)record_of(T, psid) << kActBits) | (par & kActMask);
    mt->parent = par;
  }
  return par;
}

// Record of position ep of level step t, or -1 if no belief was inserted there.
__device__ __forceinline__ int record_at(const PlanView& P, int t, int ep) {
  const size_t pos = (size_t)t * (size_t)P.n_p + (size_t)ep;
  return P.t.list[pos] ? (int)(1 + pos) : -1;
}

// Push V*N_b of a belief into its parent action's W accumulator (parent =
// (record << kActBits) | a, or kEmptyKey for none).  Beliefs of depth >= 3 mostly
// have distinct parents, so they add directly; shallower ones share a few
// parents and are combined per block first (then every thread of the block
// must call, as it contains barriers; `shared` is uniform).
constexpr int kPushDirectDepth = 3;

__device__ __forceinline__ void push_values(const PlanView& P, AggTable& G, bool shared,
                                            unsigned long long parent, float V, int N) {
  unsigned long long f = 0ull;
  if (parent != kEmptyKey && N > 0) f = to_fix(V * (float)N, P.fix_scale);
  if (!shared) {
    if (f) {
      const int pr = (int)(parent >> kActBits), a = (int)(parent & kActMask);
      if (pr == 0) atomicAdd(root_stripe(P.t, 2, a), f);
      else atomicAdd(&rec_w(P.t, pr)[a], f);
    }
    return;
  }
  if (!__syncthreads_or(f != 0ull)) return;   // uniform: nothing to push
  agg_clear(G);
  __syncthreads();
  if (f) atomicAdd(&G.a[agg_slot(G, parent)], f);
  __syncthreads();
  for (int j = threadIdx.x; j < kAggSlots; j += kBlock) {
    const unsigned long long key = G.key[j];
    if (key != kEmptyKey && G.a[j]) {
      const int pr = (int)(key >> kActBits), a = (int)(key & kActMask);
      if (pr == 0) atomicAdd(root_stripe(P.t, 2, a), G.a[j]);
      else atomicAdd(&rec_w(P.t, pr)[a], G.a[j]);
    }
  }
  __syncthreads();
}

// Leaves of this iteration take count and mean heuristic; every belief of
// depth D pushes V*N_b to its parent action.
__device__ void dev_backup_leaf(const PlanView& P, int dep, int k, int blk, int nblk,
                                Smem& sm) {
  Ranges& R = sm.ranges;
  load_ranges(P, dep, k, R);
  unsigned long long beliefs = 0;             // tree statistics (last iteration)
  // Chunks of kBlock positions: chunk c is block c % per of range c / per
  // (a division per chunk, on the scalar unit).
  const int per = (P.n_p + kBlock - 1) / kBlock;
  for (int c = blk; c < R.n * per; c += nblk) {
    const int r = c / per;
    const int ep = (c - r * per) * kBlock + threadIdx.x;
    int N = 0;
    float V = 0.0f;
    unsigned long long parent = kEmptyKey;
    const int b = ep < P.n_p ? record_at(P, R.step[r], ep) : -1;
    if (b > 0) {
      // Every field is read before the first store: on CDNA a wait for a
      // load also waits for the stores issued before it.
      BeliefHot* mt = rec_hot(P.t, b);
      BeliefLeaf* lf = rec_leaf(P.t, b);
      const int c = lf->leaf_cnt;
      const unsigned long long hs = lf->leaf_h;
      const float V0 = mt->V;
      const int N0 = mt->Nb;
      const unsigned long long par = mt->parent;
      if (c > 0) {
        V = from_fix(hs, P.fix_inv) / (float)c;
        N = c;
        mt->V = V;
        mt->Nb = N;
        lf->leaf_cnt = 0;
        if (hs) lf->leaf_h = 0ull;
      } else {
        V = V0;
        N = N0;
      }
      parent = resolve_link(P.t, mt, par);
      ++beliefs;
    }
    push_values(P, sm.agg, dep < kPushDirectDepth, parent, V, N);
  }
  if (counts_tree(P, k)) {
    beliefs = block_sum(beliefs, sm.wave);
    if (threadIdx.x == 0 && beliefs) atomicAdd(&stat_bank(P, k)[kStripes + blk % kStripes], beliefs);
  }
}

// Internal beliefs of depth dep-1 >= 1.  AM >= |A| keeps the row in registers.
template <int AM>
__device__ void dev_backup_level(const PlanView& P, int dep, int k, int blk, int nblk,
                                 Smem& sm) {
  Ranges& R = sm.ranges;
  load_ranges(P, dep - 1, k, R);
  const int A = P.m.nA;
  const float gamma = P.m.gamma, eta = P.eta, inv = P.fix_inv;
  unsigned long long nodes = 0, beliefs = 0;  // tree statistics (last iteration)
  unsigned long long internal = 0;            // beliefs with an action node
  const int per = (P.n_p + kBlock - 1) / kBlock;
  for (int c = blk; c < R.n * per; c += nblk) {
    const int r = c / per;
    const int ep = (c - r * per) * kBlock + threadIdx.x;
    int N = 0;
    float V = 0.0f;
    unsigned long long parent = kEmptyKey;
    const int b = ep < P.n_p ? record_at(P, R.step[r], ep) : -1;
    if (b > 0) {
      float* prow = rec_psi(P.t, b);
      const int* nrow = rec_n(P.t, b);
      unsigned long long* crow = rec_c(P.t, b);
      unsigned long long* wrow = rec_w(P.t, b);
      BeliefHot* mt = rec_hot(P.t, b);
      // Two rounds of loads, both before the belief's first store (a wait for
      // a load also waits for the stores issued before it): the hot fields
      // and the visit counts, then -- for a belief with an action node -- its
      // preference row and the C and W of its visited actions only.
      const uint4 hq = *reinterpret_cast<const uint4*>(mt);   // V, N_b, parent
      int n[AM];
#pragma unroll
      for (int j = 0; j < AM; j += 4) {
        int4 c = make_int4(0, 0, 0, 0);
        if (j < A) c = *reinterpret_cast<const int4*>(nrow + j);
        n[j] = c.x; n[j + 1] = c.y; n[j + 2] = c.z; n[j + 3] = c.w;
      }
      const float V0 = __uint_as_float(hq.x);
      const int N0 = (int)hq.y;
      const unsigned long long par = ((unsigned long long)hq.w << 32) | hq.z;
      float psi[AM];
      unsigned long long cf[AM], wf[AM];
#pragma unroll
      for (int j = 0; j < AM; ++j) { psi[j] = 0.0f; cf[j] = 0ull; wf[j] = 0ull; }
      bool any = false;
#pragma unroll
      for (int j = 0; j < AM; ++j) any = any || (j < A && n[j] > 0);
      if (any) {
#pragma unroll
        for (int j = 0; j < AM; j += 4) {
          float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          if (j < A) q = *reinterpret_cast<const float4*>(prow + j);
          psi[j] = q.x; psi[j + 1] = q.y; psi[j + 2] = q.z; psi[j + 3] = q.w;
        }
#pragma unroll
        for (int j = 0; j < AM; ++j)
          if (j < A && n[j] > 0) { cf[j] = crow[j]; wf[j] = wrow[j]; }
        // V_curr = L_eta Psi (Eq. 3) before the update.
        float m = psi[0];
#pragma unroll
        for (int j = 1; j < AM; ++j)
          if (j < A) m = fmaxf(m, psi[j]);
        float se = 0.0f;
#pragma unroll
        for (int j = 0; j < AM; ++j)
          if (j < A) se = se + expf(eta * (psi[j] - m));
        const float vc = m + logf(se) / eta;
        // Q = C/N + gamma W with W = sum_children V N_b / N; Psi <- Psi - V_curr + Q.
        int nsum = 0;
#pragma unroll
        for (int j = 0; j < AM; ++j) {
          if (j < A && n[j] > 0) {
            const float c = from_fix(cf[j], inv);
            const float w = from_fix(wf[j], inv);
            const float fn = (float)n[j];
            const float q = c / fn + gamma * (w / fn);
            psi[j] = (psi[j] - vc) + q;
            nsum += n[j];
          }
        }
        // V = L_eta Psi after the update; N_b = sum_a N(b, a).
        float m2 = psi[0];
#pragma unroll
        for (int j = 1; j < AM; ++j)
          if (j < A) m2 = fmaxf(m2, psi[j]);
        float se2 = 0.0f;
#pragma unroll
        for (int j = 0; j < AM; ++j)
          if (j < A) se2 = se2 + expf(eta * (psi[j] - m2));
        V = m2 + logf(se2) / eta;
        N = nsum;
#pragma unroll
        for (int j = 0; j < AM; j += 4)
          if (j < A)
            *reinterpret_cast<float4*>(prow + j) =
                make_float4(psi[j], psi[j + 1], psi[j + 2], psi[j + 3]);
        // W is rebuilt by the children's pushes of the next sweep.
#pragma unroll
        for (int j = 0; j < AM; ++j)
          if (j < A && n[j] > 0 && wf[j]) wrow[j] = 0ull;
        mt->V = V;
        mt->Nb = N;
        ++internal;
      } else {
        V = V0;
        N = N0;
      }
      parent = resolve_link(P.t, mt, par);
#pragma unroll
      for (int j = 0; j < AM; ++j) nodes += (j < A && n[j] > 0) ? 1ull : 0ull;
      ++beliefs;
    }
    push_values(P, sm.agg, dep - 1 < kPushDirectDepth, parent, V, N);
  }
  // The sweep's work over the plan (every iteration), then the tree
  // statistics (the last iteration).  A block visits fewer than 2^32 beliefs.
  const unsigned long long vi = block_sum(beliefs | (internal << 32), sm.wave);
  const unsigned long long nd = block_sum(nodes, sm.wave);
  if (threadIdx.x == 0) {
    unsigned long long* sw = P.t.stats + (size_t)kStatSweep * kStripes + blk % kStripes;
    if (vi & 0xffffffffull) atomicAdd(sw, vi & 0xffffffffull);
    if (vi >> 32) atomicAdd(sw + kStripes, vi >> 32);
    if (nd) atomicAdd(sw + 2 * kStripes, nd);
    if (counts_tree(P, k)) {
      unsigned long long* bank = stat_bank(P, k);
      if (nd) atomicAdd(&bank[blk % kStripes], nd);
      if (vi & 0xffffffffull) atomicAdd(&bank[kStripes + blk % kStripes], vi & 0xffffffffull);
    }
  }
}

// Anytime plan (Alg. 1 loops while the budget lasts), run by the first
// wavefront of the root backup: this iteration's backups are done; the next
// one runs only if time is left and K is not reached.  The decision goes to
// the later phases (gate) and to the host, which stops enqueueing.
__device__ __forceinline__ void root_gate(const PlanView& P, int k, int lane) {
  if (!P.timed) return;
  unsigned long long* next = stat_bank(P, k + 1);
  next[lane] = 0ull;
  next[kStripes + lane] = 0ull;
  if (lane == 0) {
    const unsigned long long now = (unsigned long long)wall_clock64();
    const unsigned long long stop =
        (k >= P.K || now - P.t.gate[0] >= P.budget_ticks) ? 1ull : 0ull;
    P.t.gate[1] = stop;
    P.t.gate[2] = (unsigned long long)k;
    __hip_atomic_store(P.gate_host, (unsigned long long)k | (stop << 32), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ---------------------------------------------------------------------------
// Sweeps for long action rows (|A| > kMaxA): one wavefront per belief; lane l
// holds the quads l, l + 64, ... of the row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Level sweep of the internal beliefs of depth dep-1 >= 1 (Alg. 3, Eq. 3, 5)
// over long rows, one wavefront per belief.  Lane l holds the quads l,
// l + 64, ... of the row (QPL of them; the padding past |A| and quads past the
// row masked off) in registers for the whole update, so a belief costs one
// batch of loads for Psi, N and its metadata, one batch of C and W loads per
// four quads of the lane, and the stores at the end: no load waits behind a
// store of the same belief.
constexpr int kWideChunk = 16;              // positions a wavefront scans at once

template <int QPL>
__device__ void dev_backup_level_wide(const PlanView& P, int dep, int k, int blk, int nblk,
                                      Smem& sm) {
  static_assert(QPL % 4 == 0 && 4 * QPL <= 64, "quads per lane");
  Ranges& R = sm.ranges;
  load_ranges(P, dep - 1, k, R);
  const TreeView& T = P.t;
  const int A = P.m.nA;
  const int nq = T.ra / 4;
  const float gamma = P.m.gamma, eta = P.eta, inv = P.fix_inv;
  const int lane = threadIdx.x & 63;
  const int waves = kBlock / 64;
  unsigned long long nodes = 0, beliefs = 0;  // tree statistics (lane 0 counts)
  unsigned long long internal = 0;            // beliefs with an action node
  // Each wavefront takes kWideChunk positions of one level step at a time and
  // visits the beliefs among them one after the other.
  const int per = (P.n_p + kWideChunk - 1) / kWideChunk;
  for (long long c = (long long)blk * waves + (threadIdx.x >> 6); c < (long long)R.n * per;
       c += (long long)nblk * waves) {
    const int r = (int)(c / per);
    const int ep = (int)(c - (long long)r * per) * kWideChunk + lane;
    const int bl = (lane < kWideChunk && ep < P.n_p) ? record_at(P, R.step[r], ep) : -1;
    unsigned long long todo = __ballot(bl > 0);
    while (todo) {
      // b is uniform: addresses are a scalar base plus 32-bit lane offsets.
      const int b = __builtin_amdgcn_readfirstlane(__shfl(bl, __ffsll((long long)todo) - 1, 64));
      todo &= todo - 1;
      const float4* p4 = reinterpret_cast<const float4*>(rec_psi(T, b));
      const uint32_t* bits = rec_bits(T, b);
      const int* nrow = rec_n(T, b);
      const unsigned long long* crow = rec_c(T, b);
      unsigned long long* wrow = rec_w(T, b);
      BeliefHot* mt = rec_hot(T, b);
      // Psi and the visited flags (the bitmap's nibble of each quad).
      float pf[4 * QPL];
      uint32_t vb[QPL];
#pragma unroll
      for (int i = 0; i < QPL; ++i) {
        const int q = lane + 64 * i;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        uint32_t w = 0u;
        if (q < nq) {
          v = p4[q];
          w = bits[q >> 3];
        }
        pf[4 * i] = v.x; pf[4 * i + 1] = v.y; pf[4 * i + 2] = v.z; pf[4 * i + 3] = v.w;
        vb[i] = w;
      }
      // Read after the row: these uniform values are moved to scalar
      // registers at once, which waits for them.
      const float V0 = mt->V;
      const int N0 = mt->Nb;
      const unsigned long long par = mt->parent;
#pragma unroll
      for (int i = 0; i < QPL; ++i) vb[i] = (vb[i] >> (4 * ((lane + 64 * i) & 7))) & 15u;
      bool vis = false;                         // padding is never visited
#pragma unroll
      for (int i = 0; i < QPL; ++i) vis = vis || vb[i] != 0u;
      float V;
      int N;
      const bool upd = __any(vis);
      unsigned long long clear = 0ull;          // W entries to clear (bit per action)
      uint32_t changed = 0u;                    // quads of Psi to store
      if (upd) {
        // V_curr = L_eta Psi (Eq. 3) before the update.
        float m = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4 * QPL; ++i)
          if (4 * (lane + 64 * (i >> 2)) + (i & 3) < A) m = fmaxf(m, pf[i]);
        m = wave_maxf(m);
        float se = 0.0f;
#pragma unroll
        for (int i = 0; i < 4 * QPL; ++i)
          if (4 * (lane + 64 * (i >> 2)) + (i & 3) < A) se = se + expf(eta * (pf[i] - m));
        const float vc = m + logf(wave_sumf(se)) / eta;
        // Psi <- Psi - V_curr + Q, Q = C/N + gamma W/N (Eq. 5), for visited
        // actions.  An unvisited action reads the belief's hot fields instead
        // (read above), so the loads issue without branches.
        const int* spare_n = reinterpret_cast<const int*>(mt);
        const unsigned long long* spare_l = &mt->parent;
        int nsum = 0, nn = 0;
#pragma unroll
        for (int i0 = 0; i0 < QPL; i0 += 4) {
          unsigned long long cf[16], wf[16];
          int nf[16];
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            const int i = 4 * i0 + t;
            const int j = 4 * (lane + 64 * (i >> 2)) + (i & 3);
            const bool v = (vb[i >> 2] >> (i & 3)) & 1u;
            nf[t] = *(v ? nrow + j : spare_n);
            cf[t] = *(v ? crow + j : spare_l);
            wf[t] = *(v ? wrow + j : spare_l);
          }
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            asm volatile("" : "+v"(nf[t]));
            asm volatile("" : "+v"(cf[t]));
            asm volatile("" : "+v"(wf[t]));
          }
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            const int i = 4 * i0 + t;
            if (((vb[i >> 2] >> (i & 3)) & 1u) && nf[t] > 0) {
              const float cv = from_fix(cf[t], inv);
              const float w = from_fix(wf[t], inv);
              const float fn = (float)nf[t];
              pf[i] = (pf[i] - vc) + (cv / fn + gamma * (w / fn));
              nsum += nf[t];
              ++nn;
              changed |= 1u << (i >> 2);
              if (wf[t]) clear |= 1ull << i;
            }
          }
        }
        // V = L_eta Psi after the update; N_b = sum_a N(b, a).
        float m2 = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4 * QPL; ++i)
          if (4 * (lane + 64 * (i >> 2)) + (i & 3) < A) m2 = fmaxf(m2, pf[i]);
        m2 = wave_maxf(m2);
        float se2 = 0.0f;
#pragma unroll
        for (int i = 0; i < 4 * QPL; ++i)
          if (4 * (lane + 64 * (i >> 2)) + (i & 3) < A) se2 = se2 + expf(eta * (pf[i] - m2));
        V = m2 + logf(wave_sumf(se2)) / eta;
        N = (int)wave_sum((unsigned long long)nsum);
        nodes += wave_sum((unsigned long long)nn);
        ++internal;
      } else {
        V = V0;
        N = N0;
      }
      if (lane == 0) {
        ++beliefs;
        const unsigned long long parent = resolve_link(T, mt, par);
        if (parent != kEmptyKey && N > 0) {
          const unsigned long long f = to_fix(V * (float)N, P.fix_scale);
          if (f) {
            const int pr = (int)(parent >> kActBits), a = (int)(parent & kActMask);
            if (pr == 0) atomicAdd(root_stripe(T, 2, a), f);
            else atomicAdd(&rec_w(T, pr)[a], f);
          }
        }
      }
      // The record's stores come last, so that nothing above waits for them.
      if (upd) {
        mt->V = V;                              // the same value in every lane
        mt->Nb = N;
        float4* pw4 = reinterpret_cast<float4*>(rec_psi(T, b));
#pragma unroll
        for (int i = 0; i < QPL; ++i)
          if ((changed >> i) & 1u)
            pw4[lane + 64 * i] = make_float4(pf[4 * i], pf[4 * i + 1], pf[4 * i + 2], pf[4 * i + 3]);
#pragma unroll
        for (int i = 0; i < 4 * QPL; ++i)
          if ((clear >> i) & 1ull) wrow[4 * (lane + 64 * (i >> 2)) + (i & 3)] = 0ull;
      }
    }
  }
  if (lane == 0) {
    unsigned long long* sw = T.stats + (size_t)kStatSweep * kStripes + blk % kStripes;
    if (beliefs) atomicAdd(sw, beliefs);
    if (internal) atomicAdd(sw + kStripes, internal);
    if (nodes) atomicAdd(sw + 2 * kStripes, nodes);
    if (counts_tree(P, k)) {
      unsigned long long* bank = stat_bank(P, k);
      if (nodes) atomicAdd(&bank[blk % kStripes], nodes);
      if (beliefs) atomicAdd(&bank[kStripes + blk % kStripes], beliefs);
    }
  }
}

__device__ double block_max64(double v, double* red) {
  v = wave_max64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < kBlock / 64; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// Running sums over a = 0 .. A-1 of exp(eta (x_a - m)), by a block scan over
// chunks of kBlock actions (wavefront scans, then the wavefront totals); with
// cdf set they are stored.  Every thread calls; all get the total.  The scan
// adds in a tree order rather than the serial one: the sums differ from the
// serial definition's by a few units in the last place (about 1e-15
// relative), far below the margin at which a root draw counts as a near tie.
__device__ double block_ordered_sum(const double* x, int A, double m, double eta, double* cdf,
                                    double* buf, double* bc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double carry = 0.0;
  for (int base = 0; base < A; base += kBlock) {
    const int j = base + (int)threadIdx.x;
    double v = j < A ? exp(eta * (x[j] - m)) : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double o = __shfl_up(v, off, 64);
      if (lane >= off) v += o;
    }
    if (lane == 63) buf[wv] = v;
    __syncthreads();
    double before = carry;
    for (int w = 0; w < wv; ++w) before += buf[w];
    double total = carry;
    for (int w = 0; w < kBlock / 64; ++w) total += buf[w];
    if (cdf && j < A) cdf[j] = before + v;
    carry = total;
    __syncthreads();
  }
  (void)bc;
  return carry;
}

// Running sums, in the order of block_ordered_sum, of exp(eta (x - m)) for a
// row whose entry j = i*kBlock + threadIdx.x is x[i] of the calling thread
// (held in registers); with cdf set they are stored.  Every thread calls;
// all get the total.
template <int PER>
__device__ double block_ordered_sum_regs(const double (&x)[PER], int A, double m, double eta,
                                         double* cdf, double* buf) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double carry = 0.0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int base = i * kBlock;
    if (base >= A) break;                       // uniform
    const int j = base + (int)threadIdx.x;
    double v = j < A ? exp(eta * (x[i] - m)) : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double o = __shfl_up(v, off, 64);
      if (lane >= off) v += o;
    }
    if (lane == 63) buf[wv] = v;
    __syncthreads();
    double before = carry;
    for (int w = 0; w < wv; ++w) before += buf[w];
    double total = carry;
    for (int w = 0; w < kBlock / 64; ++w) total += buf[w];
    if (cdf && j < A) cdf[j] = before + v;
    carry = total;
    __syncthreads();
  }
  return carry;
}

// The root row (|A| > kMaxA) in double precision, by one block.  Thread t
// holds actions t, t + kBlock, ... of the row and of the root's sums (one
// stripe for long rows) in registers: one batch of loads, the update and its
// sums (in the order of block_ordered_sum), then the stores, so that no load
// waits behind a store.
__device__ void dev_backup_root_wide(const PlanView& P, int k, double* buf) {
  constexpr int PER = kMaxAWide / kBlock;
  const TreeView& T = P.t;
  const int A = P.m.nA;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double eta = P.eta64;
  __shared__ double red[kBlock / 64];
  __shared__ unsigned long long cnt[2];
  if (wv == 0) root_gate(P, k, lane);
  if (threadIdx.x == 0) { cnt[0] = 0ull; cnt[1] = 0ull; }
  double* psi = T.psi_root;
  double pv[PER];
  int nv[PER];
  unsigned long long cv[PER], wv64[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = i * kBlock + (int)threadIdx.x;
    pv[i] = -INFINITY;
    nv[i] = 0;
    cv[i] = 0ull;
    wv64[i] = 0ull;
    if (j < A) {
      pv[i] = psi[j];
      nv[i] = (int)T.root_acc[((size_t)0 * T.ra + j) * kStripes];
      cv[i] = T.root_acc[((size_t)1 * T.ra + j) * kStripes];
      wv64[i] = T.root_acc[((size_t)2 * T.ra + j) * kStripes];
    }
  }
  double mloc = -INFINITY;
  unsigned long long nodes = 0, nsum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    mloc = fmax(mloc, pv[i]);
    nodes += nv[i] > 0 ? 1ull : 0ull;
    nsum += (unsigned long long)(nv[i] > 0 ? nv[i] : 0);
  }
  nodes = wave_sum(nodes);
  nsum = wave_sum(nsum);
  __syncthreads();                              // cnt cleared
  if (lane == 0) {
    atomicAdd(&cnt[0], nodes);
    atomicAdd(&cnt[1], nsum);
  }
  const double m = block_max64(mloc, red);
  const bool any = cnt[0] != 0ull;              // uniform: an action node exists
  double vc = 0.0, mm = 0.0, run = 0.0;
  if (any) {
    // V_curr = L_eta Psi before the update (Eq. 3).
    vc = m + log(block_ordered_sum_regs<PER>(pv, A, m, eta, nullptr, buf)) / eta;
    // Psi <- Psi - V_curr + Q for the actions with an action node (Eq. 5).
    double m2 = -INFINITY;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (nv[i] > 0) {
        const double c = (double)(long long)cv[i] * P.fix_inv64;
        const double w = (double)(long long)wv64[i] * P.fix_inv64;
        pv[i] = (pv[i] - vc) + (c / (double)nv[i] + P.m.gamma64 * (w / (double)nv[i]));
      }
      m2 = fmax(m2, pv[i]);
    }
    mm = block_max64(m2, red);
    // V = L_eta Psi after the update, and the running sums of the root draw.
    run = block_ordered_sum_regs<PER>(pv, A, mm, eta, T.root_cdf, buf);
  }
  // The root record's columns (N, C, W) and the updated row; W's stripe is
  // cleared for the next iteration.
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = i * kBlock + (int)threadIdx.x;
    if (j < A) {
      rec_n(T, 0)[j] = nv[i];
      rec_c(T, 0)[j] = cv[i];
      rec_w(T, 0)[j] = wv64[i];
      T.root_acc[((size_t)2 * T.ra + j) * kStripes] = 0ull;
      if (any && nv[i] > 0) psi[j] = pv[i];
    }
  }
  if (any && threadIdx.x == 0) {
    const double v = mm + log(run) / eta;
    T.v_root[0] = v;
    BeliefHot* mt = rec_hot(T, 0);
    mt->V = (float)v;
    mt->Nb = (int)cnt[1];
    if (counts_tree(P, k)) atomicAdd(&stat_bank(P, k)[0], cnt[0]);
  }
}

// The root row in double precision, updated in place (one thread).
// Run by the block's first wavefront.  Lane s sums stripe s of the root's
// action nodes; lane j then owns action j: it evaluates that action's
// exponentials, and lane 0 adds them up in action order (the order of the
// serial definition, so every sum rounds exactly as it would there).

// Sum of x over lanes 0..A-1 in lane order, broadcast to the wave.
__device__ __forceinline__ double ordered_sum(double x, int A) {
  double s = 0.0;
  for (int j = 0; j < A; ++j) s = s + __shfl(x, j, 64);
  return s;
}

__device__ void dev_backup_root(const PlanView& P, int k) {
  if (threadIdx.x >= 64) return;
  const int A = P.m.nA;
  const int lane = threadIdx.x;
  root_gate(P, k, lane);
  const bool act = lane < A;
  unsigned long long* acc = P.t.root_acc;
  long long n_me = 0, c_me = 0, w_me = 0;     // sums of action `lane`
  for (int j = 0; j < A; ++j) {
    unsigned long long* w = &acc[((size_t)2 * P.t.ra + j) * kStripes + lane];
    const unsigned long long n = wave_sum(acc[((size_t)0 * P.t.ra + j) * kStripes + lane]);
    const unsigned long long c = wave_sum(acc[((size_t)1 * P.t.ra + j) * kStripes + lane]);
    const unsigned long long wv = wave_sum(*w);
    *w = 0ull;
    if (lane == j) {
      n_me = (long long)n;
      c_me = (long long)c;
      w_me = (long long)wv;
    }
  }
  double* psi = P.t.psi_root;
  const double eta = P.eta64;
  const double p_me = act ? psi[lane] : -INFINITY;
  if (act) {                                  // record 0 keeps the totals
    rec_n(P.t, 0)[lane] = (int)n_me;
    rec_c(P.t, 0)[lane] = (unsigned long long)c_me;
  }
  const int nodes = __popcll(__ballot(act && n_me > 0));
  if (counts_tree(P, k) && lane == 0) atomicAdd(&stat_bank(P, k)[0], (unsigned long long)nodes);
  if (nodes == 0) return;
  // V_curr = L_eta Psi before the update (Eq. 3).
  const double m = wave_max64(p_me);
  const double vc = m + log(ordered_sum(act ? exp(eta * (p_me - m)) : 0.0, A)) / eta;
  // Psi <- Psi - V_curr + Q for the actions with an action node (Eq. 5).
  double p_new = p_me;
  if (act && n_me > 0) {
    const double c = (double)c_me * P.fix_inv64;
    const double w = (double)w_me * P.fix_inv64;
    const double q = c / (double)n_me + P.m.gamma64 * (w / (double)n_me);
    p_new = (p_me - vc) + q;
    psi[lane] = p_new;
  }
  // V = L_eta Psi after the update, and the running sums of the root draw.
  const double m2 = wave_max64(act ? p_new : -INFINITY);
  const double e2 = act ? exp(eta * (p_new - m2)) : 0.0;
  double run = 0.0;
  for (int j = 0; j < A; ++j) {
    run = run + __shfl(e2, j, 64);
    if (lane == 0) P.t.root_cdf[j] = run;
  }
  const long long nsum = (long long)wave_sum((unsigned long long)n_me);
  if (lane != 0) return;
  const double v = m2 + log(run) / eta;
  P.t.v_root[0] = v;
  BeliefHot* mt = rec_hot(P.t, 0);
  mt->V = (float)v;
  mt->Nb = (int)nsum;
}

// Alg. 1: argmax of the root preferences (lowest index on ties) and the
// result record; also keeps this plan's list lengths for the next set-up.
// Run by the block's first wavefront (64 lanes, one per stripe).
__device__ void dev_select(const PlanView& P) {
  static_assert(kStripes == 64, "one lane per stripe");
  if (threadIdx.x >= 64) return;
  const TreeView& T = P.t;
  const int lane = threadIdx.x;
  const int k_last = P.timed ? (int)T.gate[2] : P.K;   // iterations that ran
  const unsigned long long* bank = stat_bank(P, k_last);
  const unsigned long long steps = wave_sum(T.stats[lane]);
  const unsigned long long nodes = wave_sum(bank[lane]);
  const unsigned long long nb = 1 + wave_sum(bank[kStripes + lane]);
  const unsigned long long near = wave_sum(T.stats[kStatNear * kStripes + lane]);
  const unsigned long long sw_v = wave_sum(T.stats[kStatSweep * kStripes + lane]);
  const unsigned long long sw_i = wave_sum(T.stats[(kStatSweep + 1) * kStripes + lane]);
  const unsigned long long sw_n = wave_sum(T.stats[(kStatSweep + 2) * kStripes + lane]);
  const int A = P.m.nA;
  double* out = P.out;
  // Argmax with the lowest index on ties: each lane scans actions lane,
  // lane + 64, ..., then the wavefront keeps the larger value, or the lower
  // index of equal values.
  int best = lane < A ? lane : 0;
  double bv = T.psi_root[best];
  for (int j = lane; j < A; j += 64) {
    const double v = T.psi_root[j];
    out[1 + j] = v;
    if (v > bv) { bv = v; best = j; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int ob = __shfl_xor(best, off, 64);
    if (ov > bv || (ov == bv && ob < best)) { bv = ov; best = ob; }
  }
  if (lane != 0) return;
  out[0] = (double)best;
  out[A + 1] = T.v_root[0];
  out[A + 2] = (double)steps;
  out[A + 3] = (double)nb;
  out[A + 4] = (double)nodes;
  out[A + 5] = (double)T.counters[1];
  out[A + 6] = (double)near;
  out[A + 7] = (double)sw_v;
  out[A + 8] = (double)sw_i;
  out[A + 9] = (double)sw_n;
  // The allocation-free entry point's result holds |A| + 10 values.
  if (!P.clear_all) out[A + 10] = (double)T.counters[4];
  T.counters[2] = nb;
  T.counters[3] = 0ull;
  T.counters[5] = (unsigned long long)(P.timed ? T.step_base[k_last] : P.steps);
  T.counters[6] = (unsigned long long)P.n_p;
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    unsigned long long n = __shfl_up(v, off, 64);
    if (lane >= off) v += n;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Served episodes: one step of the true environment, then the sequential
// importance resampling belief update tau(b, a, o) (Alg. 1, belief update).
// Likelihoods are exact integers, so every side draws the same particles:
//   tabular: thr_o - thr_{o-1} of the observation row Z(s', a, .);
//   navigation: the number of 12-bit noise indices per axis whose observation
//   falls in the observed grid cell (the cell is monotone in the index, so two
//   binary searches over the 4096-entry table count them), multiplied.
// Resampling is multinomial: a 64-bit Philox word u per new particle picks
// the particle whose inclusive weight sum first exceeds (u * total) >> 64.
// ---------------------------------------------------------------------------
__device__ void dev_env(const PlanView& P, int t) {
  if (threadIdx.x != 0) return;
  const int a = (int)P.out[0];                 // the action the last plan chose
  const U4 w = philox(0u, kTagEnv << 24, 0u, (uint32_t)t, P.f.env_seed_lo, P.f.env_seed_hi);
  int* env = P.f.env;
  int obs;
  float r;
  bool term = false;
  if (P.m.kind == kTabular) {
    int sn;
    tabular_step(P.m, env[0], a, w, sn, obs, r);
    env[0] = sn;
  } else {
    float nx, ny;
    nav_step(P.m, __int_as_float(env[0]), __int_as_float(env[1]), a, w, nx, ny, obs, r,
             term);
    env[0] = __float_as_int(nx);
    env[1] = __float_as_int(ny);
  }
  env[2] = obs;
  env[3] = a;
  env[4] = __float_as_int(r);
  env[5] = term ? 1 : 0;
}

// Number of table indices j whose observation nx + sd*G[j] falls in cell kx.
__device__ __forceinline__ unsigned nav_cell_count(const ModelView& m, float nx, float sd,
                                                   int kx) {
  // first j with cell(j) >= kx, and first j with cell(j) > kx
  int lo = 0, hi = 4096;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nav_axis(m.nav, nx + sd * m.gauss[mid]) >= kx) hi = mid; else lo = mid + 1;
  }
  const int first = lo;
  hi = 4096;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nav_axis(m.nav, nx + sd * m.gauss[mid]) > kx) hi = mid; else lo = mid + 1;
  }
  return (unsigned)(lo - first);
}

__device__ void dev_pf_weight(const PlanView& P, int t, int blk) {
  const int i = blk * kBlock + threadIdx.x;
  const int M = P.f.M;
  if (i >= M) return;
  const int a = P.f.env[3], o = P.f.env[2];
  const U4 x = philox((uint32_t)i, kTagPF << 24, 0u, (uint32_t)t, P.seed_lo, P.seed_hi);
  unsigned long long wt;
  if (P.m.kind == kTabular) {
    const int s = ((const int*)P.f.part)[i];
    const int sn = tabular_next(P.m, s, a, x.y);
    ((int*)P.f.prop)[i] = sn;
    const uint32_t* zr = P.m.thrZ + ((size_t)sn * P.m.nA + a) * P.m.nO;
    wt = (unsigned long long)(zr[o] - (o > 0 ? zr[o - 1] : 0u));
  } else {
    const float* pf = (const float*)P.f.part;
    float nx, ny;
    nav_move(P.m, pf[i], pf[M + i], a, x.y, nx, ny);
    float* q = (float*)P.f.prop;
    q[i] = nx;
    q[M + i] = ny;
    const float sd = nav_obs_sd(P.m.nav, nx);
    const int kn = P.m.nav.key_n;
    wt = (unsigned long long)nav_cell_count(P.m, nx, sd, o / kn) *
         (unsigned long long)nav_cell_count(P.m, ny, sd, o % kn);
  }
  P.f.w[i] = wt;
}

// In-place inclusive scan of the M weights by one block.
__device__ void dev_pf_scan(const PlanView& P, Smem& sm) {
  const int M = P.f.M;
  unsigned long long* w = P.f.w;
  unsigned long long carry = 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int base = 0; base < M; base += kBlock * 4) {
    unsigned long long v[4];
    unsigned long long mine = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + threadIdx.x * 4 + q;
      v[q] = i < M ? w[i] : 0ull;
      mine += v[q];
    }
    const unsigned long long incl = wave_incl_scan(mine);
    if (lane == 63) sm.wave[wid] = incl;
    __syncthreads();
    unsigned long long off = carry, tot = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      if (q < wid) off += sm.wave[q];
      tot += sm.wave[q];
    }
    unsigned long long run = off + incl - mine;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + threadIdx.x * 4 + q;
      run += v[q];
      if (i < M) w[i] = run;
    }
    carry += tot;
    __syncthreads();
  }
}

__device__ void dev_pf_resample(const PlanView& P, int t, int blk) {
  const int j = blk * kBlock + threadIdx.x;
  const int M = P.f.M;
  if (j >= M) return;
  const unsigned long long total = P.f.w[M - 1];
  int src = j;                                   // zero total: keep propagation
  if (total > 0ull) {
    const U4 y = philox((uint32_t)j, kTagResample << 24, 0u, (uint32_t)t, P.seed_lo,
                        P.seed_hi);
    const unsigned long long u = ((unsigned long long)y.x << 32) | y.y;
    const unsigned long long target = __umul64hi(u, total);
    int lo = 0, hi = M - 1;                      // first i with w[i] > target
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P.f.w[mid] > target) hi = mid; else lo = mid + 1;
    }
    src = lo;
  }
  if (P.m.kind == kTabular) {
    ((int*)P.f.part)[j] = ((const int*)P.f.prop)[src];
  } else {
    const float* q = (const float*)P.f.prop;
    float* pf = (float*)P.f.part;
    pf[j] = q[src];
    pf[M + j] = q[M + src];
  }
}

// ---------------------------------------------------------------------------
// Single-plan kernels (one launch per phase).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Forward search for long action rows (|A| > kMaxA, tabular models): one
// half wavefront per episode.  The episode's state is the same in every lane
// of the half; the lanes share the softmax draw (lane l owns the quads l,
// l + 32, ... of the row), the record initialisation, and lane 0 of the half
// does the episode's table probe and its scalar writes.  The draw of Eq. (6)
// takes single-precision weights exp(eta (psi_j - max)), sums each quad of
// four in double precision and keeps it rounded once to single precision (in
// LDS), and finds the first running sum above t = u * total by an inclusive
// double-precision scan over the half per chunk of 128 actions.  Every
// running sum is then within 2^-24 of itself (relative) of the sum of the
// single-precision weights, and a row whose entries are all equal gives
// floor(u |A|) exactly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float long_row_weight(float v, float m, float eta) {
  return expf(eta * (v - m));
}

// Long-row episodes run on half a wavefront (kHalf = 32 lanes), so that a
// wavefront carries two independent episodes: each is a chain of dependent
// reads, and two chains per wavefront hide twice as much of their latency.
// The helpers below reduce, scan and vote within the caller's half (lane is
// the lane within the half).
constexpr int kHalf = 32;

__device__ __forceinline__ float half_maxf(float v) {
#pragma unroll
  for (int off = kHalf / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kHalf));
  return v;
}
// Sum and inclusive scan over the half in double precision, in a fixed
// order (the same for every call).
__device__ __forceinline__ double half_sum64(double v) {
#pragma unroll
  for (int off = kHalf / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kHalf);
  return v;
}
__device__ __forceinline__ double half_incl_scan64(double v, int lane) {
#pragma unroll
  for (int off = 1; off < kHalf; off <<= 1) {
    const double n = __shfl_up(v, off, kHalf);
    if (lane >= off) v += n;
  }
  return v;
}
// Votes of the caller's half, bit l for lane l of the half.
__device__ __forceinline__ uint32_t half_ballot(bool p) {
  return (uint32_t)(__ballot(p) >> (threadIdx.x & kHalf));
}

// The long-row draw from the double-precision running sums of a row's softmax
// weights (A <= 4096): the first a with t < cdf[a], t = u * cdf[A - 1].  Lane
// l reads the end of run l of ceil(A / 32) actions; the half then reads the
// chosen run (at most 128 entries, four per lane, in order).  Two rounds of
// loads.
__device__ int draw_long_cdf(const double* __restrict__ cdf, int A, uint32_t x0, int lane) {
  const int step = (A + kHalf - 1) / kHalf;
  const double tot = cdf[A - 1];
  const int e = min((lane + 1) * step, A) - 1;
  const bool run_ok = lane * step < A;
  const double end = run_ok ? cdf[e] : 0.0;
  const double t = (double)(x0 >> 8) * (1.0 / 16777216.0) * tot;
  const uint32_t hit = half_ballot(run_ok && t < end);
  if (!hit) return A - 1;
  const int r = __ffs(hit) - 1;
  const int lo = r * step, hi = min(lo + step, A);
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = lo + u * kHalf + lane;
    v[u] = j < hi ? cdf[j] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = lo + u * kHalf + lane;
    const uint32_t h2 = half_ballot(j < hi && t < v[u]);
    if (h2) return lo + u * kHalf + (__ffs(h2) - 1);
  }
  return A - 1;
}

constexpr int kLongChunks = kMaxAWide / (4 * kHalf);   // chunks of 128 actions

// qs: this half's LDS area of kLongChunks * kHalf quad sums (single-precision
// bits).  near: t lies within kTieRel * total of a boundary next to it (rows
// whose entries are all equal never count).
__device__ int draw_long_row(const float* __restrict__ row, int A, float eta, uint32_t x0,
                             int lane, uint32_t* qs, bool& near) {
  // Lane l of the half holds the quads l, l + 32, ... (the row is padded to
  // a multiple of 4; padding is masked off).  Each weight is evaluated once:
  // the lane keeps its quad sum of every chunk (in LDS, for registers), the
  // half scans those once the total is known, and only the chosen quad is
  // evaluated again.
  const float4* r4 = reinterpret_cast<const float4*>(row);
  const int nq = (A + 3) / 4;
  const int nc = (nq + kHalf - 1) / kHalf;
  float m = -INFINITY, mn = INFINITY;
#pragma unroll 4
  for (int q = lane; q < nq; q += kHalf) {
    const float4 v = r4[q];
    const int j = 4 * q;
    m = fmaxf(m, v.x);
    mn = fminf(mn, v.x);
    if (j + 1 < A) { m = fmaxf(m, v.y); mn = fminf(mn, v.y); }
    if (j + 2 < A) { m = fmaxf(m, v.z); mn = fminf(mn, v.z); }
    if (j + 3 < A) { m = fmaxf(m, v.w); mn = fminf(mn, v.w); }
  }
  m = half_maxf(m);
  const bool flat = -half_maxf(-mn) == m;
  auto quad = [&](int q, float (&w)[4]) {
    const float4 v = r4[q];
    const int j = 4 * q;
    w[0] = long_row_weight(v.x, m, eta);
    w[1] = j + 1 < A ? long_row_weight(v.y, m, eta) : 0.0f;
    w[2] = j + 2 < A ? long_row_weight(v.z, m, eta) : 0.0f;
    w[3] = j + 3 < A ? long_row_weight(v.w, m, eta) : 0.0f;
  };
  double tot = 0.0;
  for (int c = 0; c < nc; ++c) {
    const int q = c * kHalf + lane;
    float sq = 0.0f;
    if (q < nq) {
      float w[4];
      quad(q, w);
      sq = (float)((((double)w[0] + (double)w[1]) + (double)w[2]) + (double)w[3]);
    }
    qs[c * kHalf + lane] = __float_as_uint(sq);
    tot += (double)sq;
  }
  tot = half_sum64(tot);
  const double t = (double)(x0 >> 8) * (1.0 / 16777216.0) * tot;
  double base = 0.0;
  for (int c = 0; c < nc; ++c) {
    const double sq = (double)__uint_as_float(qs[c * kHalf + lane]);
    const double incl = half_incl_scan64(sq, lane) + base;
    const uint32_t hit = half_ballot(c * kHalf + lane < nq && t < incl);
    if (hit) {
      const int src = __ffs(hit) - 1;
      int pick = 3;                             // within the chosen quad
      int tie = 0;
      if (lane == src) {
        float w[4];
        quad(c * kHalf + lane, w);
        double run = incl - sq, below = run;
        for (int u = 0; u < 4; ++u) {
          below = run;
          run += (double)w[u];
          if (t < run) { pick = u; break; }
        }
        if (pick == 3) run = incl;              // the quad's rounded sum bounds it
        const int a = 4 * (c * kHalf + lane) + pick;
        const double lim = kTieRel * tot;
        tie = !flat && ((a > 0 && t - below <= lim) || (a < A - 1 && run - t <= lim));
      }
      near = __shfl(tie, src, kHalf) != 0;
      return 4 * (c * kHalf + src) + __shfl(pick, src, kHalf);
    }
    base = __shfl(incl, kHalf - 1, kHalf);
  }
  near = false;
  return A - 1;
}

// Four wavefronts per SIMD (128 registers, a few spilled): each episode is a
// chain of dependent reads, so residency is what hides them.
__global__ __launch_bounds__(kBlock, 4) void k_forward_wide(PlanView P, int k, int D) {
  __shared__ unsigned long long red[kBlock / 64];
  __shared__ uint32_t qsum[kBlock / kHalf][kLongChunks * kHalf];
  if (budget_spent(P)) return;
  const TreeView& T = P.t;
  const int lane = threadIdx.x & (kHalf - 1);
  const int ep = blockIdx.x * (kBlock / kHalf) + (threadIdx.x / kHalf);   // uniform per half
  const bool ep_ok = ep < P.n_p;
  const int t0 = T.step_base[k - 1];
  const int A = P.m.nA;
  const size_t n_p = (size_t)P.n_p;
  const unsigned long long stamp = (unsigned long long)(k - 1) << kStampShift;
  int s = 0, sid = 0, rid = 0;
  bool fresh = false, alive = false;
  if (ep_ok) {
    const U4 w = draw(P, (uint32_t)ep, kTagRoot, 0, (uint32_t)k);
    const uint32_t idx = __umulhi(w.x, (uint32_t)P.e.n_belief);
    s = ((const int*)P.e.belief)[idx];
    if ((unsigned)s >= (unsigned)P.m.nS) {
      if (lane == 0) atomicOr((unsigned int*)&T.counters[1], 1u);
      s = 0;
    }
    alive = true;
  }
  unsigned long long g = 0, nt = 0;
  for (int d = 0; d < D; ++d) {
    unsigned long long tk = kEmptyKey, link = kEmptyKey;
    float r = 0.0f;
    bool won = false;
    int obs = 0, a = 0;
    uint32_t h = 0;
    const bool drew = alive;
    int own = 0;
    if (alive) {
      const U4 w = draw(P, (uint32_t)ep, kTagStep, (uint32_t)d, (uint32_t)k);
      bool tie = false;
      if (sid == 0) {
        a = draw_cdf64_bisect(T.root_cdf, A, w.x);
        tie = (k > 1 || P.carry) && near_tie64(T.root_cdf, A, w.x, a);
      } else if (fresh) {
        a = draw_long_cdf(T.psi0_cdf64, A, w.x, lane);
      } else {
        a = draw_long_row(rec_psi(T, rid), A, P.eta, w.x, lane, qsum[threadIdx.x / kHalf], tie);
      }
      nt += tie ? 1u : 0u;
      own = a;
      if (T.dbg_force) {
        const short f = T.dbg_force[(size_t)(t0 + d - T.dbg_step0) * n_p + ep];
        if (f >= 0 && f < A) a = f;
      }
      int sn;
      tabular_step(P.m, s, a, w, sn, obs, r);
      s = sn;
      ++g;
      // Every visit goes to the trace: the first visit of (b, a) clears its
      // columns in the claim pass, before any count is added.
      tk = rid >= 0 ? (((unsigned long long)(uint32_t)rid << kActBits) | (uint32_t)a | kTraceRec)
                    : (((unsigned long long)(uint32_t)sid << kActBits) | (uint32_t)a);
      link = rid >= 0 ? (((unsigned long long)(uint32_t)rid << kActBits) | (uint32_t)a)
                      : (kLinkSlot | ((unsigned long long)(uint32_t)sid << kActBits) | (uint32_t)a);
      // AppendBeliefs by lane 0 of the half; the outcome goes to the half.
      int fr = 0, id = -1, wn = 0;
      if (lane == 0) {
        bool b_won = false, b_fr = false;
        h = probe(T, belief_key(sid, a, obs, P.m.obs_bits), stamp, b_won, b_fr, id);
        wn = b_won;
        fr = b_fr;
      }
      h = __shfl(h, 0, kHalf);
      wn = __shfl(wn, 0, kHalf);
      fr = __shfl(fr, 0, kHalf);
      id = __shfl(id, 0, kHalf);
      won = wn != 0;
      if (h == ~0u) {
        if (lane == 0) atomicOr((unsigned int*)&T.counters[1], 2u);
        alive = false;
      } else {
        sid = (int)h + 1;
        fresh = fr != 0;
        rid = won ? 1 + (t0 + d) * P.n_p + ep : id;
      }
    }
    if (ep_ok) {
      if (lane == 0) {
        const int t = t0 + d;
        T.tr_key[(size_t)d * n_p + ep] = tk;
        T.tr_val[(size_t)d * n_p + ep] = r;
        T.list[(size_t)t * n_p + ep] = won ? sid : 0;
        if (won) T.h_slot[h].id = rid;
        if (T.dbg_act) {
          const size_t i = (size_t)(t - T.dbg_step0) * n_p + ep;
          T.dbg_act[i] = drew ? (short)own : (short)-1;
          T.dbg_obs[i] = drew ? obs : -1;
        }
      }
      if (won) {                                // the new record, by the half
        // Psi, the metadata and a cleared bitmap; N, C and W of (b, a) are
        // cleared by its first visit.
        uint4* q = reinterpret_cast<uint4*>(rec_psi(T, rid));
        const uint4* p0 = reinterpret_cast<const uint4*>(T.psi0);
        const int nq = T.ra / 4, nbq = rec_bitmap_quads(T.ra);
        for (int i = lane; i < nq; i += kHalf) q[i] = p0[i];
        if (lane == 0) {
          *rec_hot(T, rid) = BeliefHot{0.0f, 0, link};
          *rec_leaf(T, rid) = BeliefLeaf{0, obs, 0ull};
        }
        uint4* bq = reinterpret_cast<uint4*>(rec_bits(T, rid));
        for (int i = lane; i < nbq; i += kHalf) bq[i] = make_uint4(0u, 0u, 0u, 0u);
      }
    }
  }
  if (ep_ok && lane == 0) {
    unsigned long long tk = kEmptyKey;
    float hv = 0.0f;
    if (alive) {
      if (P.m.H) hv = P.m.H[s];
      if (D >= kDirectLevel && rid >= 0) {
        BeliefLeaf* lf = rec_leaf(T, rid);
        atomicAdd(&lf->leaf_cnt, 1);
        const unsigned long long fx = to_fix(hv, P.fix_scale);
        if (fx) atomicAdd(&lf->leaf_h, fx);
      } else {
        tk = rid >= 0 ? ((unsigned long long)(uint32_t)rid | kTraceRec)
                      : (unsigned long long)(uint32_t)sid;
      }
    }
    T.tr_key[(size_t)D * n_p + ep] = tk;
    T.tr_val[(size_t)D * n_p + ep] = hv;
  }
  g = block_sum(lane == 0 ? (g | (nt << 32)) : 0ull, red);
  if (threadIdx.x == 0 && (g & 0xffffffffull))
    atomicAdd(&T.stats[blockIdx.x % kStripes], g & 0xffffffffull);
  if (threadIdx.x == 0 && (g >> 32))
    atomicAdd(&T.stats[kStatNear * kStripes + blockIdx.x % kStripes], g >> 32);
}

__global__ void k_env(PlanView P, int t) { dev_env(P, t); }
__global__ __launch_bounds__(kBlock) void k_pf_weight(PlanView P, int t) {
  dev_pf_weight(P, t, blockIdx.x);
}
__global__ __launch_bounds__(kBlock) void k_pf_scan(PlanView P) {
  __shared__ Smem sm;
  dev_pf_scan(P, sm);
}
__global__ __launch_bounds__(kBlock) void k_pf_resample(PlanView P, int t) {
  dev_pf_resample(P, t, blockIdx.x);
}
__global__ __launch_bounds__(kBlock) void k_setup(PlanView P) {
  __shared__ SetupSmem ss;
  dev_setup(P, blockIdx.x, gridDim.x, &ss);
}
// The phases of one iteration return at once when a time budget ran out
// at the end of an earlier iteration.
template <int AM>
__global__ __launch_bounds__(kBlock) void k_forward(PlanView P, int k, int D) {
  __shared__ unsigned long long red[kBlock / 64];
  __shared__ float psi0s[kMaxA];
  if (budget_spent(P)) return;
  dev_forward<AM>(P, k, D, blockIdx.x, red, psi0s);
}
__global__ __launch_bounds__(kBlock) void k_accum(PlanView P, int D) {
  __shared__ Smem sm;
  if (budget_spent(P)) return;
  dev_accum(P, D, blockIdx.x, gridDim.x, sm);
}
__global__ __launch_bounds__(kBlock) void k_backup_leaf(PlanView P, int dep, int k) {
  __shared__ Smem sm;
  if (budget_spent(P)) return;
  dev_backup_leaf(P, dep, k, blockIdx.x, gridDim.x, sm);
}
template <int AM>
__global__ __launch_bounds__(kBlock) void k_backup_level(PlanView P, int dep, int k) {
  __shared__ Smem sm;
  if (budget_spent(P)) return;
  dev_backup_level<AM>(P, dep, k, blockIdx.x, gridDim.x, sm);
}
__global__ void k_backup_root(PlanView P, int k) {
  if (budget_spent(P)) return;
  dev_backup_root(P, k);
}
template <int QPL>
__global__ __launch_bounds__(kBlock) void k_backup_level_wide(PlanView P, int dep, int k) {
  __shared__ Smem sm;
  if (budget_spent(P)) return;
  dev_backup_level_wide<QPL>(P, dep, k, blockIdx.x, gridDim.x, sm);
}
__global__ __launch_bounds__(kBlock) void k_backup_root_wide(PlanView P, int k) {
  __shared__ double buf[kBlock];
  if (budget_spent(P)) return;
  dev_backup_root_wide(P, k, buf);
}
__global__ void k_select(PlanView P) { dev_select(P); }

// ---------------------------------------------------------------------------
// Batched kernel: block -> (instance, phase) through the item list, sorted by
// first block.  AMAX bounds the padded action count of the batch.
// ---------------------------------------------------------------------------
// One phase item of one instance, as block blk of its nblk (LDS in sm).
template <int AMAX>
__device__ __forceinline__ void run_item(const PlanView& P, const BatchItem& it, int blk,
                                         Smem& sm) {
  const int Apad = P.m.Apad;
  switch (it.kind) {
    case kPhaseSetup: dev_setup(P, blk, it.nblk, nullptr); break;   // |A| <= 16
    case kPhaseForward:
      if (Apad <= 4) {
        dev_forward_inorder<4>(P, it.a0, it.a1, blk, sm.wave, sm.psi0);
      } else if constexpr (AMAX >= 8) {
        if (Apad <= 8) dev_forward_inorder<8>(P, it.a0, it.a1, blk, sm.wave, sm.psi0);
        else if constexpr (AMAX >= 16) dev_forward_inorder<16>(P, it.a0, it.a1, blk, sm.wave, sm.psi0);
      }
      break;
    case kPhaseAccum: dev_accum(P, it.a0, blk, it.nblk, sm); break;
    case kPhaseLeaf: dev_backup_leaf(P, it.a0, it.a1, blk, it.nblk, sm); break;
    case kPhaseLevel:
      if (Apad <= 4) {
        dev_backup_level<4>(P, it.a0, it.a1, blk, it.nblk, sm);
      } else if constexpr (AMAX >= 8) {
        if (Apad <= 8) dev_backup_level<8>(P, it.a0, it.a1, blk, it.nblk, sm);
        else if constexpr (AMAX >= 16) dev_backup_level<16>(P, it.a0, it.a1, blk, it.nblk, sm);
      }
      break;
    case kPhaseRoot: dev_backup_root(P, it.a0); break;
    case kPhaseSelect: dev_select(P); break;
    case kPhaseEnv: dev_env(P, it.a0); break;
    case kPhasePFWeight: dev_pf_weight(P, it.a0, blk); break;
    case kPhasePFScan: dev_pf_scan(P, sm); break;
    case kPhasePFResample: dev_pf_resample(P, it.a0, blk); break;
    default: break;
  }
}

template <int AMAX>
__global__ __launch_bounds__(kBlock) void k_batch(const PlanView* __restrict__ views,
                                                  const BatchItem* __restrict__ items,
                                                  int n_items) {
  __shared__ Smem sm;
  const int g = blockIdx.x;
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].blk0 <= g) lo = mid; else hi = mid - 1;
  }
  const BatchItem it = items[lo];
  const int blk = g - it.blk0;
  if (blk >= it.nblk) return;          // uniform per block
  run_item<AMAX>(views[it.inst], it, blk, sm);
}

// The persistent batched launch.  Every block loops: take a tile (one block's
// share) of some instance's current phase from the queue, run it, and report
// it finished; the last finisher of a phase moves its instance to the next
// phase.  Taking a tile is one atomic add on the instance's word, whose old
// value names the phase and the tile together, so a block never runs a tile
// of a phase that has not started.  Memory order: each finisher releases its
// block's writes (agent scope) before it counts; the last finisher publishes
// the next phase with a release; a taker acquires after the add.  A block
// that finds no tile sleeps briefly and looks again; it returns once every
// instance is past its last phase.  Tiles never wait on anything, so every
// taken tile finishes and the queue drains whatever the residency.
__global__ void k_persist_reset(PersistView V) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < V.n) {
    V.word[i] = 0ull;
    V.done[i] = 0u;
  }
  if (i == 0) *V.finished = 0u;
}

template <int AMAX>
__global__ __launch_bounds__(kBlock) void k_batch_persistent(const PlanView* __restrict__ views,
                                                             PersistView V) {
  __shared__ Smem sm;
  __shared__ int take[3];
  int cur = (int)(blockIdx.x % (unsigned)V.n);
  for (;;) {
    if (threadIdx.x < 64) {
      // Wavefront 0 looks for a tile: its lanes read 64 instances' words at
      // once (this block's last instance first, then the others in turn), and
      // the instances with a tile left are tried in that order, one atomic
      // add each, until one yields a tile.
      const int lane = (int)threadIdx.x;
      int inst = -1, ph = 0, tile = 0;
      for (int base = 0; base < V.n && inst < 0; base += 64) {
        const int q = base + lane;
        int i = 0;
        bool avail = false;
        if (q < V.n) {
          i = cur + q < V.n ? cur + q : cur + q - V.n;
          const int np = V.ph_off[i + 1] - V.ph_off[i];
          const unsigned long long w =
              __hip_atomic_load(&V.word[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int g = (int)(w >> 32);
          avail = g < np && (unsigned)w < (unsigned)V.phases[V.ph_off[i] + g].nblk;
        }
        unsigned long long m = __ballot(avail);
        while (m && inst < 0) {
          const int src = __ffsll((long long)m) - 1;
          m &= m - 1;
          int got = 0, g2 = 0, t2 = 0;
          if (lane == src) {
            const unsigned long long o = atomicAdd(&V.word[i], 1ull);
            g2 = (int)(o >> 32);
            t2 = (int)(unsigned)o;
            const int np = V.ph_off[i + 1] - V.ph_off[i];
            got = g2 < np && (unsigned)t2 < (unsigned)V.phases[V.ph_off[i] + g2].nblk;
          }
          if (__shfl(got, src, 64)) {
            inst = __shfl(i, src, 64);
            ph = __shfl(g2, src, 64);
            tile = __shfl(t2, src, 64);
          }
        }
      }
      if (lane == 0) {
        if (inst >= 0) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        } else if (__hip_atomic_load(V.finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                   (unsigned)V.n) {
          inst = -2;
        }
        take[0] = inst;
        take[1] = ph;
        take[2] = tile;
      }
    }
    __syncthreads();
    const int inst = take[0], ph = take[1], tile = take[2];
    __syncthreads();
    if (inst == -2) return;
    if (inst == -1) {
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    cur = inst;
    const BatchItem it = V.phases[V.ph_off[inst] + ph];
    if (it.kind == kPhaseForward) {
      // A forward tile runs several of the phase's blocks of episodes
      // (blk0 of them in all, nblk tiles).
      for (int sub = tile; sub < it.blk0; sub += it.nblk) {
        run_item<AMAX>(views[inst], it, sub, sm);
        __syncthreads();
      }
    } else {
      run_item<AMAX>(views[inst], it, tile, sm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned d = atomicAdd(&V.done[inst], 1u) + 1u;
      if (d == (unsigned)it.nblk) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&V.done[inst], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int np = V.ph_off[inst + 1] - V.ph_off[inst];
        __hip_atomic_exchange(&V.word[inst], (unsigned long long)(ph + 1) << 32,
                              __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (ph + 1 == np) atomicAdd(V.finished, 1u);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers (host side).
// ---------------------------------------------------------------------------
static inline int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

int setup_blocks(const PlanView& P) {
  const long long work = (long long)P.t.h_mask + 1;         // 16-byte stores
  long long g = (work + kBlock * 8 - 1) / (kBlock * 8);
  return (int)std::max(1ll, std::min(g, 1024ll));
}

int forward_blocks(const PlanView& P) { return blocks_for(P.n_p); }

int accum_blocks(const PlanView& P, int D, int cap) {
  const long long g = (long long)blocks_for(P.n_p) * (D + 1);
  return (int)std::max(1ll, std::min(g, (long long)cap));
}

LaunchTiming& launch_timing() {
  static thread_local LaunchTiming t;
  return t;
}

// A plan kernel's launch, timed by its own dispatch when a profiling bracket
// is open on this thread (launch_timing).
template <typename... KArgs, typename... Args>
static void plan_launch(void (*kernel)(KArgs...), dim3 g, dim3 b, uint32_t shm, hipStream_t s,
                        Args... args) {
  LaunchTiming& t = launch_timing();
  if (t.stop) {
    hipExtLaunchKernelGGL(kernel, g, b, shm, s, t.start, t.stop, 0u, args...);
    t.start = nullptr;
    t.used = true;
  } else {
    hipLaunchKernelGGL(kernel, g, b, shm, s, args...);
  }
}

hipError_t launch_setup(const PlanView& P, hipStream_t s) {
  plan_launch(k_setup, dim3(setup_blocks(P)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_forward(const PlanView& P, int k, int D, hipStream_t s) {
  const dim3 g(forward_blocks(P)), b(kBlock);
  const int Ap = P.m.Apad;
  if (Ap <= 4) plan_launch(k_forward<4>, g, b, 0, s, P, k, D);
  else if (Ap <= 8) plan_launch(k_forward<8>, g, b, 0, s, P, k, D);
  else if (Ap <= 16) plan_launch(k_forward<16>, g, b, 0, s, P, k, D);
  else if (Ap <= 32) plan_launch(k_forward<32>, g, b, 0, s, P, k, D);
  else if (Ap <= kMaxA) plan_launch(k_forward<64>, g, b, 0, s, P, k, D);
  else
    plan_launch(k_forward_wide, dim3((P.n_p + kBlock / kHalf - 1) / (kBlock / kHalf)), b, 0, s,
                P, k, D);
  return hipGetLastError();
}
hipError_t launch_accum(const PlanView& P, int D, int grid, hipStream_t s) {
  if (P.t.ra > kMaxA) {
    plan_launch(k_claim_wide, dim3(blocks_for(std::min((long long)D * P.n_p, 1ll << 24))),
                dim3(kBlock), 0, s, P, D);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  plan_launch(k_accum, dim3(grid), dim3(kBlock), 0, s, P, D);
  return hipGetLastError();
}
hipError_t launch_backup_leaf(const PlanView& P, int dep, int k, int grid, hipStream_t s) {
  plan_launch(k_backup_leaf, dim3(grid), dim3(kBlock), 0, s, P, dep, k);
  return hipGetLastError();
}
hipError_t launch_backup_level(const PlanView& P, int dep, int k, int grid, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  const int Ap = P.m.Apad;
  if (Ap <= 4) plan_launch(k_backup_level<4>, g, b, 0, s, P, dep, k);
  else if (Ap <= 8) plan_launch(k_backup_level<8>, g, b, 0, s, P, dep, k);
  else if (Ap <= 16) plan_launch(k_backup_level<16>, g, b, 0, s, P, dep, k);
  else if (Ap <= 32) plan_launch(k_backup_level<32>, g, b, 0, s, P, dep, k);
  else if (Ap <= kMaxA) plan_launch(k_backup_level<64>, g, b, 0, s, P, dep, k);
  else {
    // Quads of the row per lane: rows of up to 1024, 2048, 3072, 4096 actions.
    const int qpl = (Ap / 4 + 63) / 64;
    if (qpl <= 4) plan_launch(k_backup_level_wide<4>, g, b, 0, s, P, dep, k);
    else if (qpl <= 8) plan_launch(k_backup_level_wide<8>, g, b, 0, s, P, dep, k);
    else if (qpl <= 12) plan_launch(k_backup_level_wide<12>, g, b, 0, s, P, dep, k);
    else plan_launch(k_backup_level_wide<16>, g, b, 0, s, P, dep, k);
  }
  return hipGetLastError();
}
hipError_t launch_backup_root(const PlanView& P, int k, hipStream_t s) {
  if (P.m.Apad > kMaxA) plan_launch(k_backup_root_wide, dim3(1), dim3(kBlock), 0, s, P, k);
  else plan_launch(k_backup_root, dim3(1), dim3(64), 0, s, P, k);
  return hipGetLastError();
}
hipError_t launch_select(const PlanView& P, hipStream_t s) {
  plan_launch(k_select, dim3(1), dim3(64), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_env(const PlanView& P, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_env, dim3(1), dim3(64), 0, s, P, t);
  return hipGetLastError();
}
hipError_t launch_pf_part(const PlanView& P, int part, int t, hipStream_t s) {
  const dim3 g(blocks_for(P.f.M)), b(kBlock);
  if (part == 0) hipLaunchKernelGGL(k_pf_weight, g, b, 0, s, P, t);
  else if (part == 1) hipLaunchKernelGGL(k_pf_scan, dim3(1), b, 0, s, P);
  else hipLaunchKernelGGL(k_pf_resample, g, b, 0, s, P, t);
  return hipGetLastError();
}
hipError_t launch_pf(const PlanView& P, int t, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int part = 0; part < 3 && e == hipSuccess; ++part) e = launch_pf_part(P, part, t, s);
  return e;
}
// The tree dump: belief ids[i]'s fields packed at out + i * dump_bytes(ra)
// (layout in vopp_device.hpp), one thread per belief.
__global__ __launch_bounds__(kBlock) void k_gather(TreeView t, const int* ids, int n,
                                                   unsigned char* out) {
  const int ra = t.ra;
  const size_t db = (size_t)dump_bytes(ra);
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const int id = ids[i];
    unsigned char* o = out + (size_t)i * db;
    float* po = reinterpret_cast<float*>(o);
    int* no = reinterpret_cast<int*>(o + dump_n_off(ra));
    unsigned long long* co = reinterpret_cast<unsigned long long*>(o + dump_c_off(ra));
    for (int j = 0; j < ra; ++j) {
      po[j] = rec_psi(t, id)[j];
      no[j] = rec_n(t, id)[j];
      co[j] = rec_c(t, id)[j];
    }
    const BeliefHot h = *rec_hot(t, id);
    const BeliefLeaf l = *rec_leaf(t, id);
    unsigned char* tl = o + dump_tail_off(ra);
    *reinterpret_cast<float*>(tl) = h.V;
    *reinterpret_cast<int*>(tl + 4) = h.Nb;
    *reinterpret_cast<int*>(tl + 8) = l.obs;
    *reinterpret_cast<int*>(tl + 12) = 0;
    *reinterpret_cast<unsigned long long*>(tl + 16) = h.parent;
    uint32_t* bo = reinterpret_cast<uint32_t*>(o + dump_bits_off(ra));
    for (int j = 0; j < t.bw; ++j) bo[j] = rec_bits(t, id)[j];
  }
}
hipError_t launch_gather(const TreeView& t, const int* ids, int n, unsigned char* out,
                         hipStream_t s) {
  const int g = (int)std::max(1ll, std::min(((long long)n + kBlock - 1) / kBlock, 4096ll));
  hipLaunchKernelGGL(k_gather, dim3(g), dim3(kBlock), 0, s, t, ids, n, out);
  return hipGetLastError();
}
// ---------------------------------------------------------------------------
// Tree re-rooting between real steps (the outer loop of Alg. 1): the belief
// reached from the root by the executed action and the perceived observation
// becomes the root of the next plan; its descendants keep their records
// (statistics) and move one level up.  The passes run depth by depth, so a
// belief's parent is always done before it.
// ---------------------------------------------------------------------------

// Slot of `key` (any stamp) in a table no kernel is inserting into, or ~0u.
// An insert takes the first empty-or-matching slot of the key's line in the
// key's rotated order and moves to the next line only when the line is full,
// and slots are never emptied during a plan, so the first such slot decides.
__device__ uint32_t find_slot(const TreeView& t, unsigned long long key) {
  const unsigned long long hk = mix64(key);
  uint32_t base = (uint32_t)hk & t.h_mask & ~7u;
  const uint32_t rot = (uint32_t)(hk >> 40) & 7u;
  const uint32_t lines = (t.h_mask >> 3) + 1;
  for (uint32_t n = 0; n < lines; ++n) {
    uint32_t best = 8;
    int at = -1;
    bool empty = false;
    for (int j = 0; j < 8; ++j) {
      const unsigned long long cur = t.h_slot[base + j].key;
      const uint32_t pos = ((uint32_t)j - rot) & 7u;
      if ((cur == kEmptyKey || (cur & ~kStampMask) == key) && pos < best) {
        best = pos;
        at = j;
        empty = cur == kEmptyKey;
      }
    }
    if (at >= 0) return empty ? ~0u : base + (uint32_t)at;
    base = (base + 8u) & t.h_mask;
  }
  return ~0u;
}

__global__ void k_reroot_find(TreeView t, int a, int obs, int ob, int* out) {
  if (threadIdx.x != 0) return;
  const uint32_t h = find_slot(t, belief_key(0, a, obs, ob));
  out[0] = h == ~0u ? -1 : t.h_slot[h].id;
}

// Source record of position i of the launch's level steps, or -1.
__device__ __forceinline__ int reroot_record(const RerootView& V, long long i) {
  const int s = V.steps[i / V.src_n_p];
  const size_t pos = (size_t)s * (size_t)V.src_n_p + (size_t)(i % V.src_n_p);
  return V.src.list[pos] ? (int)(1 + pos) : -1;
}

// The parent link (record << kActBits | action) of a source record, resolved.
__device__ __forceinline__ unsigned long long reroot_parent(const TreeView& T, int r) {
  unsigned long long par = rec_hot(T, r)->parent;
  if (par != kEmptyKey && (par & kLinkSlot)) {
    const int psid = (int)((par & ~kLinkSlot) >> kActBits);
    par = ((unsigned long long)(uint32_t)record_of(T, psid) << kActBits) | (par & kActMask);
  }
  return par;
}

// Mark pass: kept[r] for the beliefs of one source depth, with counts of the
// kept beliefs and of their action nodes (and, at depth 1, the root's visits).
__global__ __launch_bounds__(kBlock) void k_reroot_mark(RerootView V) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long nb = 0, nn = 0, nv = 0;
  if (i < (long long)V.n_steps * V.src_n_p) {
    const int r = reroot_record(V, i);
    if (r > 0) {
      bool keep;
      if (V.src_depth == 1) {
        keep = r == V.root_rec;
      } else {
        const unsigned long long par = reroot_parent(V.src, r);
        keep = par != kEmptyKey && V.kept[par >> kActBits] != 0;
      }
      if (keep) {
        V.kept[r] = 1;
        nb = 1;
        const int* n = rec_n(V.src, r);
        const uint32_t* bits = rec_bits(V.src, r);
        const bool wide = V.src.ra > kMaxA;   // long rows: columns valid per bitmap
        for (int j = 0; j < V.A; ++j) {
          const int c = (!wide || ((bits[j >> 5] >> (j & 31)) & 1u)) ? n[j] : 0;
          nn += c > 0 ? 1ull : 0ull;
          nv += (unsigned long long)(c > 0 ? c : 0);
        }
      }
    }
  }
  nb = wave_sum(nb);
  nn = wave_sum(nn);
  nv = wave_sum(nv);
  if ((threadIdx.x & 63) == 0 && nb) {
    atomicAdd(&V.cnt[V.src_depth], nb);
    atomicAdd(&V.cnt[kRerootCnt + V.src_depth], nn);
    if (V.src_depth == 1) atomicAdd(&V.cnt[2 * kRerootCnt + 1], nv);
  }
}

// Copy pass: each kept belief of one source depth gets the next position of
// its new depth's level steps (the root: record 0), its record is copied with
// the fixed-point sums rescaled, and it is inserted in the destination table
// under its new parent's slot id.
__global__ __launch_bounds__(kBlock) void k_reroot_copy(RerootView V) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (long long)V.n_steps * V.src_n_p) return;
  const int r = reroot_record(V, i);
  if (r <= 0 || !V.kept[r]) return;
  const int d_new = V.src_depth - 1;
  int nr = 0;
  if (d_new > 0) {
    const unsigned long long q = atomicAdd(&V.cnt[3 * kRerootCnt + d_new], 1ull);
    const long long t = (long long)V.first_step + (long long)(q / (unsigned long long)V.dst_n_p);
    nr = (int)(1 + t * V.dst_n_p + (long long)(q % (unsigned long long)V.dst_n_p));
  }
  V.new_id[r] = nr;
  {                                           // every field of the belief
    const int ra = V.src.ra;
    for (int j = 0; j < ra; ++j) {
      rec_psi(V.dst, nr)[j] = rec_psi(V.src, r)[j];
      rec_n(V.dst, nr)[j] = rec_n(V.src, r)[j];
      rec_c(V.dst, nr)[j] = rec_c(V.src, r)[j];
      rec_w(V.dst, nr)[j] = rec_w(V.src, r)[j];
    }
    for (int j = 0; j < V.src.bw; ++j) rec_bits(V.dst, nr)[j] = rec_bits(V.src, r)[j];
    *rec_hot(V.dst, nr) = *rec_hot(V.src, r);
    *rec_leaf(V.dst, nr) = *rec_leaf(V.src, r);
  }
  unsigned long long* c = rec_c(V.dst, nr);
  unsigned long long* w = rec_w(V.dst, nr);
  const uint32_t* bits = rec_bits(V.dst, nr);
  const bool wide = V.dst.ra > kMaxA;       // long rows: columns valid per bitmap
  for (int j = 0; j < V.dst.ra; ++j) {
    if (wide && !((bits[j >> 5] >> (j & 31)) & 1u)) continue;
    if (V.rescale != 1.0 && c[j])
      c[j] = (unsigned long long)llrint((double)(long long)c[j] * V.rescale);
    w[j] = 0ull;
  }
  BeliefHot* mt = rec_hot(V.dst, nr);
  BeliefLeaf* lf = rec_leaf(V.dst, nr);
  lf->leaf_cnt = 0;
  lf->leaf_h = 0ull;
  if (d_new == 0) {
    lf->obs = -1;
    mt->parent = kEmptyKey;
    return;
  }
  const unsigned long long par = reroot_parent(V.src, r);
  const int a_par = (int)(par & kActMask);
  const int np = V.new_id[(int)(par >> kActBits)];
  const int psid = np == 0 ? 0 : V.dst.list[np - 1];
  const unsigned long long key = belief_key(psid, a_par, lf->obs, V.obs_bits);
  bool won = false, fresh = false;
  int id = -1;
  const uint32_t h = probe(V.dst, key, kCarryStamp, won, fresh, id);
  if (h == ~0u || !won) {
    atomicOr((unsigned int*)&V.cnt[4 * kRerootCnt], 1u);
    return;
  }
  V.dst.list[nr - 1] = (int)h + 1;
  V.dst.h_slot[h].id = nr;
  mt->parent = ((unsigned long long)(uint32_t)np << kActBits) | (unsigned long long)a_par;
}

__global__ __launch_bounds__(kBlock) void k_fill16(uint4* p, size_t n, uint4 v) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kBlock)
    p[i] = v;
}

hipError_t launch_reroot_find(const TreeView& t, int a, int obs, int ob, int* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_reroot_find, dim3(1), dim3(64), 0, s, t, a, obs, ob, out);
  return hipGetLastError();
}
static int reroot_blocks(const RerootView& V) {
  return (int)std::max(1ll, ((long long)V.n_steps * V.src_n_p + kBlock - 1) / kBlock);
}
hipError_t launch_reroot_mark(const RerootView& V, hipStream_t s) {
  if (V.n_steps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reroot_mark, dim3(reroot_blocks(V)), dim3(kBlock), 0, s, V);
  return hipGetLastError();
}
hipError_t launch_reroot_copy(const RerootView& V, hipStream_t s) {
  if (V.n_steps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reroot_copy, dim3(reroot_blocks(V)), dim3(kBlock), 0, s, V);
  return hipGetLastError();
}
hipError_t launch_fill16(void* p, size_t n, uint4 v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_fill16, dim3(g), dim3(kBlock), 0, s, reinterpret_cast<uint4*>(p), n, v);
  return hipGetLastError();
}

hipError_t launch_persistent(const PlanView* views, const PersistView& V, int n_blocks,
                             int amax, hipStream_t s) {
  hipLaunchKernelGGL(k_persist_reset, dim3((V.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, V);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 g(n_blocks), b(kBlock);
  if (amax <= 4) hipLaunchKernelGGL(k_batch_persistent<4>, g, b, 0, s, views, V);
  else if (amax <= 8) hipLaunchKernelGGL(k_batch_persistent<8>, g, b, 0, s, views, V);
  else hipLaunchKernelGGL(k_batch_persistent<16>, g, b, 0, s, views, V);
  return hipGetLastError();
}

int persistent_blocks_per_cu(int amax) {
  const void* f = amax <= 4 ? (const void*)k_batch_persistent<4>
                 : amax <= 8 ? (const void*)k_batch_persistent<8>
                             : (const void*)k_batch_persistent<16>;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, 0) != hipSuccess || n < 1)
    n = 1;
  return n;
}

hipError_t launch_batch(const PlanView* views, const BatchItem* items, int n_items,
                        int n_blocks, int amax, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  const dim3 g(n_blocks), b(kBlock);
  if (amax <= 4) hipLaunchKernelGGL(k_batch<4>, g, b, 0, s, views, items, n_items);
  else if (amax <= 8) hipLaunchKernelGGL(k_batch<8>, g, b, 0, s, views, items, n_items);
  else hipLaunchKernelGGL(k_batch<16>, g, b, 0, s, views, items, n_items);
  return hipGetLastError();
}

}  // namespace vopp

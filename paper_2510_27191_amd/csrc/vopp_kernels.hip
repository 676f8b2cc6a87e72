// vopp_kernels.hip -- HIP kernels of one VOPP planning step for gfx950.
//
// One level of the vectorized forward search (Alg. 2) is two phases:
//
//   expand   one thread per episode: close the previous level (visit count and
//            reward sum of the action node, parent of a new belief), draw the
//            action from the softmax of the belief's preferences (Eq. 6), call
//            G, and claim the (belief, action) slot of the dense child table
//            and the (belief, action, observation) slot of the open-addressing
//            table with atomicMin(kClaimBase + episode).
//   resolve  the smallest claiming episode of each new pair is its creator;
//            creators are ranked in episode order by a single-pass
//            decoupled look-back scan (dynamic tile tickets), which numbers new
//            action nodes and beliefs in first-visitor order, initialises
//            their rows and publishes the indices in the tables.
//
// After the deepest level, `finish` closes it and accumulates this
// iteration's leaf visits and heuristic sums.  The backup of Alg. 3 is one
// phase per depth over every belief of that depth in the tree: leaves take
// their mean heuristic, internal beliefs update their preference row with
// Q = C/N + gamma W and V = L_eta Psi, and each belief pushes V*N_b into its
// parent action's W accumulator.  The root level runs in double precision.
//
// All cross-episode sums (rewards, heuristics, V*N_b) are 64-bit fixed-point
// integer atomics, so the results do not depend on thread order.
//
// Every phase is a __device__ function of (plan view, block index within the
// phase, block count of the phase).  The single-plan path launches one kernel
// per phase; the batched path launches k_batch, whose blocks each run one
// phase of one instance of a batch (BatchItem), so one launch advances every
// instance of the batch by one phase.
#include <algorithm>

#include "vopp_device.hpp"
#include "vopp_launch.hpp"

namespace vopp {

// ---------------------------------------------------------------------------
// Open-addressing table: find or insert the key, return its slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int hash_slot(const TreeView& t, unsigned long long key) {
  uint32_t h = (uint32_t)mix64(key) & t.h_mask;
  while (true) {
    unsigned long long cur = __hip_atomic_load(&t.h_key[h], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    if (cur == key) return (int)h;
    if (cur == kEmptyKey) {
      unsigned long long prev = atomicCAS(&t.h_key[h], kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) return (int)h;
    }
    h = (h + 1) & t.h_mask;
  }
}

__device__ __forceinline__ unsigned long long belief_key(int b, int a, int obs) {
  return ((unsigned long long)(uint32_t)b << 32) |
         ((unsigned long long)(uint32_t)a << 24) | (uint32_t)obs;
}

// ---------------------------------------------------------------------------
// Shared memory of every phase (one static allocation per kernel).
// ---------------------------------------------------------------------------

// Block-level pre-aggregation.  Shallow tree levels funnel many episodes into
// few nodes (every episode of an iteration passes through one of the |A| root
// action nodes), so same-address global atomics would serialise.  Each block
// first combines its contributions per key in an LDS hash table and then
// issues one global atomic per distinct key.  Integer adds and min are
// order-independent, so results stay bit-identical.
constexpr int kAggSlots = 2 * kBlock;      // at most kBlock keys per block

struct AggTable {
  int key[kAggSlots];
  unsigned long long a[kAggSlots];
  unsigned long long b[kAggSlots];
};

// Row ranges of the beliefs of one depth: level step t of every iteration
// that reached that depth created one contiguous range.
struct Ranges {
  int n;
  int lo[kMaxRanges];
  int off[kMaxRanges + 1];
};

struct Smem {
  AggTable agg;
  Ranges ranges;
  int tile;
  unsigned long long wave[kBlock / 64];
  unsigned long long prefix;
};

__device__ __forceinline__ void agg_clear(AggTable& T, unsigned long long init) {
  for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
    T.key[i] = -1;
    T.a[i] = init;
    T.b[i] = 0ull;
  }
}

__device__ __forceinline__ int agg_slot(AggTable& T, int key) {
  uint32_t h = ((uint32_t)key * 2654435761u) >> 23;   // 9 bits
  while (true) {
    const int prev = atomicCAS(&T.key[h], -1, key);
    if (prev == -1 || prev == key) return (int)h;
    h = (h + 1) & (kAggSlots - 1);
  }
}

// Visit count and reward sum of the previous level's action nodes, then the
// belief the episode now sits at (-1 if it stopped).  Called by every thread
// of the block (it contains barriers); `ep_ok` marks threads with an episode.
__device__ __forceinline__ int close_level(const PlanView& P, int ep, bool ep_ok,
                                           AggTable& T) {
  int an = -1, b = -1;
  unsigned long long rf = 0ull;
  if (ep_ok) {
    const int as = P.e.aslot[ep];
    if (as >= 0) {
      an = P.t.b_child[as];
      rf = to_fix(P.e.r[ep], P.fix_scale);
      const int hs = P.e.hslot[ep];
      if (hs >= 0) {
        b = P.t.h_val[hs & kSlotMask];
        if (hs & kWinBit) P.t.b_parent[b] = an;
      }
    }
  }
  agg_clear(T, 0ull);
  __syncthreads();
  if (an >= 0) {
    const int sl = agg_slot(T, an);
    atomicAdd(&T.a[sl], 1ull);
    if (rf) atomicAdd(&T.b[sl], rf);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
    const int k = T.key[i];
    if (k >= 0) {
      atomicAdd(&P.t.a_N[k], (int)T.a[i]);
      if (T.b[i]) atomicAdd(&P.t.a_C[k], T.b[i]);
    }
  }
  __syncthreads();
  return b;
}

// First-visitor claim: table[key] = min(table[key], kClaimBase + ep), with the
// per-block minimum episode taken in LDS first.
__device__ __forceinline__ void claim_min(AggTable& T, int* table, int key, int ep) {
  agg_clear(T, 0x7FFFFFFFull);
  __syncthreads();
  if (key >= 0) {
    const int sl = agg_slot(T, key);
    atomicMin(&T.a[sl], (unsigned long long)ep);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
    const int k = T.key[i];
    if (k >= 0) atomicMin(&table[k], kClaimBase + (int)T.a[i]);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Phase: set-up of a plan.  Clears the belief table (a full fill, or only the
// slots the previous plan used when that is cheaper), the scan state and the
// root row.  The previous plan's belief count is read on the device, so the
// phase is identical on every replay of a captured launch sequence.
// ---------------------------------------------------------------------------
__device__ void dev_setup(const PlanView& P, int blk, int nblk) {
  const unsigned long long n_prev = P.t.counters[2];
  const bool full = P.t.counters[3] != 0ull ||
                    n_prev * 10ull >= (unsigned long long)P.t.h_mask + 1ull;
  const size_t tid = (size_t)blk * kBlock + threadIdx.x;
  const size_t stride = (size_t)nblk * kBlock;
  const size_t hcap = (size_t)P.t.h_mask + 1;
  if (full) {
    uint4* hk = reinterpret_cast<uint4*>(P.t.h_key);
    uint4* hv = reinterpret_cast<uint4*>(P.t.h_val);
    const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (size_t i = tid; i < hcap / 2; i += stride) hk[i] = ones;
    for (size_t i = tid; i < hcap / 4; i += stride) hv[i] = ones;
  } else {
    for (size_t b = 1 + tid; b < n_prev; b += stride) {
      const int hs = P.t.b_hslot[b];
      P.t.h_key[hs] = kEmptyKey;
      P.t.h_val[hs] = -1;
    }
  }
  const size_t nlb = (size_t)P.steps * P.t.res_tiles;
  for (size_t i = tid; i < nlb; i += stride) P.t.lookback[i] = 0ull;
  for (size_t i = tid; i < (size_t)P.steps; i += stride) P.t.tickets[i] = 0;
  if (blk == 0) {
    const int j = threadIdx.x;
    const int A = P.m.nA, Apad = P.m.Apad;
    if (j < Apad) {
      P.t.b_child[j] = -1;
      P.t.psi[j] = j < A ? P.psi0 : 0.0f;
      if (j < A) P.t.psi_root[j] = P.psi0_64;
    }
    if (j == 0) {
      P.t.b_parent[0] = -1;
      P.t.b_obs[0] = -1;
      P.t.b_V[0] = 0.0f;
      P.t.b_N[0] = 0;
      P.t.leaf_cnt[0] = 0;
      P.t.leaf_h[0] = 0ull;
      P.t.b_hslot[0] = 0;
      P.t.v_root[0] = 0.0;
      P.t.bel_base[0] = 1;
      P.t.act_base[0] = 0;
      P.t.counters[0] = 0ull;
      P.t.counters[1] = 0ull;
    }
  }
}

// ---------------------------------------------------------------------------
// Phase: expand one level (Alg. 2, one recursion step).
// ---------------------------------------------------------------------------
template <int AM>
__device__ void dev_expand(const PlanView& P, int k, int d, int blk, Smem& sm) {
  AggTable& T = sm.agg;
  const int ep = blk * kBlock + threadIdx.x;
  const bool ep_ok = ep < P.n_p;
  bool alive = false;
  int b = -1, s = 0;
  float x = 0.0f, y = 0.0f;
  if (d == 0) {
    if (ep_ok) {
      // Alg. 1: the episode starts at the root with a state drawn from the
      // belief particles.
      const U4 w = draw(P, (uint32_t)ep, kTagRoot, 0, (uint32_t)k);
      const uint32_t idx = __umulhi(w.x, (uint32_t)P.e.n_belief);
      if (P.m.kind == kTabular) {
        s = ((const int*)P.e.belief)[idx];
        if ((unsigned)s >= (unsigned)P.m.nS) {   // caller's particle out of range
          atomicOr((unsigned int*)&P.t.counters[1], 1u);
          s = 0;
        }
      } else {
        const float* bf = (const float*)P.e.belief;
        x = bf[idx];
        y = bf[P.e.n_belief + idx];
      }
      b = 0;
      alive = true;
    }
  } else {
    // The state load does not depend on the previous level's tables.
    if (ep_ok) {
      if (P.m.kind == kTabular) s = P.e.s_i[ep];
      else { x = P.e.s_x[ep]; y = P.e.s_y[ep]; }
    }
    b = close_level(P, ep, ep_ok, T);
    alive = b >= 0;
  }
  int as = -1, hs = -1;
  bool claim_a = false, claim_b = false;
  if (alive) {
    const U4 w = draw(P, (uint32_t)ep, kTagStep, (uint32_t)d, (uint32_t)k);
    const int A = P.m.nA;
    int a;
    if (b == 0) {
      a = draw_action64(P.t.psi_root, A, P.eta64, w.x);
    } else {
      a = draw_action32<AM>(P.t.psi + (size_t)b * P.m.Apad, A, P.eta, w.x);
    }
    int obs;
    float r;
    bool term = false;
    if (P.m.kind == kTabular) {
      int sn;
      tabular_step(P.m, s, a, w, sn, obs, r);
      P.e.s_i[ep] = sn;
    } else {
      float nx, ny;
      nav_step(P.m, x, y, a, w, nx, ny, obs, r, term);
      P.e.s_x[ep] = nx;
      P.e.s_y[ep] = ny;
    }
    P.e.r[ep] = r;
    as = b * P.m.Apad + a;
    claim_a = P.t.b_child[as] < 0;
    if (!term) {                              // FilterTerminals
      hs = hash_slot(P.t, belief_key(b, a, obs));
      claim_b = P.t.h_val[hs] < 0;
    }
  }
  if (ep_ok) {
    P.e.aslot[ep] = as;
    P.e.hslot[ep] = hs;
  }
  // AppendActions / AppendBeliefs claims: the smallest episode id per new
  // pair wins.
  if (__syncthreads_or(claim_a)) claim_min(T, P.t.b_child, claim_a ? as : -1, ep);
  if (__syncthreads_or(claim_b)) claim_min(T, P.t.h_val, claim_b ? hs : -1, ep);
  // Particle-step count: one generative-model call per running episode.
  const unsigned long long ballot = __ballot(alive);
  if ((threadIdx.x & 63) == 0 && ballot)
    atomicAdd(&P.t.counters[0], (unsigned long long)__popcll(ballot));
}

// ---------------------------------------------------------------------------
// Phase: resolve the claims of level step t (first-visitor numbering).
// Packed scan word: (count_a << 31) | count_b, both < 2^31.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    unsigned long long n = __shfl_up(v, off, 64);
    if (lane >= off) v += n;
  }
  return v;
}

constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagIncl = 2ull << 62;
constexpr unsigned long long kPayload = (1ull << 62) - 1;

__device__ void dev_resolve(const PlanView& P, int t, Smem& sm) {
  if (threadIdx.x == 0) sm.tile = atomicAdd(&P.t.tickets[t], 1);
  __syncthreads();
  const int tile = sm.tile;
  const int items = P.t.res_items;
  const int base_ep = (tile * kBlock + threadIdx.x) * items;

  int aslot[kResItemsMax], hslot[kResItemsMax];
  unsigned flags = 0;   // bit i: action creator, bit 16+i: belief creator
  unsigned long long mine = 0;
#pragma unroll
  for (int i = 0; i < kResItemsMax; ++i) {
    const int ep = base_ep + i;
    aslot[i] = -1;
    hslot[i] = -1;
    if (i < items && ep < P.n_p) {
      aslot[i] = P.e.aslot[ep];
      hslot[i] = P.e.hslot[ep];
      if (aslot[i] >= 0 && P.t.b_child[aslot[i]] == kClaimBase + ep) {
        flags |= 1u << i;
        mine += 1ull << 31;
      }
      if (hslot[i] >= 0 && P.t.h_val[hslot[i]] == kClaimBase + ep) {
        flags |= 1u << (16 + i);
        mine += 1ull;
      }
    }
  }
  // Block scan.
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned long long incl = wave_incl_scan(mine);
  if (lane == 63) sm.wave[wid] = incl;
  __syncthreads();
  unsigned long long wave_off = 0, block_total = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < wid) wave_off += sm.wave[i];
    block_total += sm.wave[i];
  }
  const unsigned long long local_excl = wave_off + incl - mine;

  // Decoupled look-back across tiles, one wavefront probing 64 predecessors
  // at a time.
  if (wid == 0) {
    unsigned long long* st = P.t.lookback + (size_t)t * P.t.res_tiles;
    if (lane == 0)
      __hip_atomic_store(&st[tile], (tile == 0 ? kFlagIncl : kFlagAgg) | block_total,
                         __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long excl = 0;
    int hi = tile - 1;
    while (hi >= 0) {
      const int j = hi - lane;
      unsigned long long v = kFlagIncl;          // before tile 0: inclusive 0
      if (j >= 0) {
        v = __hip_atomic_load(&st[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        while ((v >> 62) == 0) {
          __builtin_amdgcn_s_sleep(1);
          v = __hip_atomic_load(&st[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      const unsigned long long incl_mask = __ballot((v >> 62) == 2);
      unsigned long long part;
      if (incl_mask) {
        const int first = __ffsll((long long)incl_mask) - 1;   // nearest inclusive
        part = lane <= first ? (v & kPayload) : 0ull;
      } else {
        part = v & kPayload;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
      excl += part;
      if (incl_mask) break;
      hi -= 64;
    }
    if (lane == 0) {
      if (tile > 0)
        __hip_atomic_store(&st[tile], kFlagIncl | (excl + block_total),
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      sm.prefix = excl;
      if (tile == P.t.res_tiles - 1) {
        const unsigned long long tot = excl + block_total;
        P.t.act_base[t + 1] = P.t.act_base[t] + (int)(tot >> 31);
        P.t.bel_base[t + 1] = P.t.bel_base[t] + (int)(tot & 0x7FFFFFFFull);
      }
    }
  }
  __syncthreads();
  if (!flags) return;
  const unsigned long long pre = sm.prefix + local_excl;
  int na = P.t.act_base[t] + (int)(pre >> 31);
  int nb = P.t.bel_base[t] + (int)(pre & 0x7FFFFFFFull);
  const int Apad = P.m.Apad, A = P.m.nA;
#pragma unroll
  for (int i = 0; i < kResItemsMax; ++i) {
    if (flags & (1u << i)) {
      const int as = aslot[i];
      P.t.b_child[as] = na;
      P.t.a_parent[na] = as / Apad;
      P.t.a_act[na] = as % Apad;
      P.t.a_C[na] = 0ull;
      P.t.a_N[na] = 0;
      P.t.a_W[na] = 0ull;
      ++na;
    }
    if (flags & (1u << (16 + i))) {
      const int hs = hslot[i];
      const unsigned long long key = P.t.h_key[hs];
      P.t.h_val[hs] = nb;
      P.t.b_obs[nb] = (int)(key & 0xFFFFFFull);
      P.t.b_hslot[nb] = hs;
      P.t.b_V[nb] = 0.0f;
      P.t.b_N[nb] = 0;
      P.t.leaf_cnt[nb] = 0;
      P.t.leaf_h[nb] = 0ull;
      float4* row = reinterpret_cast<float4*>(P.t.psi + (size_t)nb * Apad);
      int4* crow = reinterpret_cast<int4*>(P.t.b_child + (size_t)nb * Apad);
      for (int j = 0; j < Apad; j += 4) {
        const float p0 = P.psi0;
        row[j >> 2] = make_float4(j < A ? p0 : 0.0f, j + 1 < A ? p0 : 0.0f,
                                  j + 2 < A ? p0 : 0.0f, j + 3 < A ? p0 : 0.0f);
        crow[j >> 2] = make_int4(-1, -1, -1, -1);
      }
      P.e.hslot[base_ep + i] = hs | kWinBit;
      ++nb;
    }
  }
}

// ---------------------------------------------------------------------------
// Phase: close the deepest level and accumulate this iteration's leaves.
// ---------------------------------------------------------------------------
__device__ void dev_finish(const PlanView& P, int blk, Smem& sm) {
  AggTable& T = sm.agg;
  const int ep = blk * kBlock + threadIdx.x;
  const bool ep_ok = ep < P.n_p;
  const int b = close_level(P, ep, ep_ok, T);
  unsigned long long hf = 0ull;
  if (b >= 0) {
    float h = 0.0f;                           // ValueHeuristic
    if (P.m.kind == kTabular) {
      if (P.m.H) h = P.m.H[P.e.s_i[ep]];
    } else {
      h = nav_heuristic(P.m.nav, P.e.s_x[ep], P.e.s_y[ep]);
    }
    hf = to_fix(h, P.fix_scale);
  }
  agg_clear(T, 0ull);
  __syncthreads();
  if (b >= 0) {
    const int sl = agg_slot(T, b);
    atomicAdd(&T.a[sl], 1ull);
    if (hf) atomicAdd(&T.b[sl], hf);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
    const int key = T.key[i];
    if (key >= 0) {
      atomicAdd(&P.t.leaf_cnt[key], (int)T.a[i]);
      if (T.b[i]) atomicAdd(&P.t.leaf_h[key], T.b[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// Backup (Alg. 3).  Beliefs of depth `dep` were created by level dep-1 of
// every iteration k' <= k whose depth D_k' >= dep.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_ranges(const PlanView& P, int dep, int k,
                                            Ranges& R) {
  if (threadIdx.x == 0) {
    int n = 0, off = 0;
    for (int kk = 1; kk <= k; ++kk) {
      const int s0 = P.t.step_base[kk - 1];
      const int Dk = P.t.step_base[kk] - s0;
      if (Dk >= dep) {
        const int t = s0 + dep - 1;
        const int lo = P.t.bel_base[t];
        const int len = P.t.bel_base[t + 1] - lo;
        R.lo[n] = lo;
        R.off[n] = off;
        off += len;
        ++n;
      }
    }
    R.off[n] = off;
    R.n = n;
  }
  __syncthreads();
}

__device__ __forceinline__ int range_row(const Ranges& R, int i) {
  int lo = 0, hi = R.n - 1;          // last r with off[r] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (R.off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return R.lo[lo] + (i - R.off[lo]);
}

// Push V*N_b of belief b (or nothing if b < 0) into its parent action's W
// accumulator, aggregated per block.  Called by every thread of the block.
__device__ __forceinline__ void push_values(const PlanView& P, AggTable& T, int b,
                                            float V, int N) {
  int par = -1;
  unsigned long long f = 0ull;
  if (b >= 0 && N > 0) {
    f = to_fix(V * (float)N, P.fix_scale);
    if (f) par = P.t.b_parent[b];
  }
  agg_clear(T, 0ull);
  __syncthreads();
  if (par >= 0) atomicAdd(&T.a[agg_slot(T, par)], f);
  __syncthreads();
  for (int i = threadIdx.x; i < kAggSlots; i += kBlock) {
    const int key = T.key[i];
    if (key >= 0 && T.a[i]) atomicAdd(&P.t.a_W[key], T.a[i]);
  }
  __syncthreads();
}

// Leaves of this iteration take count and mean heuristic; every belief of
// depth D pushes V*N_b to its parent action.
__device__ void dev_backup_leaf(const PlanView& P, int dep, int k, int blk, int nblk,
                                Smem& sm) {
  Ranges& R = sm.ranges;
  load_ranges(P, dep, k, R);
  const int total = R.off[R.n];
  for (int base = blk * kBlock; base < total; base += nblk * kBlock) {
    const int i = base + threadIdx.x;
    int b = -1, N = 0;
    float V = 0.0f;
    if (i < total) {
      b = range_row(R, i);
      const int c = P.t.leaf_cnt[b];
      if (c > 0) {
        const unsigned long long hs = P.t.leaf_h[b];
        V = from_fix(hs, P.fix_inv) / (float)c;
        N = c;
        P.t.b_V[b] = V;
        P.t.b_N[b] = N;
        P.t.leaf_cnt[b] = 0;
        if (hs) P.t.leaf_h[b] = 0ull;
      } else {
        V = P.t.b_V[b];
        N = P.t.b_N[b];
      }
    }
    push_values(P, sm.agg, b, V, N);
  }
}

// Internal beliefs of depth dep-1 >= 1.  AM >= |A| keeps the row in registers.
template <int AM>
__device__ void dev_backup_level(const PlanView& P, int dep, int k, int blk, int nblk,
                                 Smem& sm) {
  Ranges& R = sm.ranges;
  load_ranges(P, dep - 1, k, R);
  const int total = R.off[R.n];
  const int A = P.m.nA, Apad = P.m.Apad;
  const float gamma = P.m.gamma, eta = P.eta, inv = P.fix_inv;
  for (int base = blk * kBlock; base < total; base += nblk * kBlock) {
    const int i = base + threadIdx.x;
    int b = -1, N = 0;
    float V = 0.0f;
    if (i < total) {
      b = range_row(R, i);
      const int* crow = P.t.b_child + (size_t)b * Apad;
      float* prow = P.t.psi + (size_t)b * Apad;
      int child[AM];
      bool any = false;
#pragma unroll
      for (int j = 0; j < AM; j += 4) {
        int4 c = make_int4(-1, -1, -1, -1);
        if (j < A) c = *reinterpret_cast<const int4*>(crow + j);
        child[j] = c.x; child[j + 1] = c.y; child[j + 2] = c.z; child[j + 3] = c.w;
      }
#pragma unroll
      for (int j = 0; j < AM; ++j) any = any || (j < A && child[j] >= 0);
      if (any) {
        float psi[AM];
#pragma unroll
        for (int j = 0; j < AM; j += 4) {
          float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          if (j < A) q = *reinterpret_cast<const float4*>(prow + j);
          psi[j] = q.x; psi[j + 1] = q.y; psi[j + 2] = q.z; psi[j + 3] = q.w;
        }
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
          const int an = child[j];
          if (j < A && an >= 0) {
            const int n = P.t.a_N[an];
            const float c = from_fix(P.t.a_C[an], inv);
            const unsigned long long wf = P.t.a_W[an];
            const float w = from_fix(wf, inv);
            if (wf) P.t.a_W[an] = 0ull;
            const float fn = (float)n;
            const float q = c / fn + gamma * (w / fn);
            psi[j] = (psi[j] - vc) + q;
            nsum += n;
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
        P.t.b_V[b] = V;
        P.t.b_N[b] = N;
      } else {
        V = P.t.b_V[b];
        N = P.t.b_N[b];
      }
    }
    push_values(P, sm.agg, b, V, N);
  }
}

// The root row in double precision, updated in place (one thread).
__device__ void dev_backup_root(const PlanView& P) {
  if (threadIdx.x != 0) return;
  const int A = P.m.nA;
  double* psi = P.t.psi_root;
  const double vc = lse64(psi, A, P.eta64);
  long long nsum = 0;
  bool any = false;
  for (int j = 0; j < A; ++j) {
    const int an = P.t.b_child[j];
    if (an < 0) continue;
    any = true;
    const int n = P.t.a_N[an];
    const double c = (double)(long long)P.t.a_C[an] * P.fix_inv64;
    const double w = (double)(long long)P.t.a_W[an] * P.fix_inv64;
    P.t.a_W[an] = 0ull;
    const double q = c / (double)n + P.m.gamma64 * (w / (double)n);
    psi[j] = (psi[j] - vc) + q;
    nsum += n;
  }
  if (!any) return;
  const double v = lse64(psi, A, P.eta64);
  P.t.v_root[0] = v;
  P.t.b_V[0] = (float)v;
  P.t.b_N[0] = (int)nsum;
}

// Alg. 1: argmax of the root preferences (lowest index on ties) and the
// result record; also records the belief count for the next plan's set-up.
__device__ void dev_select(const PlanView& P, int last_step) {
  if (threadIdx.x != 0) return;
  const int A = P.m.nA;
  int best = 0;
  for (int j = 1; j < A; ++j)
    if (P.t.psi_root[j] > P.t.psi_root[best]) best = j;
  double* out = P.out;
  out[0] = (double)best;
  for (int j = 0; j < A; ++j) out[1 + j] = P.t.psi_root[j];
  out[A + 1] = P.t.v_root[0];
  out[A + 2] = (double)P.t.counters[0];
  out[A + 3] = (double)P.t.bel_base[last_step];
  out[A + 4] = (double)P.t.act_base[last_step];
  out[A + 5] = (double)P.t.counters[1];
  P.t.counters[2] = (unsigned long long)P.t.bel_base[last_step];
  P.t.counters[3] = 0ull;
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
  dev_setup(P, blockIdx.x, gridDim.x);
}
template <int AM>
__global__ __launch_bounds__(kBlock) void k_expand(PlanView P, int k, int d) {
  __shared__ Smem sm;
  dev_expand<AM>(P, k, d, blockIdx.x, sm);
}
__global__ __launch_bounds__(kBlock) void k_resolve(PlanView P, int t) {
  __shared__ Smem sm;
  dev_resolve(P, t, sm);
}
__global__ __launch_bounds__(kBlock) void k_finish(PlanView P) {
  __shared__ Smem sm;
  dev_finish(P, blockIdx.x, sm);
}
__global__ __launch_bounds__(kBlock) void k_backup_leaf(PlanView P, int dep, int k) {
  __shared__ Smem sm;
  dev_backup_leaf(P, dep, k, blockIdx.x, gridDim.x, sm);
}
template <int AM>
__global__ __launch_bounds__(kBlock) void k_backup_level(PlanView P, int dep, int k) {
  __shared__ Smem sm;
  dev_backup_level<AM>(P, dep, k, blockIdx.x, gridDim.x, sm);
}
__global__ void k_backup_root(PlanView P) { dev_backup_root(P); }
__global__ void k_select(PlanView P, int last_step) { dev_select(P, last_step); }

// ---------------------------------------------------------------------------
// Batched kernel: block -> (instance, phase) through the item list, sorted by
// first block.  AMAX bounds the padded action count of the batch.
// ---------------------------------------------------------------------------
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
  const PlanView& P = views[it.inst];
  const int Apad = P.m.Apad;
  switch (it.kind) {
    case kPhaseSetup: dev_setup(P, blk, it.nblk); break;
    case kPhaseExpand:
      if (Apad <= 4) {
        dev_expand<4>(P, it.a0, it.a1, blk, sm);
      } else if constexpr (AMAX >= 8) {
        if (Apad <= 8) dev_expand<8>(P, it.a0, it.a1, blk, sm);
        else if constexpr (AMAX >= 16) dev_expand<16>(P, it.a0, it.a1, blk, sm);
      }
      break;
    case kPhaseResolve: dev_resolve(P, it.a0, sm); break;
    case kPhaseFinish: dev_finish(P, blk, sm); break;
    case kPhaseLeaf: dev_backup_leaf(P, it.a0, it.a1, blk, it.nblk, sm); break;
    case kPhaseLevel:
      if (Apad <= 4) {
        dev_backup_level<4>(P, it.a0, it.a1, blk, it.nblk, sm);
      } else if constexpr (AMAX >= 8) {
        if (Apad <= 8) dev_backup_level<8>(P, it.a0, it.a1, blk, it.nblk, sm);
        else if constexpr (AMAX >= 16) dev_backup_level<16>(P, it.a0, it.a1, blk, it.nblk, sm);
      }
      break;
    case kPhaseRoot: dev_backup_root(P); break;
    case kPhaseSelect: dev_select(P, it.a0); break;
    case kPhaseEnv: dev_env(P, it.a0); break;
    case kPhasePFWeight: dev_pf_weight(P, it.a0, blk); break;
    case kPhasePFScan: dev_pf_scan(P, sm); break;
    case kPhasePFResample: dev_pf_resample(P, it.a0, blk); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Launchers (host side).
// ---------------------------------------------------------------------------
static inline int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

int setup_blocks(const PlanView& P) {
  const long long work = ((long long)P.t.h_mask + 1) / 2;   // 16-byte stores
  long long g = (work + kBlock * 8 - 1) / (kBlock * 8);
  return (int)std::max(1ll, std::min(g, 1024ll));
}

hipError_t launch_setup(const PlanView& P, hipStream_t s) {
  hipLaunchKernelGGL(k_setup, dim3(setup_blocks(P)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_expand(const PlanView& P, int k, int d, hipStream_t s) {
  const dim3 g(blocks_for(P.n_p)), b(kBlock);
  const int Ap = P.m.Apad;
  if (Ap <= 4) hipLaunchKernelGGL(k_expand<4>, g, b, 0, s, P, k, d);
  else if (Ap <= 8) hipLaunchKernelGGL(k_expand<8>, g, b, 0, s, P, k, d);
  else if (Ap <= 16) hipLaunchKernelGGL(k_expand<16>, g, b, 0, s, P, k, d);
  else if (Ap <= 32) hipLaunchKernelGGL(k_expand<32>, g, b, 0, s, P, k, d);
  else hipLaunchKernelGGL(k_expand<64>, g, b, 0, s, P, k, d);
  return hipGetLastError();
}
hipError_t launch_resolve(const PlanView& P, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_resolve, dim3(P.t.res_tiles), dim3(kBlock), 0, s, P, t);
  return hipGetLastError();
}
hipError_t launch_finish(const PlanView& P, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(blocks_for(P.n_p)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_backup_leaf(const PlanView& P, int dep, int k, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_backup_leaf, dim3(grid), dim3(kBlock), 0, s, P, dep, k);
  return hipGetLastError();
}
hipError_t launch_backup_level(const PlanView& P, int dep, int k, int grid, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  const int Ap = P.m.Apad;
  if (Ap <= 4) hipLaunchKernelGGL(k_backup_level<4>, g, b, 0, s, P, dep, k);
  else if (Ap <= 8) hipLaunchKernelGGL(k_backup_level<8>, g, b, 0, s, P, dep, k);
  else if (Ap <= 16) hipLaunchKernelGGL(k_backup_level<16>, g, b, 0, s, P, dep, k);
  else if (Ap <= 32) hipLaunchKernelGGL(k_backup_level<32>, g, b, 0, s, P, dep, k);
  else hipLaunchKernelGGL(k_backup_level<64>, g, b, 0, s, P, dep, k);
  return hipGetLastError();
}
hipError_t launch_backup_root(const PlanView& P, hipStream_t s) {
  hipLaunchKernelGGL(k_backup_root, dim3(1), dim3(64), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_select(const PlanView& P, int last_step, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, P, last_step);
  return hipGetLastError();
}
hipError_t launch_env(const PlanView& P, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_env, dim3(1), dim3(64), 0, s, P, t);
  return hipGetLastError();
}
hipError_t launch_pf(const PlanView& P, int t, hipStream_t s) {
  const dim3 g(blocks_for(P.f.M)), b(kBlock);
  hipLaunchKernelGGL(k_pf_weight, g, b, 0, s, P, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pf_scan, dim3(1), b, 0, s, P);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pf_resample, g, b, 0, s, P, t);
  return hipGetLastError();
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

/*
 * vopp_oracle.cpp -- serial CPU oracle for one VOPP planning step.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no source,
 * header, table or helper with the GPU path; the two meet only at the seeded
 * instance arrays.
 *
 * What it computes (Vectorized Online POMDP Planning, Hoerger, Sudrajat and
 * Kurniawati):
 *   - Alg. 1 (planning loop): K iterations; iteration k samples n_p root
 *     states from the belief, runs the forward search to depth D_k and then
 *     the backup; the chosen action is the argmax of the root preferences.
 *   - Alg. 2 (forward search): per level, a softmax policy over the current
 *     belief's preferences (Eq. 6), one sampled action per episode, one call
 *     of the generative model G, AppendActions (reward sum C and visit count N
 *     of the (belief, action) node), FilterTerminals, AppendBeliefs.
 *   - Alg. 3 (backup): leaf visit counts and mean heuristic values, then for
 *     d = D .. 1 over every node of depth d-1 in the tree:
 *     Q = C/N + gamma * sum_children V*N_b / N, N_b = sum_a N(b,a),
 *     Psi <- Psi - L_eta Psi + Q (Eq. 5), V = L_eta Psi (Eq. 3).
 *   - Sec. III-C: the tree is three row-indexed tables (beliefs, action
 *     nodes, preferences); the root is belief row 0.
 *
 * It runs the method literally: one episode at a time in ascending episode
 * id, every value (C, Psi, V, W, Q) in double precision, dictionaries for the
 * (belief, action) and (action node, observation) matching.
 *
 * Readings where the paper leaves a choice open (each side implements them
 * on its own):
 *   - Levels d = 0 .. D-1 are expanded; leaves sit at depth D.
 *   - The budget is K iterations; D_k = min(k, depth) (deepening schedule of
 *     Alg. 1) or D_k = depth (fixed schedule).
 *   - Reference policy pi0 (Eq. 4, first term): Psi0(b,a) = ln(pi0(a)) / eta
 *     with pi0 normalised by its sum, the same at every belief; uniform by
 *     default, Psi0 = -ln|A| / eta.  Either way L_eta Psi0 = 0.
 *   - Only actions that own an action node are updated in the backup; all
 *     of them use the same V_curr.  Every node of the backed-up depth in the
 *     whole tree takes part; an action node without child beliefs has W = 0.
 *   - A leaf reached this iteration gets this iteration's visit count and
 *     mean heuristic; an internal belief gets sum_a N(b,a) and L_eta Psi; a
 *     node not touched keeps its stored V and N_b.
 *   - New nodes are numbered in first-visitor order: inside one (iteration,
 *     level), by the smallest episode id that creates them; rows are global
 *     creation order and the root is row 0.  Running episodes serially in
 *     ascending id produces exactly this order.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = 64-bit
 *     seed, counter = (episode, tag<<24 | level, iteration, real step).
 *     Tags: ROOT = 1, STEP = 2.  A STEP block gives word 0 to the action
 *     draw and words 1, 2 to the model.
 *   - Root state draw: index = (x0 * M) >> 32 over the M belief particles.
 *   - Action draw (Eq. 6), the same rule at every belief: weights
 *     w_j = exp(eta (Psi_j - max Psi)) in double precision, P_j their running
 *     sums in action order, t = u * P_last with u = (x0 >> 8) * 2^-24, action
 *     = first j with t < P_j (clamped to |A|-1).  A row whose preferences are
 *     all equal therefore gives floor(u |A|) exactly.  The oracle also reports
 *     how close t lies to the nearest interior boundary P_j: a draw is a near
 *     tie when some |t - P_j| <= (tau + tau_psi * eta * max_j |Psi_j|) *
 *     P_last + tau_abs (all three passed in by the caller; max weight = 1).
 *     Any planner that keeps its preferences in another precision may decide
 *     such a draw either way.
 *   - Tabular G: thresholds thr_j = rint(cum_j / total * 2^31) from the
 *     sequential double sum of the fp32 row (last = 2^31); outcome = first j
 *     with (x >> 1) < thr_j.  Successor from word 1, observation from word 2
 *     using the row Z[s', a, .]; reward R[s, a]; never terminal.
 *   - Between real steps (Alg. 1): the true environment is G with its own
 *     stream (tag ENV = 4); the belief update is sequential importance
 *     resampling with exact integer likelihoods (tabular: the observation
 *     threshold difference; navigation: the count of noise-table index pairs
 *     whose observation lands in the observed cell) and multinomial draws
 *     (tags PF = 5, RESAMPLE = 6).
 *   - Navigation G: single-precision arithmetic with no contraction, noise
 *     from the instance's 4096-entry Gaussian quantile table; observation
 *     key from the 0.5 grid cell of the noisy position; reward -1 per step,
 *     +100 on reaching the goal disk (terminal), -100 inside an obstacle.
 */
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <unordered_map>
#include <vector>
#include <algorithm>
#include <limits>

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
// easy as 1, 2, 3", SC'11).  Ten rounds of the 4x32 S-P network with the
// multipliers and Weyl key increments of the published definition.
// ---------------------------------------------------------------------------
struct Words { uint32_t w[4]; };

Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                    uint32_t k0, uint32_t k1) {
  const uint32_t mulA = 0xD2511F53u, mulB = 0xCD9E8D57u;
  const uint32_t weylA = 0x9E3779B9u, weylB = 0xBB67AE85u;
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += weylA; k1 += weylB; }
    uint64_t pa = (uint64_t)mulA * c0;
    uint64_t pb = (uint64_t)mulB * c2;
    uint32_t hiA = (uint32_t)(pa >> 32), loA = (uint32_t)pa;
    uint32_t hiB = (uint32_t)(pb >> 32), loB = (uint32_t)pb;
    uint32_t n0 = hiB ^ c1 ^ k0;
    uint32_t n1 = loB;
    uint32_t n2 = hiA ^ c3 ^ k1;
    uint32_t n3 = loA;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  Words out = {{c0, c1, c2, c3}};
  return out;
}

const uint32_t TAG_ROOT = 1, TAG_STEP = 2, TAG_ENV = 4, TAG_PF = 5, TAG_RESAMPLE = 6;

Words draw(uint64_t seed, uint32_t ep, uint32_t tag, uint32_t level,
           uint32_t iter, uint32_t step) {
  return philox4x32_10(ep, (tag << 24) | level, iter, step,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// Categorical sampling by integer thresholds.
// ---------------------------------------------------------------------------
const double TWO31 = 2147483648.0;

// thr_j = rint(cum_j / total * 2^31), cum by sequential double summation of
// the fp32 probabilities; the last threshold is 2^31.
std::vector<uint32_t> thresholds(const float* p, int n) {
  std::vector<uint32_t> thr(n);
  double total = 0.0;
  for (int j = 0; j < n; ++j) total += (double)p[j];
  double cum = 0.0;
  for (int j = 0; j < n; ++j) {
    cum += (double)p[j];
    double v = rint(cum / total * TWO31);
    if (v > TWO31) v = TWO31;
    if (v < 0.0) v = 0.0;
    thr[j] = (uint32_t)v;
  }
  thr[n - 1] = (uint32_t)TWO31;
  return thr;
}

// First j with u31 < thr[j]; u31 = x >> 1.
int pick(const uint32_t* thr, int n, uint32_t x) {
  uint32_t u = x >> 1;
  for (int j = 0; j < n; ++j)
    if (u < thr[j]) return j;
  return n - 1;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Public descriptors (plain C).
// ---------------------------------------------------------------------------
typedef struct {
  int32_t nS, nA, nO;
  const int32_t* rowptr;  // [nS*nA + 1]
  const int32_t* col;     // [nnz]
  const float* tprob;     // [nnz]
  const float* zprob;     // [nS*nA*nO], indexed [s'][a][o]
  const float* reward;    // [nS*nA]
  const float* heur;      // [nS] or NULL (zero heuristic)
  double gamma;
} orc_tabular;

typedef struct {
  float lo, hi, step, sigma_move, sigma_obs0, sigma_obs_slope, obs_center_x,
      inv_bin;
  int32_t key_lo, key_n;
  float goal_x, goal_y, goal_r2, disk_r2, r_step, r_goal, r_hit;
  int32_t heuristic;       // 0: zero, 1: -(|x-gx| + |y-gy|)
  int32_t n_disks;
  const float* disks;      // [2*n_disks]
  const float* gauss;      // [4096]
  double gamma;
} orc_nav;

typedef struct {
  int32_t n_particles, budget, depth, schedule;  // schedule 0 deepen, 1 fixed
  double eta;
  uint64_t seed;
  uint32_t step;
  double tau;      // near-tie screen: |t - P_j| <= lim with
  double tau_abs;  // lim = (tau + tau_psi * eta * max_j |Psi_j|) * P_last + tau_abs
  double tau_psi;
  int32_t trace;   // keep a per-draw trace
  int32_t mutate;  // 0: none.  >0 plants a known mistake (pin sensitivity)
  const double* pi0;  // [A] reference policy weights (> 0), or NULL: uniform
  const void* start;  // a re-rooted tree (orc_reroot) to plan from, or NULL
} orc_params;

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Generative models.  State for tabular: int32; for navigation: (x, y) fp32.
// ---------------------------------------------------------------------------
struct State { int32_t s; float x, y; };

struct Outcome { State next; int32_t obs; float r; bool term; };

struct TabularModel {
  int nS, nA, nO;
  std::vector<int32_t> rowptr, col;
  std::vector<uint32_t> thrT, thrZ;   // per CSR row / per (s', a) row
  std::vector<float> R, H;
  double gamma;
  double r_max;

  explicit TabularModel(const orc_tabular* m)
      : nS(m->nS), nA(m->nA), nO(m->nO), gamma(m->gamma) {
    int rows = nS * nA;
    rowptr.assign(m->rowptr, m->rowptr + rows + 1);
    int nnz = rowptr[rows];
    col.assign(m->col, m->col + nnz);
    thrT.resize(nnz);
    for (int r = 0; r < rows; ++r) {
      int lo = rowptr[r], n = rowptr[r + 1] - lo;
      std::vector<uint32_t> t = thresholds(m->tprob + lo, n);
      std::copy(t.begin(), t.end(), thrT.begin() + lo);
    }
    thrZ.resize((size_t)rows * nO);
    for (int r = 0; r < rows; ++r) {
      std::vector<uint32_t> t = thresholds(m->zprob + (size_t)r * nO, nO);
      std::copy(t.begin(), t.end(), thrZ.begin() + (size_t)r * nO);
    }
    R.assign(m->reward, m->reward + rows);
    H.assign(nS, 0.0f);
    if (m->heur) H.assign(m->heur, m->heur + nS);
    r_max = 0.0;
    for (float v : R) r_max = std::max(r_max, (double)std::fabs(v));
  }

  int successor(int s, int a, uint32_t word) const {
    int row = s * nA + a;
    int lo = rowptr[row], n = rowptr[row + 1] - lo;
    return col[lo + pick(&thrT[lo], n, word)];
  }
  // Probability of observation o after (a, s'), in units of 2^-31.
  uint64_t obs_weight(int sn, int a, int o) const {
    const uint32_t* t = &thrZ[((size_t)sn * nA + a) * nO];
    return (uint64_t)t[o] - (o > 0 ? (uint64_t)t[o - 1] : 0ull);
  }

  Outcome step(const State& st, int a, const Words& x) const {
    Outcome o;
    int row = st.s * nA + a;
    int sn = successor(st.s, a, x.w[1]);
    int ob = pick(&thrZ[((size_t)sn * nA + a) * nO], nO, x.w[2]);
    o.next.s = sn; o.next.x = 0.0f; o.next.y = 0.0f;
    o.obs = ob;
    o.r = R[row];
    o.term = false;
    return o;
  }
  double heuristic(const State& st) const { return (double)H[st.s]; }
};

// All navigation arithmetic is single precision; the library is built with
// contraction off so every operation below rounds once.
struct NavModel {
  orc_nav p;
  std::vector<float> disks, gauss;
  double gamma;
  double r_max;

  explicit NavModel(const orc_nav* m) : p(*m), gamma(m->gamma) {
    disks.assign(m->disks, m->disks + 2 * m->n_disks);
    gauss.assign(m->gauss, m->gauss + 4096);
    r_max = std::max({std::fabs((double)p.r_step),
                      std::fabs((double)p.r_step + p.r_goal),
                      std::fabs((double)p.r_step + p.r_hit),
                      std::fabs((double)p.r_step + p.r_goal + p.r_hit)});
  }

  static float clampf(float v, float lo, float hi) {
    return std::fmin(std::fmax(v, lo), hi);
  }
  int key_axis(float v) const {
    float c = std::floor(v * p.inv_bin);
    int i = (int)std::fmax(std::fmin(c, (float)(p.key_lo + p.key_n - 1)),
                           (float)p.key_lo);
    return i - p.key_lo;
  }

  // Motion part of G: moves 0 = +y, 1 = +x, 2 = -y, 3 = -x, plus noise.
  void move(float x, float y, int a, uint32_t word, float* nx, float* ny) const {
    float dx = 0.0f, dy = 0.0f;
    if (a == 0) dy = p.step;
    else if (a == 1) dx = p.step;
    else if (a == 2) dy = -p.step;
    else dx = -p.step;
    float zx = gauss[word >> 20];
    float zy = gauss[(word >> 8) & 4095u];
    float mx = x + dx;
    float my = y + dy;
    *nx = clampf(mx + p.sigma_move * zx, p.lo, p.hi);
    *ny = clampf(my + p.sigma_move * zy, p.lo, p.hi);
  }
  float obs_sd(float nx) const {
    return p.sigma_obs0 + p.sigma_obs_slope * std::fabs(nx - p.obs_center_x);
  }
  // Likelihood of observation key o at (nx, ny), in units of 2^-24: the number
  // of (12-bit, 12-bit) noise index pairs whose observation lands in o's cell.
  uint64_t obs_weight(float nx, float ny, int o) const {
    const float sd = obs_sd(nx);
    const int kx = o / p.key_n, ky = o % p.key_n;
    uint64_t cx = 0, cy = 0;
    for (int j = 0; j < 4096; ++j) {
      if (key_axis(nx + sd * gauss[j]) == kx) ++cx;
      if (key_axis(ny + sd * gauss[j]) == ky) ++cy;
    }
    return cx * cy;
  }

  Outcome step(const State& st, int a, const Words& x) const {
    float nx, ny;
    move(st.x, st.y, a, x.w[1], &nx, &ny);
    float sd = obs_sd(nx);
    float ox = nx + sd * gauss[x.w[2] >> 20];
    float oy = ny + sd * gauss[(x.w[2] >> 8) & 4095u];
    int key = key_axis(ox) * p.key_n + key_axis(oy);
    float gx = nx - p.goal_x, gy = ny - p.goal_y;
    bool goal = (gx * gx + gy * gy) <= p.goal_r2;
    bool hit = false;
    for (int i = 0; i < p.n_disks; ++i) {
      float ex = nx - disks[2 * i], ey = ny - disks[2 * i + 1];
      if (ex * ex + ey * ey <= p.disk_r2) hit = true;
    }
    float r = p.r_step;
    if (goal) r = r + p.r_goal;
    if (hit) r = r + p.r_hit;
    Outcome o;
    o.next.s = 0; o.next.x = nx; o.next.y = ny;
    o.obs = key; o.r = r; o.term = goal;
    return o;
  }
  double heuristic(const State& st) const {
    if (p.heuristic == 0) return 0.0;
    float h = -(std::fabs(st.x - p.goal_x) + std::fabs(st.y - p.goal_y));
    return (double)h;
  }
};

// ---------------------------------------------------------------------------
// Tree (Sec. III-C): belief rows, action-node rows, preference rows.
// ---------------------------------------------------------------------------
struct Tree {
  int A;
  std::vector<int32_t> b_parent, b_obs, b_depth;
  std::vector<double> psi, b_V;
  std::vector<int64_t> b_N;
  std::vector<int32_t> b_child;      // [belief][a] -> action node or -1
  std::vector<int32_t> a_parent, a_act, a_depth;
  std::vector<double> a_C;
  std::vector<int64_t> a_N;
  std::unordered_map<uint64_t, int32_t> obs_child;  // (action node, obs)
  std::vector<std::vector<int32_t>> beliefs_at, actions_at;

  std::vector<double> psi0;          // initial preference row (Eq. 4, first term)

  void set_psi0(int nA, double eta, const double* pi0) {
    A = nA;
    psi0.assign(A, -std::log((double)A) / eta);
    if (pi0) {
      double sum = 0.0;
      for (int a = 0; a < A; ++a) sum += pi0[a];
      for (int a = 0; a < A; ++a) psi0[a] = std::log(pi0[a] / sum) / eta;
    }
  }
  void init(int nA, double eta, const double* pi0) {
    set_psi0(nA, eta, pi0);
    new_belief(-1, -1, 0, eta);
  }
  int32_t new_belief(int32_t parent, int32_t obs, int32_t depth, double eta) {
    (void)eta;
    int32_t id = (int32_t)b_parent.size();
    b_parent.push_back(parent);
    b_obs.push_back(obs);
    b_depth.push_back(depth);
    for (int a = 0; a < A; ++a) { psi.push_back(psi0[a]); b_child.push_back(-1); }
    b_V.push_back(0.0);
    b_N.push_back(0);
    if ((int)beliefs_at.size() <= depth) beliefs_at.resize(depth + 1);
    beliefs_at[depth].push_back(id);
    return id;
  }
  int32_t action_node(int32_t b, int a) {
    int32_t& slot = b_child[(size_t)b * A + a];
    if (slot >= 0) return slot;
    int32_t id = (int32_t)a_parent.size();
    a_parent.push_back(b);
    a_act.push_back(a);
    a_depth.push_back(b_depth[b]);
    a_C.push_back(0.0);
    a_N.push_back(0);
    int d = b_depth[b];
    if ((int)actions_at.size() <= d) actions_at.resize(d + 1);
    actions_at[d].push_back(id);
    slot = id;
    return id;
  }
  int32_t belief_node(int32_t an, int32_t obs, double eta) {
    uint64_t key = ((uint64_t)(uint32_t)an << 32) | (uint32_t)obs;
    auto it = obs_child.find(key);
    if (it != obs_child.end()) return it->second;
    int32_t id = new_belief(an, obs, a_depth[an] + 1, eta);
    obs_child.emplace(key, id);
    return id;
  }
};

// Tree re-rooting between real steps (Alg. 1 outer loop): after action a is
// executed and observation o perceived, the belief reached by (a, o) from the
// root becomes the new root and its descendants are kept with every
// statistic (preference rows, C, N, V, N_b), one level shallower; everything
// else is dropped.  Rows keep their relative order (parents precede their
// children).  If the tree has no such belief, the result is empty and the
// next plan starts from a fresh root as Alg. 1 does.
Tree reroot(const Tree& T, int a, int o) {
  Tree R;
  R.A = T.A;
  R.psi0 = T.psi0;
  const int A = T.A;
  int32_t an = T.b_child[(size_t)0 * A + a];
  if (an < 0) return R;
  auto it = T.obs_child.find(((uint64_t)(uint32_t)an << 32) | (uint32_t)o);
  if (it == T.obs_child.end()) return R;
  const int32_t nb = (int32_t)T.b_parent.size();
  std::vector<int32_t> bmap(nb, -1), amap(T.a_parent.size(), -1);
  bmap[it->second] = 0;
  // Rows are in creation order, so a belief's parent action node and that
  // node's parent belief precede it.
  for (int32_t b = 0; b < nb; ++b) {
    if (b != it->second) {
      const int32_t pa = T.b_parent[b];
      if (pa < 0 || amap[pa] < 0) continue;
    }
    const int32_t id = (int32_t)R.b_parent.size();
    bmap[b] = id;
    const bool root = b == it->second;
    R.b_parent.push_back(root ? -1 : amap[T.b_parent[b]]);
    R.b_obs.push_back(root ? -1 : T.b_obs[b]);
    R.b_depth.push_back(T.b_depth[b] - 1);
    for (int j = 0; j < A; ++j) {
      R.psi.push_back(T.psi[(size_t)b * A + j]);
      R.b_child.push_back(-1);
    }
    R.b_V.push_back(T.b_V[b]);
    R.b_N.push_back(T.b_N[b]);
    const int d = T.b_depth[b] - 1;
    if ((int)R.beliefs_at.size() <= d) R.beliefs_at.resize(d + 1);
    R.beliefs_at[d].push_back(id);
    if (!root) {
      const uint64_t key = ((uint64_t)(uint32_t)R.b_parent[id] << 32) | (uint32_t)T.b_obs[b];
      R.obs_child.emplace(key, id);
    }
    // The action nodes of b follow b in this construction; in the source
    // they were created after b as well.
    for (int j = 0; j < A; ++j) {
      const int32_t src = T.b_child[(size_t)b * A + j];
      if (src < 0) continue;
      const int32_t na = (int32_t)R.a_parent.size();
      amap[src] = na;
      R.a_parent.push_back(id);
      R.a_act.push_back(j);
      R.a_depth.push_back(d);
      R.a_C.push_back(T.a_C[src]);
      R.a_N.push_back(T.a_N[src]);
      if ((int)R.actions_at.size() <= d) R.actions_at.resize(d + 1);
      R.actions_at[d].push_back(na);
      R.b_child[(size_t)id * A + j] = na;
    }
  }
  return R;
}

// L_eta x = (1/eta) log sum_j exp(eta x_j), evaluated with the max shift.
double lse(const double* x, int n, double eta) {
  double m = x[0];
  for (int j = 1; j < n; ++j) m = std::max(m, x[j]);
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += std::exp(eta * (x[j] - m));
  return m + std::log(s) / eta;
}

struct TraceRow {
  int32_t k, d, ep, b, a, obs, term, an, near;
  float r;
  double margin;
};

struct Result {
  Tree tree;
  int32_t action = -1;
  double v_root = 0.0;
  int64_t particle_steps = 0;
  int64_t n_draws = 0;
  int64_t near_ties = 0;
  double min_margin = 1.0;
  std::vector<TraceRow> trace;
};

// Action draw of Eq. (6) in double precision.  *margin: distance of t from
// the nearest interior boundary, relative to P_last (1 for a flat row, whose
// draw floor(u |A|) is exact in any precision); *near: some interior boundary
// lies within lim = (tau + tau_psi * eta * max_j |Psi_j|) * P_last + tau_abs
// of t.  The tau_psi term scales with the row's magnitude: a planner that
// keeps preferences in a precision with relative rounding e perturbs every
// weight exp(eta (Psi_j - max)) by a relative amount of order
// eta * e * max |Psi|, and so every running sum by that much of P_last.
int sample_action(const double* psi, int A, double eta, uint32_t x0, double tau,
                  double tau_abs, double tau_psi, double* margin, bool* near) {
  const double u = (double)(x0 >> 8) * (1.0 / 16777216.0);
  double m = psi[0];
  double mag = std::fabs(psi[0]);
  bool flat = true;
  for (int j = 1; j < A; ++j) {
    m = std::max(m, psi[j]);
    mag = std::max(mag, std::fabs(psi[j]));
    flat = flat && (psi[j] == psi[0]);
  }
  std::vector<double> P(A);
  double run = 0.0;
  for (int j = 0; j < A; ++j) { run += std::exp(eta * (psi[j] - m)); P[j] = run; }
  const double t = u * P[A - 1];
  int a = A - 1;
  for (int j = 0; j < A; ++j)
    if (t < P[j]) { a = j; break; }
  *margin = 1.0;
  *near = false;
  if (!flat) {
    const double lim = (tau + tau_psi * eta * mag) * P[A - 1] + tau_abs;
    for (int j = 0; j + 1 < A; ++j) {
      const double dist = std::fabs(t - P[j]);
      *margin = std::min(*margin, dist / P[A - 1]);
      if (dist <= lim) *near = true;
    }
  }
  return a;
}

struct Particle { int32_t ep; State st; int32_t b; };

template <class Model>
Result* plan(const Model& model, int A, const State* belief, int M,
             const orc_params* prm) {
  Result* res = new Result();
  Tree& T = res->tree;
  const double eta = prm->eta;
  const double gamma = model.gamma;
  const Tree* start = prm->start ? &((const Result*)prm->start)->tree : nullptr;
  const bool kept_root = start && !start->b_parent.empty();
  if (kept_root) {
    T = *start;                                // plan from the kept subtree
    T.set_psi0(A, eta, prm->pi0);
  } else {
    T.init(A, eta, prm->pi0);
  }
  const int K = prm->budget;
  const int n_p = prm->n_particles;
  const int mut = prm->mutate;

  for (int k = 1; k <= K; ++k) {
    const int D = (prm->schedule == 1) ? prm->depth : std::min(k, prm->depth);
    // Alg. 1: sample n_p root states; every episode starts at the root.
    std::vector<Particle> live;
    live.reserve(n_p);
    for (int ep = 0; ep < n_p; ++ep) {
      Words x = draw(prm->seed, (uint32_t)ep, TAG_ROOT, 0, (uint32_t)k, prm->step);
      uint32_t idx = (uint32_t)(((uint64_t)x.w[0] * (uint64_t)M) >> 32);
      live.push_back(Particle{ep, belief[idx], 0});
    }
    // Alg. 2: level-by-level forward search.
    for (int d = 0; d < D; ++d) {
      std::vector<Particle> next;
      next.reserve(live.size());
      for (Particle& P : live) {
        Words x = draw(prm->seed, (uint32_t)P.ep, TAG_STEP, (uint32_t)d,
                       (uint32_t)k, prm->step);
        double margin = 1.0;
        bool near = false;
        int a = sample_action(&T.psi[(size_t)P.b * A], A, eta, x.w[0], prm->tau,
                              prm->tau_abs, prm->tau_psi, &margin, &near);
        res->n_draws++;
        if (near) res->near_ties++;
        res->min_margin = std::min(res->min_margin, margin);
        Outcome o = model.step(P.st, a, x);
        res->particle_steps++;
        int32_t an = T.action_node(P.b, a);       // AppendActions
        T.a_C[an] += (double)o.r;
        T.a_N[an] += 1;
        int32_t bn = -1;
        if (!o.term) {                            // FilterTerminals
          bn = T.belief_node(an, o.obs, eta);     // AppendBeliefs
          next.push_back(Particle{P.ep, o.next, bn});
        }
        if (prm->trace)
          res->trace.push_back(TraceRow{k, d, P.ep, P.b, a, o.obs,
                                        o.term ? 1 : 0, an, near ? 1 : 0, o.r, margin});
      }
      live.swap(next);
    }
    // Alg. 3, leaves: this iteration's visit count and mean heuristic.
    std::unordered_map<int32_t, std::pair<int64_t, double>> leaf;
    std::vector<int32_t> leaf_order;
    for (const Particle& P : live) {
      auto it = leaf.find(P.b);
      if (it == leaf.end()) {
        leaf_order.push_back(P.b);
        it = leaf.emplace(P.b, std::make_pair((int64_t)0, 0.0)).first;
      }
      it->second.first += 1;
      it->second.second += model.heuristic(P.st);
    }
    for (int32_t b : leaf_order) {
      T.b_N[b] = leaf[b].first;
      T.b_V[b] = leaf[b].second / (double)leaf[b].first;
    }
    // Alg. 3, per depth, bottom-up.
    for (int d = D; d >= 1; --d) {
      std::unordered_map<int32_t, double> W;
      if ((int)T.beliefs_at.size() > d)
        for (int32_t c : T.beliefs_at[d])
          W[T.b_parent[c]] += T.b_V[c] * (double)T.b_N[c];
      std::unordered_map<int32_t, double> Q;
      if ((int)T.actions_at.size() > d - 1)
        for (int32_t an : T.actions_at[d - 1]) {
          double n = (double)T.a_N[an];
          double w = W.count(an) ? W[an] : 0.0;
          double g = (mut == 1) ? 1.0 : gamma;            // planted: drop gamma
          Q[an] = T.a_C[an] / n + g * (w / n);
        }
      if ((int)T.beliefs_at.size() <= d - 1) continue;
      for (int32_t b : T.beliefs_at[d - 1]) {
        bool any = false;
        int64_t nb = 0;
        for (int a = 0; a < A; ++a) {
          int32_t an = T.b_child[(size_t)b * A + a];
          if (an >= 0) { any = true; nb += T.a_N[an]; }
        }
        if (!any) continue;
        double* row = &T.psi[(size_t)b * A];
        double vc = lse(row, A, eta);
        if (mut == 2) vc = 0.0;                            // planted: no -V_curr
        for (int a = 0; a < A; ++a) {
          int32_t an = T.b_child[(size_t)b * A + a];
          if (an >= 0) row[a] = (row[a] - vc) + Q[an];
        }
        T.b_N[b] = nb;
        T.b_V[b] = lse(row, A, eta);
      }
    }
  }
  // Alg. 1: act greedily on the root preferences (lowest index on ties).
  int best = 0;
  for (int a = 1; a < A; ++a)
    if (T.psi[a] > T.psi[best]) best = a;
  res->action = best;
  res->v_root = T.b_V[0];
  return res;
}

}  // namespace

extern "C" {

void* orc_plan_tabular(const orc_tabular* m, const int32_t* belief, int32_t M,
                       const orc_params* prm) {
  TabularModel model(m);
  std::vector<State> bel(M);
  for (int i = 0; i < M; ++i) { bel[i].s = belief[i]; bel[i].x = bel[i].y = 0.0f; }
  return plan(model, m->nA, bel.data(), M, prm);
}

void* orc_plan_nav(const orc_nav* m, const float* bx, const float* by,
                   int32_t M, const orc_params* prm) {
  NavModel model(m);
  std::vector<State> bel(M);
  for (int i = 0; i < M; ++i) { bel[i].s = 0; bel[i].x = bx[i]; bel[i].y = by[i]; }
  return plan(model, 4, bel.data(), M, prm);
}

// info: [0] n_beliefs [1] n_actions [2] action [3] particle_steps
//       [4] n_draws [5] near_ties [6] trace rows
void orc_result_info(const void* h, int64_t* info, double* min_margin,
                     double* v_root) {
  const Result* r = (const Result*)h;
  info[0] = (int64_t)r->tree.b_parent.size();
  info[1] = (int64_t)r->tree.a_parent.size();
  info[2] = r->action;
  info[3] = r->particle_steps;
  info[4] = r->n_draws;
  info[5] = r->near_ties;
  info[6] = (int64_t)r->trace.size();
  *min_margin = r->min_margin;
  *v_root = r->v_root;
}

void orc_result_tree(const void* h, int32_t* b_parent, int32_t* b_obs,
                     int32_t* b_depth, double* psi, double* b_V, int64_t* b_N,
                     int32_t* a_parent, int32_t* a_act, double* a_C,
                     int64_t* a_N) {
  const Tree& T = ((const Result*)h)->tree;
  size_t nb = T.b_parent.size(), na = T.a_parent.size();
  std::copy(T.b_parent.begin(), T.b_parent.end(), b_parent);
  std::copy(T.b_obs.begin(), T.b_obs.end(), b_obs);
  std::copy(T.b_depth.begin(), T.b_depth.end(), b_depth);
  std::copy(T.psi.begin(), T.psi.begin() + nb * T.A, psi);
  std::copy(T.b_V.begin(), T.b_V.end(), b_V);
  std::copy(T.b_N.begin(), T.b_N.end(), b_N);
  std::copy(T.a_parent.begin(), T.a_parent.end(), a_parent);
  std::copy(T.a_act.begin(), T.a_act.end(), a_act);
  std::copy(T.a_C.begin(), T.a_C.begin() + na, a_C);
  std::copy(T.a_N.begin(), T.a_N.end(), a_N);
}

// Per-draw trace rows: int32 [rows][8] = k, d, ep, b, a, obs, term, an;
// float r [rows]; double margin [rows].
void orc_result_trace(const void* h, int32_t* ints, float* r, double* margin) {
  const Result* res = (const Result*)h;
  for (size_t i = 0; i < res->trace.size(); ++i) {
    const TraceRow& t = res->trace[i];
    int32_t* o = ints + 8 * i;
    o[0] = t.k; o[1] = t.d; o[2] = t.ep; o[3] = t.b;
    o[4] = t.a; o[5] = t.obs; o[6] = t.term; o[7] = t.an;
    r[i] = t.r;
    margin[i] = t.margin;
  }
}

// The per-draw trace as dense arrays indexed by (level step, episode): level
// step t = step_base[k-1] + d is level d of iteration k.  act [steps*n_p]
// (-1 where no draw), obs, flags: bit 0 drawn, bit 1 terminal, bit 2 near tie.
void orc_result_draws(const void* h, const int32_t* step_base, int32_t n_p, int16_t* act,
                      int32_t* obs, uint8_t* flags) {
  const Result* res = (const Result*)h;
  for (const TraceRow& t : res->trace) {
    const size_t i = (size_t)(step_base[t.k - 1] + t.d) * (size_t)n_p + (size_t)t.ep;
    act[i] = (int16_t)t.a;
    obs[i] = t.obs;
    flags[i] = (uint8_t)(1u | (t.term ? 2u : 0u) | (t.near ? 4u : 0u));
  }
}

void orc_result_free(void* h) { delete (Result*)h; }

// The tree of a finished plan re-rooted at (a, o); a result handle holding
// only the tree (empty when the plan's tree has no such belief).
void* orc_reroot(const void* h, int32_t a, int32_t o) {
  Result* r = new Result();
  r->tree = reroot(((const Result*)h)->tree, a, o);
  if (!r->tree.b_parent.empty()) r->v_root = r->tree.b_V[0];
  return r;
}

// Building blocks exposed for the pins.
void orc_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                uint32_t k0, uint32_t k1, uint32_t* out) {
  Words w = philox4x32_10(c0, c1, c2, c3, k0, k1);
  std::memcpy(out, w.w, sizeof(w.w));
}

void orc_thresholds(const float* p, int32_t n, uint32_t* thr) {
  std::vector<uint32_t> t = thresholds(p, n);
  std::copy(t.begin(), t.end(), thr);
}

int32_t orc_pick(const uint32_t* thr, int32_t n, uint32_t x) {
  return pick(thr, n, x);
}

int32_t orc_sample_action(const double* psi, int32_t A, double eta, uint32_t x0,
                          double tau, double tau_abs, double tau_psi, double* margin,
                          int32_t* near) {
  bool nr = false;
  const int a = sample_action(psi, A, eta, x0, tau, tau_abs, tau_psi, margin, &nr);
  if (near) *near = nr ? 1 : 0;
  return a;
}

// Likelihood of observation key o at navigation position (x, y), in units of
// 2^-24 (the count of noise-index pairs whose observation lands in o's cell).
uint64_t orc_nav_obs_weight(const orc_nav* m, float x, float y, int32_t o) {
  NavModel model(m);
  return model.obs_weight(x, y, o);
}

// One navigation model step, for the fp32 arithmetic pins.
void orc_nav_step(const orc_nav* m, float x, float y, int32_t a, uint32_t w1,
                  uint32_t w2, float* nx, float* ny, int32_t* key, float* r,
                  int32_t* term) {
  NavModel model(m);
  State s; s.s = 0; s.x = x; s.y = y;
  Words w = {{0u, w1, w2, 0u}};
  Outcome o = model.step(s, a, w);
  *nx = o.next.x; *ny = o.next.y; *key = o.obs; *r = o.r; *term = o.term ? 1 : 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Between real steps (Alg. 1: execute, perceive, update the belief).
// ---------------------------------------------------------------------------
namespace {

template <class Model>
Outcome env_step(const Model& model, const State& st, int a, uint64_t seed, uint32_t step) {
  Words x = philox4x32_10(0u, TAG_ENV << 24, 0u, step, (uint32_t)seed,
                          (uint32_t)(seed >> 32));
  return model.step(st, a, x);
}

// SIR update: move every particle under a, weight it by the exact integer
// likelihood of o, draw n new particles multinomially.
template <class Model, class Move, class Weight>
uint64_t pf_update(const Model& model, std::vector<State>& parts, int a, int o, uint64_t seed,
                   uint32_t step, Move mv, Weight wt) {
  const int n = (int)parts.size();
  std::vector<State> moved(n);
  std::vector<uint64_t> cum(n);
  uint64_t total = 0;
  for (int i = 0; i < n; ++i) {
    Words x = philox4x32_10((uint32_t)i, TAG_PF << 24, 0u, step, (uint32_t)seed,
                            (uint32_t)(seed >> 32));
    moved[i] = mv(parts[i], x.w[1]);
    total += wt(moved[i]);
    cum[i] = total;
  }
  if (total == 0) {
    parts = moved;
    return 0;
  }
  for (int j = 0; j < n; ++j) {
    Words y = philox4x32_10((uint32_t)j, TAG_RESAMPLE << 24, 0u, step, (uint32_t)seed,
                            (uint32_t)(seed >> 32));
    const uint64_t u = ((uint64_t)y.w[0] << 32) | y.w[1];
    const uint64_t target = (uint64_t)(((unsigned __int128)u * total) >> 64);
    const int i = (int)(std::upper_bound(cum.begin(), cum.end(), target) - cum.begin());
    parts[j] = moved[i];
  }
  return total;
}

}  // namespace

extern "C" {

void orc_env_step_tabular(const orc_tabular* m, int32_t* s, int32_t a, uint64_t seed,
                          uint32_t step, int32_t* obs, float* r, int32_t* term) {
  TabularModel model(m);
  State st; st.s = *s; st.x = st.y = 0.0f;
  Outcome o = env_step(model, st, a, seed, step);
  *s = o.next.s; *obs = o.obs; *r = o.r; *term = o.term ? 1 : 0;
}

void orc_env_step_nav(const orc_nav* m, float* x, float* y, int32_t a, uint64_t seed,
                      uint32_t step, int32_t* obs, float* r, int32_t* term) {
  NavModel model(m);
  State st; st.s = 0; st.x = *x; st.y = *y;
  Outcome o = env_step(model, st, a, seed, step);
  *x = o.next.x; *y = o.next.y; *obs = o.obs; *r = o.r; *term = o.term ? 1 : 0;
}

uint64_t orc_pf_update_tabular(const orc_tabular* m, int32_t* parts, int32_t n, int32_t a,
                               int32_t o, uint64_t seed, uint32_t step) {
  TabularModel model(m);
  std::vector<State> P(n);
  for (int i = 0; i < n; ++i) { P[i].s = parts[i]; P[i].x = P[i].y = 0.0f; }
  uint64_t tot = pf_update(model, P, a, o, seed, step,
      [&](const State& s, uint32_t w) { State r = s; r.s = model.successor(s.s, a, w); return r; },
      [&](const State& s) { return model.obs_weight(s.s, a, o); });
  for (int i = 0; i < n; ++i) parts[i] = P[i].s;
  return tot;
}

uint64_t orc_pf_update_nav(const orc_nav* m, float* px, float* py, int32_t n, int32_t a,
                           int32_t o, uint64_t seed, uint32_t step) {
  NavModel model(m);
  std::vector<State> P(n);
  for (int i = 0; i < n; ++i) { P[i].s = 0; P[i].x = px[i]; P[i].y = py[i]; }
  uint64_t tot = pf_update(model, P, a, o, seed, step,
      [&](const State& s, uint32_t w) {
        State r = s;
        model.move(s.x, s.y, a, w, &r.x, &r.y);
        return r;
      },
      [&](const State& s) { return model.obs_weight(s.x, s.y, o); });
  for (int i = 0; i < n; ++i) { px[i] = P[i].x; py[i] = P[i].y; }
  return tot;
}

}  // extern "C"

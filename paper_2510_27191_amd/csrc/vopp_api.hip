// vopp_api.hip -- host side of the C ABI declared in include/vopp.h.
//
// Model handles own a device copy of the POMDP (with integer sampling
// thresholds derived here), workspaces own one plan's tree arena, and
// vopp_plan() drives the launches of one planning step (Alg. 1) on a stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/vopp.h"
#include "vopp_device.hpp"
#include "vopp_launch.hpp"
#include "vopp_internal.hpp"

using namespace vopp;

namespace {
thread_local std::string g_err;
}

namespace vopp {

vopp_status fail(vopp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

vopp_status hip_fail(hipError_t e, const char* what) {
  return fail(VOPP_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Sampling thresholds of a categorical row: thr_j = rint(cum_j / total * 2^31)
// with cum the running double sum of the fp32 probabilities; last = 2^31.
static void row_thresholds(const float* p, int n, uint32_t* out) {
  const double two31 = 2147483648.0;
  double total = 0.0;
  for (int j = 0; j < n; ++j) total += (double)p[j];
  double cum = 0.0;
  for (int j = 0; j < n; ++j) {
    cum += (double)p[j];
    double v = std::rint(cum / total * two31);
    v = std::min(std::max(v, 0.0), two31);
    out[j] = (uint32_t)v;
  }
  out[n - 1] = (uint32_t)two31;
}

static bool valid_row(const float* p, int n) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) {
    if (!(p[j] >= 0.0f) || !std::isfinite(p[j])) return false;
    s += (double)p[j];
  }
  return std::fabs(s - 1.0) <= 1e-5;
}

// Entries of a model's ln pi0 row (at least kMaxA, at least |A| rounded up to 4).
static int prior_len(int nA) { return std::max(kMaxA, (nA + 3) / 4 * 4); }

// ln pi0(a) of a reference policy (Eq. 4), normalised by its sequential double
// sum, written to the model's device row of prior_len(nA) entries (zero past
// nA).  A null pi0 gives the uniform row -ln nA.
static hipError_t upload_log_prior(double* dst, int nA, const double* pi0) {
  std::vector<double> row(prior_len(nA), 0.0);
  if (pi0) {
    double sum = 0.0;
    for (int a = 0; a < nA; ++a) sum += pi0[a];
    for (int a = 0; a < nA; ++a) row[a] = std::log(pi0[a] / sum);
  } else {
    for (int a = 0; a < nA; ++a) row[a] = -std::log((double)nA);
  }
  return hipMemcpy(dst, row.data(), row.size() * sizeof(double), hipMemcpyHostToDevice);
}

// Carves aligned sub-buffers out of one device allocation.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t n) {
    off = align_up(off, 256);
    T* p = (T*)(base + off);
    off += n * sizeof(T);
    return p;
  }
};

}  // namespace vopp

extern "C" const char* vopp_last_error(void) { return g_err.c_str(); }
extern "C" const char* vopp_version(void) { return "vopp-mi355x 0.1"; }

// ---------------------------------------------------------------------------
// Models.
// ---------------------------------------------------------------------------
extern "C" vopp_status vopp_pomdp_tabular(const vopp_tabular_desc* d, vopp_pomdp** out) {
  clear_error();
  if (!d || !out) return fail(VOPP_E_INVALID, "null argument");
  *out = nullptr;
  int act_bits = 6;                               // action field of belief keys
  while (d->nA > 0 && (1 << act_bits) < d->nA) ++act_bits;
  const int obs_bits = kKeyLowBits - act_bits;
  if (d->nS < 1 || d->nA < 1 || d->nA > kMaxAWide || d->nO < 1 || d->nO > (1 << obs_bits))
    return fail(VOPP_E_INVALID, "sizes out of range (nS=%d nA=%d nO=%d)", d->nS, d->nA, d->nO);
  if (!(d->gamma > 0.0 && d->gamma < 1.0)) return fail(VOPP_E_INVALID, "gamma must be in (0,1)");
  if (!d->rowptr || !d->col || !d->tprob || !d->zprob || !d->reward)
    return fail(VOPP_E_INVALID, "null model array");
  const long long rows = (long long)d->nS * d->nA;
  if (rows > INT32_MAX / 2 || rows * d->nO > (long long)1 << 40)
    return fail(VOPP_E_INVALID, "model too large");
  if (d->rowptr[0] != 0) return fail(VOPP_E_INVALID, "rowptr[0] must be 0");
  for (long long r = 0; r < rows; ++r) {
    if (d->rowptr[r + 1] <= d->rowptr[r])
      return fail(VOPP_E_INVALID, "transition row %lld is empty or rowptr decreases", r);
  }
  const int nnz = d->rowptr[rows];
  for (int i = 0; i < nnz; ++i)
    if (d->col[i] < 0 || d->col[i] >= d->nS)
      return fail(VOPP_E_INVALID, "successor index %d out of range at %d", d->col[i], i);
  for (long long r = 0; r < rows; ++r) {
    int lo = d->rowptr[r], n = d->rowptr[r + 1] - lo;
    if (!valid_row(d->tprob + lo, n))
      return fail(VOPP_E_INVALID, "transition row %lld does not sum to 1", r);
    if (!valid_row(d->zprob + r * d->nO, d->nO))
      return fail(VOPP_E_INVALID, "observation row %lld does not sum to 1", r);
  }
  double rmax = 0.0, hmax = 0.0;
  for (long long i = 0; i < rows; ++i) {
    if (!std::isfinite(d->reward[i])) return fail(VOPP_E_INVALID, "non-finite reward");
    rmax = std::max(rmax, (double)std::fabs(d->reward[i]));
  }
  if (d->heur)
    for (int i = 0; i < d->nS; ++i) {
      if (!std::isfinite(d->heur[i])) return fail(VOPP_E_INVALID, "non-finite heuristic");
      hmax = std::max(hmax, (double)std::fabs(d->heur[i]));
    }

  std::vector<uint32_t> thrT(nnz), thrZ((size_t)rows * d->nO);
  for (long long r = 0; r < rows; ++r) {
    int lo = d->rowptr[r], n = d->rowptr[r + 1] - lo;
    row_thresholds(d->tprob + lo, n, thrT.data() + lo);
    row_thresholds(d->zprob + r * d->nO, d->nO, thrZ.data() + r * d->nO);
  }

  vopp_pomdp* p = new vopp_pomdp();
  p->kind = kTabular;
  p->nA = d->nA;
  p->r_max = rmax;
  p->h_max = hmax;
  p->gamma = d->gamma;
  p->branch = (double)d->nA * d->nO;
  (void)hipGetDevice(&p->device);
  size_t bytes = 0;
  bytes += align_up((rows + 1) * 4, 256) + align_up((size_t)nnz * 4, 256) * 2;
  bytes += align_up(thrZ.size() * 4, 256) + align_up(rows * 4, 256) +
           align_up((size_t)d->nS * 4, 256) + align_up((size_t)prior_len(d->nA) * 8, 256) + 1024;
  hipError_t e = hipMalloc(&p->arena, bytes);
  if (e != hipSuccess) { delete p; return hip_fail(e, "hipMalloc(model)"); }
  p->bytes = bytes;
  Carver c(p->arena);
  int* rowptr = c.take<int>(rows + 1);
  int* col = c.take<int>(nnz);
  uint32_t* tT = c.take<uint32_t>(nnz);
  uint32_t* tZ = c.take<uint32_t>(thrZ.size());
  float* R = c.take<float>(rows);
  float* H = d->heur ? c.take<float>(d->nS) : nullptr;
  double* logpi0 = c.take<double>(prior_len(d->nA));
  e = hipMemcpy(rowptr, d->rowptr, (rows + 1) * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(col, d->col, (size_t)nnz * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(tT, thrT.data(), (size_t)nnz * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(tZ, thrZ.data(), thrZ.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(R, d->reward, rows * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && H) e = hipMemcpy(H, d->heur, (size_t)d->nS * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = upload_log_prior(logpi0, d->nA, nullptr);
  if (e != hipSuccess) { (void)hipFree(p->arena); delete p; return hip_fail(e, "hipMemcpy(model)"); }
  ModelView& m = p->view;
  std::memset(&m, 0, sizeof(m));
  m.kind = kTabular;
  m.nS = d->nS; m.nA = d->nA; m.nO = d->nO;
  m.Apad = (d->nA + 3) / 4 * 4;
  m.rowptr = rowptr; m.col = col; m.thrT = tT; m.thrZ = tZ; m.R = R; m.H = H;
  m.logpi0 = logpi0;
  m.obs_bits = obs_bits;
  m.gamma = (float)d->gamma;
  m.gamma64 = d->gamma;
  *out = p;
  return VOPP_OK;
}

extern "C" vopp_status vopp_pomdp_nav2d(const vopp_nav2d_desc* d, vopp_pomdp** out) {
  clear_error();
  if (!d || !out) return fail(VOPP_E_INVALID, "null argument");
  *out = nullptr;
  if (!(d->gamma > 0.0 && d->gamma < 1.0)) return fail(VOPP_E_INVALID, "gamma must be in (0,1)");
  if (!d->gauss) return fail(VOPP_E_INVALID, "null Gaussian table");
  if (d->n_disks < 0 || d->n_disks > 4096 || (d->n_disks > 0 && !d->disks))
    return fail(VOPP_E_INVALID, "bad obstacle list");
  if (!(d->hi > d->lo) || d->key_n < 1 || d->key_n > 1024 || !(d->inv_bin > 0.0f))
    return fail(VOPP_E_INVALID, "bad navigation geometry");
  for (int i = 0; i < 4096; ++i)
    if (!std::isfinite(d->gauss[i])) return fail(VOPP_E_INVALID, "non-finite Gaussian table");
  vopp_pomdp* p = new vopp_pomdp();
  p->kind = kNav;
  p->nA = 4;
  p->gamma = d->gamma;
  double rs = d->r_step, rg = d->r_goal, rh = d->r_hit;
  p->r_max = std::max({std::fabs(rs), std::fabs(rs + rg), std::fabs(rs + rh),
                       std::fabs(rs + rg + rh)});
  p->h_max = d->heuristic ? 2.0 * (double)(d->hi - d->lo) + 1.0 : 0.0;
  p->branch = 4.0 * (double)d->key_n * d->key_n;
  (void)hipGetDevice(&p->device);
  size_t bytes = align_up(4096 * 4, 256) + align_up((size_t)2 * d->n_disks * 4 + 4, 256) +
                 align_up(kMaxA * 8, 256) + 512;
  hipError_t e = hipMalloc(&p->arena, bytes);
  if (e != hipSuccess) { delete p; return hip_fail(e, "hipMalloc(model)"); }
  p->bytes = bytes;
  Carver c(p->arena);
  float* g = c.take<float>(4096);
  float* disks = c.take<float>(2 * (size_t)d->n_disks + 1);
  double* logpi0 = c.take<double>(prior_len(4));
  e = hipMemcpy(g, d->gauss, 4096 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && d->n_disks)
    e = hipMemcpy(disks, d->disks, 2 * (size_t)d->n_disks * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = upload_log_prior(logpi0, 4, nullptr);
  if (e != hipSuccess) { (void)hipFree(p->arena); delete p; return hip_fail(e, "hipMemcpy(model)"); }
  ModelView& m = p->view;
  std::memset(&m, 0, sizeof(m));
  m.kind = kNav;
  m.nS = 0; m.nA = 4; m.nO = d->key_n * d->key_n; m.Apad = 4;
  NavParams& np = m.nav;
  np.lo = d->lo; np.hi = d->hi; np.step = d->step; np.sigma_move = d->sigma_move;
  np.sigma_obs0 = d->sigma_obs0; np.sigma_obs_slope = d->sigma_obs_slope;
  np.obs_center_x = d->obs_center_x; np.inv_bin = d->inv_bin;
  np.key_lo = d->key_lo; np.key_n = d->key_n;
  np.goal_x = d->goal_x; np.goal_y = d->goal_y; np.goal_r2 = d->goal_r2;
  np.disk_r2 = d->disk_r2; np.r_step = d->r_step; np.r_goal = d->r_goal;
  np.r_hit = d->r_hit; np.heuristic = d->heuristic; np.n_disks = d->n_disks;
  m.gauss = g; m.disks = disks;
  m.logpi0 = logpi0;
  m.obs_bits = kObsBits;
  m.gamma = (float)d->gamma;
  m.gamma64 = d->gamma;
  *out = p;
  return VOPP_OK;
}

extern "C" int32_t vopp_pomdp_num_actions(const vopp_pomdp* p) { return p ? p->nA : 0; }

extern "C" vopp_status vopp_pomdp_set_reference_policy(vopp_pomdp* p, const double* pi0) {
  clear_error();
  if (!p) return fail(VOPP_E_INVALID, "null model");
  if (pi0)
    for (int a = 0; a < p->nA; ++a)
      if (!(std::isfinite(pi0[a]) && pi0[a] > 0.0))
        return fail(VOPP_E_INVALID, "reference policy entry %d is not a positive finite number", a);
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != p->device)
    return fail(VOPP_E_INVALID, "model lives on device %d, current is %d", p->device, dev);
  const hipError_t e = upload_log_prior(const_cast<double*>(p->view.logpi0), p->nA, pi0);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(reference policy)");
  return VOPP_OK;
}

extern "C" void vopp_pomdp_free(vopp_pomdp* p) {
  if (!p) return;
  if (p->own_ws) vopp_workspace_free(p->own_ws);
  if (p->filt) (void)hipFree(p->filt);
  if (p->arena) (void)hipFree(p->arena);
  delete p;
}

// ---------------------------------------------------------------------------
// Workspaces.
// ---------------------------------------------------------------------------
namespace vopp {

int sum_depths(int K, int depth, int schedule) {
  long long s = 0;
  for (int k = 1; k <= K; ++k) s += schedule == VOPP_SCHEDULE_FIXED ? depth : std::min(k, depth);
  return (int)s;
}

WsSizes sizes_for(const vopp_pomdp* p, int n_p, int K, int depth, int schedule,
                  int extra_steps) {
  WsSizes z;
  z.n_p = n_p;
  z.steps = sum_depths(K, depth, schedule) + extra_steps;
  z.K = K;
  z.depth = depth;
  z.Apad = p->view.Apad;
  z.rs = rec_bytes(z.Apad);
  z.cap_b = 1 + (long long)n_p * z.steps;
  uint64_t h = 1024;
  while (h < 2 * (uint64_t)z.cap_b) h <<= 1;      // load <= 1/2
  z.hcap = h;
  return z;
}

// Doubles of a workspace's result record: action, |A| root preferences, V,
// counts and flags.
size_t out_len(const WsSizes& z) { return (size_t)std::max(kOutStride, z.Apad + 12); }

size_t bytes_for(const WsSizes& z) {
  size_t b = 0;
  auto add = [&](size_t n) { b += align_up(n, 256); };
  const size_t cb = (size_t)z.cap_b;                 // the belief field arrays
  add(cb * z.Apad * 4); add(cb * z.Apad * 4); add(cb * z.Apad * 8); add(cb * z.Apad * 8);
  add(cb * sizeof(BeliefHot)); add(cb * sizeof(BeliefLeaf));
  add(cb * (size_t)rec_bitmap_words(z.Apad) * 4);
  add(z.hcap * sizeof(HSlot));                       // table
  const size_t ar = (size_t)std::max(kMaxA, z.Apad);
  add(ar * 8); add(ar * 8); add(8);                  // root row and its CDF, V(root)
  add(ar * 8);                                       // running sums of the initial row
  add(ar * 4);                                       // initial preference row
  add((size_t)3 * z.Apad * kStripes * 8);            // striped root action nodes
  add((size_t)z.steps * z.n_p * 4);                  // level-step lists
  add(64); add(kStatRows * kStripes * 8); add(32); add((z.K + 1) * 4);
  add(2 * (kMaxDepth + 1) * 4);                      // kept-subtree steps by depth
  add((size_t)(z.depth + 1) * z.n_p * 8);            // trace words
  add((size_t)(z.depth + 1) * z.n_p * 4);            // trace values
  add(out_len(z) * 8);                               // result record
  return b + 4096;
}

bool fits(const WsSizes& have, const WsSizes& need) {
  return have.n_p >= need.n_p && have.cap_b >= need.cap_b && have.steps >= need.steps &&
         have.K >= need.K && have.Apad >= need.Apad && have.depth >= need.depth &&
         have.hcap >= need.hcap;
}

// Lays out the buffers of one plan's tree (sizes z) in device memory at base,
// bytes_for(z) of it, in the order bytes_for counts them.
void carve_tree(void* base, const WsSizes& z, TreeView& t, int** carry_rng, int** step_base,
                double** out) {
  Carver c(base);
  const size_t cb = (size_t)z.cap_b;
  t.ra = z.Apad;
  t.bw = rec_bitmap_words(z.Apad);
  t.psi = c.take<float>(cb * z.Apad);
  t.nv = c.take<int>(cb * z.Apad);
  t.cv = c.take<unsigned long long>(cb * z.Apad);
  t.wv = c.take<unsigned long long>(cb * z.Apad);
  t.hot = c.take<BeliefHot>(cb);
  t.leaf = c.take<BeliefLeaf>(cb);
  t.bits = c.take<uint32_t>(cb * (size_t)t.bw);
  t.h_slot = c.take<HSlot>(z.hcap);
  t.h_mask = (uint32_t)(z.hcap - 1);
  const size_t ar = (size_t)std::max(kMaxA, z.Apad);
  t.psi_root = c.take<double>(ar);
  t.psi0 = c.take<float>(ar);
  t.root_cdf = c.take<double>(ar);
  t.psi0_cdf64 = c.take<double>(ar);
  t.root_acc = c.take<unsigned long long>((size_t)3 * z.Apad * kStripes);
  t.v_root = c.take<double>(1);
  t.list = c.take<int>((size_t)z.steps * z.n_p);
  t.counters = c.take<unsigned long long>(8);
  t.stats = c.take<unsigned long long>(kStatRows * kStripes);
  t.gate = c.take<unsigned long long>(4);
  *carry_rng = c.take<int>(2 * (kMaxDepth + 1));
  t.carry_rng = *carry_rng;
  *step_base = c.take<int>(z.K + 1);
  t.step_base = *step_base;
  t.tr_key = c.take<unsigned long long>((size_t)(z.depth + 1) * z.n_p);
  t.tr_val = c.take<float>((size_t)(z.depth + 1) * z.n_p);
  *out = c.take<double>(out_len(z));
}

vopp_status ws_alloc(const WsSizes& z, vopp_workspace** out) {
  vopp_workspace* w = new vopp_workspace();
  w->z = z;
  w->bytes = bytes_for(z);
  (void)hipGetDevice(&w->device);
  hipError_t e = hipMalloc(&w->arena, w->bytes);
  if (e != hipSuccess) {
    delete w;
    return fail(VOPP_E_NOMEM, "hipMalloc(%zu bytes) for the workspace: %s", bytes_for(z),
                hipGetErrorString(e));
  }
  TreeView& t = w->tree;
  carve_tree(w->arena, z, t, &w->carry_rng_dev, &w->step_base_dev, &w->out_dev);
  e = hipHostMalloc((void**)&w->out_host, out_len(z) * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&w->step_host, (kMaxBudget + 8) * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) {
    // step_host[kMaxBudget + 1 ..] holds the 64-bit constant 1 (dirty flag).
    const unsigned long long one = 1ull;
    std::memcpy(&w->step_host[kMaxBudget + 1], &one, sizeof(one));
  }
  if (e == hipSuccess) e = hipEventCreate(&w->ev0);
  if (e == hipSuccess) e = hipEventCreate(&w->ev1);
  if (e != hipSuccess) {
    vopp_workspace_free(w);
    return hip_fail(e, "workspace set-up");
  }
  // Counters: [3] = 1 marks the belief table as dirty (fully cleared by the
  // next plan's set-up).
  unsigned long long init[8] = {0, 0, 0, 1, 0, 0, 0, 0};
  e = hipMemcpy(t.counters, init, sizeof(init), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    vopp_workspace_free(w);
    return hip_fail(e, "workspace counters");
  }
  w->hash_dirty = false;
  *out = w;
  return VOPP_OK;
}

vopp_status check_params(const vopp_pomdp* p, const vopp_params* prm, int32_t budget,
                         int32_t depth) {
  if (!p) return fail(VOPP_E_INVALID, "null pomdp");
  if (!prm) return fail(VOPP_E_INVALID, "null params");
  if (prm->n_particles < 1 || prm->n_particles > (1 << 24))
    return fail(VOPP_E_INVALID, "n_particles must be in [1, 2^24]");
  if (budget < 1 || budget > kMaxBudget)
    return fail(VOPP_E_INVALID, "budget must be in [1, %d]", kMaxBudget);
  if (depth < 1 || depth > 64) return fail(VOPP_E_INVALID, "depth must be in [1, 64]");
  if (!(prm->eta > 0.0) || !std::isfinite(prm->eta)) return fail(VOPP_E_INVALID, "eta must be > 0");
  if (prm->schedule != VOPP_SCHEDULE_DEEPEN && prm->schedule != VOPP_SCHEDULE_FIXED)
    return fail(VOPP_E_INVALID, "unknown schedule");
  const long long steps = sum_depths(budget, depth, prm->schedule);
  if ((long long)prm->n_particles * steps + 1 > kMaxBeliefs)
    return fail(VOPP_E_INVALID, "n_particles * sum of depths exceeds 2^28 beliefs");
  return VOPP_OK;
}

}  // namespace vopp

extern "C" size_t vopp_plan_footprint(const vopp_pomdp* p, const vopp_params* prm,
                                      int32_t budget, int32_t depth) {
  if (check_params(p, prm, budget, depth) != VOPP_OK) return 0;
  return bytes_for(sizes_for(p, prm->n_particles, budget, depth, prm->schedule));
}

extern "C" vopp_status vopp_workspace_create(const vopp_pomdp* p, const vopp_params* prm,
                                             int32_t budget, int32_t depth,
                                             vopp_workspace** out) {
  clear_error();
  if (!out) return fail(VOPP_E_INVALID, "null out");
  *out = nullptr;
  vopp_status st = check_params(p, prm, budget, depth);
  if (st != VOPP_OK) return st;
  return ws_alloc(sizes_for(p, prm->n_particles, budget, depth, prm->schedule), out);
}

extern "C" void vopp_workspace_free(vopp_workspace* w) {
  if (!w) return;
  if (w->arena) (void)hipFree(w->arena);
  if (w->out_host) (void)hipHostFree(w->out_host);
  if (w->step_host) (void)hipHostFree(w->step_host);
  if (w->gate_host) (void)hipHostFree(w->gate_host);
  if (w->ev0) (void)hipEventDestroy(w->ev0);
  if (w->ev1) (void)hipEventDestroy(w->ev1);
  for (hipEvent_t ev : w->prof_events) (void)hipEventDestroy(ev);
  delete w;
}

// ---------------------------------------------------------------------------
// One planning step.
// ---------------------------------------------------------------------------
namespace vopp {

// Fixed-point scale 2^S for the cross-episode sums: every partial sum is
// bounded by n_p * K * vmax with vmax >= |V| = R_max/(1-gamma) + H_max, and S
// keeps that bound below 2^61.
int fixed_shift(const vopp_pomdp* p, double visits) {
  const double vmax = p->r_max / (1.0 - p->gamma) + p->h_max + 1.0;
  const double lg = std::log2(visits * vmax);
  int S = (int)std::floor(61.0 - lg);
  return std::min(std::max(S, 4), 40);
}

PlanView make_view(const vopp_pomdp* p, vopp_workspace* w, const void* belief,
                   int n_belief, int K, int depth, const vopp_params* prm) {
  PlanView P;
  std::memset(&P, 0, sizeof(P));
  P.m = p->view;
  P.t = w->tree;
  P.e.belief = belief;
  P.e.n_belief = n_belief;
  P.n_p = prm->n_particles;
  P.eta = (float)prm->eta;
  P.eta64 = prm->eta;
  P.seed_lo = (uint32_t)prm->seed;
  P.seed_hi = (uint32_t)(prm->seed >> 32);
  P.step = prm->step;
  // A kept subtree's sums were scaled when it was kept, for a bound on the
  // iterations that covers this plan.
  const bool carry = w->carry.pending;
  const int S = carry ? w->carry.shift : fixed_shift(p, (double)prm->n_particles * (double)K);
  P.fix_scale = std::ldexp(1.0f, S);
  P.fix_inv = std::ldexp(1.0f, -S);
  P.fix_inv64 = std::ldexp(1.0, -S);
  P.K = K;
  P.depth = depth;
  P.schedule = prm->schedule;
  P.steps = sum_depths(K, depth, prm->schedule) + (carry ? w->carry.n_steps : 0);
  P.carry = carry ? 1 : 0;
  P.out = w->out_dev;
  return P;
}

// Grid for a backup sweep over the beliefs of depth `dep` after iteration k.
int backup_grid(const vopp_pomdp* p, int n_p, const int* D, int dep, int k,
                int cap, int extra, bool wide) {
  (void)p;
  // One chunk of record positions per block over the level steps that hold
  // depth dep: kBlock positions (a thread each), or 64 for the sweeps of long
  // rows (a wavefront per 16 positions), which may use four times the blocks.
  long long iters = extra;
  for (int kk = 1; kk <= k; ++kk) iters += D[kk] >= dep ? 1 : 0;
  const int per = wide ? 64 : kBlock;
  const long long g = ((long long)n_p + per - 1) / per * iters;
  return (int)std::max(1ll, std::min(g, (long long)cap * (wide ? 4 : 1)));
}

// Enqueue one planning step on stream s.  Returns the level-step count.
// Anytime plans: iterations enqueued ahead of the last finished one.  Two
// keep the device busy while the host enqueues the next.
constexpr int kTimedAhead = 2;

// Before iteration k of an anytime plan is enqueued: wait until fewer than
// kTimedAhead iterations are in flight.  *go is false once the device has
// stopped the plan (budget spent or K reached).
static vopp_status timed_gate(const vopp_workspace* w, hipStream_t s, int k, bool* go) {
  for (;;) {
    const unsigned long long g = __atomic_load_n(w->gate_host, __ATOMIC_ACQUIRE);
    if (g >> 32) { *go = false; return VOPP_OK; }
    if (k - 1 - (int)(g & 0xffffffffull) < kTimedAhead) { *go = true; return VOPP_OK; }
    // The stream may have drained (the word is then final): read it once more.
    const hipError_t q = hipStreamQuery(s);
    if (q == hipSuccess) {
      const unsigned long long g2 = __atomic_load_n(w->gate_host, __ATOMIC_ACQUIRE);
      if (g2 >> 32) { *go = false; return VOPP_OK; }
      if (k - 1 - (int)(g2 & 0xffffffffull) < kTimedAhead) { *go = true; return VOPP_OK; }
      return fail(VOPP_E_INTERNAL, "anytime plan: iteration %d not reported by the device", k - 1);
    }
    if (q != hipErrorNotReady) return hip_fail(q, "anytime plan");
    std::this_thread::yield();
  }
}

vopp_status enqueue_plan(const vopp_pomdp* p, vopp_workspace* w, const PlanView& P,
                         hipStream_t s, int* n_steps_out) {
  const int K = P.K;
  int D[kMaxBudget + 1] = {0};
  const int c0 = P.carry ? w->carry.n_steps : 0;   // a kept subtree's steps first
  int steps = c0;
  hipError_t e = hipSuccess;
  if (!P.clear_all) w->step_host[0] = c0;
  for (int k = 1; k <= K; ++k) {
    D[k] = P.schedule == VOPP_SCHEDULE_FIXED ? P.depth : std::min(k, P.depth);
    steps += D[k];
    if (!P.clear_all) w->step_host[k] = steps;
  }
  // Without a workspace (P.clear_all) the set-up kernel writes the schedule.
  if (!P.clear_all)
    e = hipMemcpyAsync(w->step_base_dev, w->step_host, (K + 1) * sizeof(int),
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "upload schedule");
  w->prof_used = 0;
  // Each launch below is bracketed by prof_begin/prof_end (no-ops unless
  // profiling is enabled on the workspace); prof_end runs whenever prof_begin
  // did, so no bracket stays open past its launch.
#define VOPP_TIMED(kind, call)                              \
  do {                                                      \
    if (e == hipSuccess) {                                  \
      e = prof_begin(w, kind, s);                           \
      if (e == hipSuccess) e = (call);                      \
      const hipError_t e_end = prof_end(w, s);              \
      if (e == hipSuccess) e = e_end;                       \
    }                                                       \
  } while (0)
  if (w->hash_dirty && !P.clear_all) {
    // A plan did not finish: the table state is unknown, clear it fully.
    e = hipMemcpyAsync(&w->tree.counters[3], &w->step_host[kMaxBudget + 1],
                       sizeof(unsigned long long), hipMemcpyHostToDevice, s);
  }
  VOPP_TIMED(VOPP_KERNEL_SETUP, launch_setup(P, s));
  if (e != hipSuccess) return hip_fail(e, "plan set-up launch");
  w->hash_dirty = true;   // until the plan has finished
  int t = c0;
  for (int k = 1; k <= K; ++k) {
    if (P.timed && k > 1) {
      bool go = true;
      const vopp_status gs = timed_gate(w, s, k, &go);
      if (gs != VOPP_OK) return gs;
      if (!go) break;
    }
    VOPP_TIMED(VOPP_KERNEL_FORWARD, launch_forward(P, k, D[k], s));
    VOPP_TIMED(VOPP_KERNEL_ACCUMULATE,
               launch_accum(P, D[k], accum_blocks(P, D[k], kAccumCap), s));
    if (e != hipSuccess) return hip_fail(e, "forward-search launch");
    t += D[k];
    VOPP_TIMED(VOPP_KERNEL_BACKUP_LEAF,
               launch_backup_leaf(P, D[k], k,
                                  backup_grid(p, P.n_p, D, D[k], k, kBackupCap,
                                              P.carry ? w->carry.count[D[k]] : 0), s));
    for (int dep = D[k]; dep >= 2; --dep)
      VOPP_TIMED(VOPP_KERNEL_BACKUP_LEVEL,
                 launch_backup_level(P, dep, k,
                                     backup_grid(p, P.n_p, D, dep - 1, k, kBackupCap,
                                                 P.carry ? w->carry.count[dep - 1] : 0,
                                                 P.m.Apad > kMaxA), s));
    VOPP_TIMED(VOPP_KERNEL_BACKUP_ROOT, launch_backup_root(P, k, s));
    if (e != hipSuccess) return hip_fail(e, "backup launch");
  }
  VOPP_TIMED(VOPP_KERNEL_SELECT, launch_select(P, s));
#undef VOPP_TIMED
  if (e != hipSuccess) return hip_fail(e, "select launch");
  *n_steps_out = t;
  return VOPP_OK;
}

// A bracket's events are the start and end timestamps of its launches' own
// dispatches (launch_timing), the times a kernel trace reports, not markers
// recorded on the stream around them.
hipError_t prof_begin(vopp_workspace* w, int kind, hipStream_t s) {
  (void)s;
  w->prof_open = w->prof_on && ((w->prof_mask >> kind) & 1u);
  if (!w->prof_open) return hipSuccess;
  while (w->prof_events.size() < w->prof_used + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      w->prof_open = false;
      return e;
    }
    w->prof_events.push_back(ev);
  }
  if (w->prof_kinds.size() < w->prof_used / 2 + 1) w->prof_kinds.resize(w->prof_used / 2 + 1);
  w->prof_kinds[w->prof_used / 2] = kind;
  launch_timing() = LaunchTiming{w->prof_events[w->prof_used], w->prof_events[w->prof_used + 1],
                                 false};
  return hipSuccess;
}

hipError_t prof_end(vopp_workspace* w, hipStream_t s) {
  if (!w->prof_open) return hipSuccess;
  w->prof_open = false;
  const bool used = launch_timing().used;
  launch_timing() = LaunchTiming{};
  hipError_t e = hipSuccess;
  if (!used) {
    // Nothing was launched: an empty bracket.
    e = hipEventRecord(w->prof_events[w->prof_used], s);
    if (e == hipSuccess) e = hipEventRecord(w->prof_events[w->prof_used + 1], s);
  }
  w->prof_used += 2;
  return e;
}

void prof_collect(vopp_workspace* w) {
  if (!w->prof_on) return;
  for (size_t i = 0; i + 1 < w->prof_used; i += 2) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, w->prof_events[i], w->prof_events[i + 1]) == hipSuccess) {
      const int kind = w->prof_kinds[i / 2];
      w->prof_ms[kind] += ms;
      w->prof_count[kind] += 1;
    }
  }
  w->prof_used = 0;
}

vopp_status ensure_ws(const vopp_pomdp* p, vopp_workspace** ws, const vopp_params* prm,
                      int K, int depth) {
  const WsSizes need = sizes_for(p, prm->n_particles, K, depth, prm->schedule);
  vopp_workspace* w = *ws;
  if (w && fits(w->z, need)) return VOPP_OK;
  if (w) {
    vopp_workspace_free(w);
    *ws = nullptr;
  }
  return ws_alloc(need, ws);
}

}  // namespace vopp

namespace vopp {
// vopp_plan (time_ms = 0) and vopp_plan_anytime (time_ms > 0; budget is then
// the iteration cap).
// draw_act / draw_obs: the optional per-draw export (vopp_plan_trace).
static vopp_status plan_common(const vopp_pomdp* p, const void* belief, int32_t n_belief,
                               int32_t budget, int32_t depth, const vopp_params* prm,
                               vopp_workspace* ws, void* stream, double time_ms,
                               int32_t* action, double* values, double* v_root,
                               vopp_stats* stats, int32_t* iterations,
                               int16_t* draw_act = nullptr, int32_t* draw_obs = nullptr,
                               const int16_t* force_act = nullptr, int64_t trace_len = 0) {
  vopp_status st = check_params(p, prm, budget, depth);
  if (st != VOPP_OK) return st;
  if ((draw_act == nullptr) != (draw_obs == nullptr))
    return fail(VOPP_E_INVALID, "the draw trace needs both arrays");
  if (draw_act &&
      trace_len < (int64_t)sum_depths(budget, depth, prm->schedule) * prm->n_particles)
    return fail(VOPP_E_INVALID, "draw trace holds %lld entries, the plan needs %lld",
                (long long)trace_len,
                (long long)sum_depths(budget, depth, prm->schedule) * prm->n_particles);
  if (!belief || n_belief < 1) return fail(VOPP_E_INVALID, "empty belief");
  if (!action) return fail(VOPP_E_INVALID, "null action pointer");
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != p->device) return fail(VOPP_E_INVALID, "model lives on device %d, current is %d", p->device, dev);
  if (ws && ws->carry.pending) {
    // The plan starts from the subtree kept by vopp_reroot.
    if (prm->n_particles != ws->carry.n_p)
      return fail(VOPP_E_INVALID, "a plan from a kept subtree must use n_particles = %d",
                  ws->carry.n_p);
    if (budget > ws->carry.budget)
      return fail(VOPP_E_INVALID, "the kept subtree was prepared for at most %d iterations",
                  ws->carry.budget);
    if (!fits(ws->z, sizes_for(p, prm->n_particles, budget, depth, prm->schedule,
                               ws->carry.n_steps)))
      return fail(VOPP_E_INVALID, "workspace too small for this plan and its kept subtree");
  } else if (ws) {
    if (!fits(ws->z, sizes_for(p, prm->n_particles, budget, depth, prm->schedule)))
      return fail(VOPP_E_INVALID, "workspace too small for this plan");
  } else {
    vopp_pomdp* mp = const_cast<vopp_pomdp*>(p);
    st = ensure_ws(p, &mp->own_ws, prm, budget, depth);
    if (st != VOPP_OK) return st;
    ws = mp->own_ws;
  }
  if (ws->z.Apad < p->view.Apad) return fail(VOPP_E_INVALID, "workspace built for fewer actions");
  hipStream_t s = (hipStream_t)stream;
  PlanView P = make_view(p, ws, belief, n_belief, budget, depth, prm);
  if (draw_act) {
    P.t.dbg_act = draw_act;
    P.t.dbg_obs = draw_obs;
    P.t.dbg_force = force_act;
    P.t.dbg_step0 = P.carry ? ws->carry.n_steps : 0;
  }
  hipError_t e = hipSuccess;
  if (time_ms > 0.0) {
    int khz = 0;
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device);
    if (e != hipSuccess) return hip_fail(e, "wall-clock rate");
    if (khz <= 0) return fail(VOPP_E_DEVICE, "the device reports no wall-clock rate");
    if (!ws->gate_host) {
      e = hipHostMalloc((void**)&ws->gate_host, 64, hipHostMallocMapped | hipHostMallocCoherent);
      if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&ws->gate_dev, ws->gate_host, 0);
      if (e != hipSuccess) return hip_fail(e, "anytime gate");
    }
    __atomic_store_n(ws->gate_host, 0ull, __ATOMIC_RELEASE);
    P.timed = 1;
    P.budget_ticks = (unsigned long long)std::max(1.0, std::floor(time_ms * (double)khz));
    P.gate_host = ws->gate_dev;
  }
  e = hipEventRecord(ws->ev0, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  int steps = 0;
  st = enqueue_plan(p, ws, P, s, &steps);
  if (st != VOPP_OK) return st;
  const int A = p->nA;
  e = hipMemcpyAsync(ws->out_host, ws->out_dev, out_len(ws->z) * sizeof(double),
                     hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(ws->ev1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "plan execution");
  prof_collect(ws);
  const double* o = ws->out_host;
  ws->n_prev_beliefs = (int)o[A + 3];
  ws->hash_dirty = false;
  const int flags = (int)o[A + 5];
  if (flags & 1) return fail(VOPP_E_INVALID, "a belief particle holds a state outside [0, nS)");
  if (flags & 2) return fail(VOPP_E_INTERNAL, "belief table overflow");
  int k_run = budget;
  const int c0 = P.carry ? ws->carry.n_steps : 0;
  if (P.timed) {
    k_run = (int)(__atomic_load_n(ws->gate_host, __ATOMIC_ACQUIRE) & 0xffffffffull);
    if (k_run < 1 || k_run > budget)
      return fail(VOPP_E_INTERNAL, "anytime plan reported %d iterations", k_run);
    steps = c0 + sum_depths(k_run, depth, prm->schedule);
  }
  if (iterations) *iterations = k_run;
  // The backups count the beliefs of depth <= D_K and the action nodes of
  // beliefs shallower than D_K.  A kept subtree may reach deeper; no episode
  // of this plan went there, so those parts are as kept.
  long long nb = (long long)o[A + 3], na = (long long)o[A + 4];
  const int D_last = prm->schedule == VOPP_SCHEDULE_FIXED ? depth : std::min(k_run, depth);
  if (P.carry)
    for (int d = 1; d <= kMaxDepth; ++d) {
      if (d > D_last) nb += ws->carry.beliefs[d];
      if (d >= D_last) na += ws->carry.nodes[d];
    }
  // Level-step depths of this tree.
  ws->step_depth.clear();
  if (P.carry)
    for (int d = 1; d <= kMaxDepth; ++d)
      for (int i = 0; i < ws->carry.count[d]; ++i) ws->step_depth.push_back(d);
  for (int k = 1; k <= k_run; ++k) {
    const int D = prm->schedule == VOPP_SCHEDULE_FIXED ? depth : std::min(k, depth);
    for (int d = 0; d < D; ++d) ws->step_depth.push_back(d + 1);
  }
  ws->carried = P.carry != 0;
  ws->carry.pending = false;
  *action = (int32_t)o[0];
  if (values) for (int j = 0; j < A; ++j) values[j] = o[1 + j];
  if (v_root) *v_root = o[A + 1];
  ws->n_prev_beliefs = (int)nb;
  ws->n_prev_actions = (int)na;
  ws->hash_dirty = false;
  ws->last_A = A;
  ws->last_apad = p->view.Apad;
  ws->last_steps = steps;
  ws->last_n_p = prm->n_particles;
  ws->last_K = k_run;
  ws->last_depth = depth;
  ws->last_schedule = prm->schedule;
  ws->last_fix_inv64 = P.fix_inv64;
  if (stats) {
    stats->particle_steps = (int64_t)o[A + 2];
    stats->n_beliefs = (int64_t)nb;
    stats->n_actions = (int64_t)na;
    stats->near_ties = (int64_t)o[A + 6];
    stats->sweep_visits = (int64_t)o[A + 7];
    stats->sweep_internal = (int64_t)o[A + 8];
    stats->sweep_nodes = (int64_t)o[A + 9];
    stats->insert_reprobes = (int64_t)o[A + 10];
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ws->ev0, ws->ev1);
    stats->device_ms = ms;
  }
  return VOPP_OK;
}

}  // namespace vopp

extern "C" vopp_status vopp_plan(const vopp_pomdp* p, const void* belief, int32_t n_belief,
                                 int32_t budget, int32_t depth, const vopp_params* prm,
                                 vopp_workspace* ws, void* stream, int32_t* action,
                                 double* values, double* v_root, vopp_stats* stats) {
  clear_error();
  return plan_common(p, belief, n_belief, budget, depth, prm, ws, stream, 0.0, action, values,
                     v_root, stats, nullptr);
}

extern "C" vopp_status vopp_plan_trace(const vopp_pomdp* p, const void* belief,
                                       int32_t n_belief, int32_t budget, int32_t depth,
                                       const vopp_params* prm, vopp_workspace* ws, void* stream,
                                       int32_t* action, double* values, double* v_root,
                                       vopp_stats* stats, int16_t* draw_act, int32_t* draw_obs,
                                       const int16_t* force_act, int64_t trace_len) {
  clear_error();
  if (!draw_act || !draw_obs) return fail(VOPP_E_INVALID, "null draw trace");
  return plan_common(p, belief, n_belief, budget, depth, prm, ws, stream, 0.0, action, values,
                     v_root, stats, nullptr, draw_act, draw_obs, force_act, trace_len);
}

// ---------------------------------------------------------------------------
// The allocation-free plan: the tree lives in a file-scope device array of
// VOPP_NOALLOC_SCRATCH_BYTES per GPU instead of a workspace.  In host code the
// array's name only stands for the symbol; its device address on each GPU
// comes from hipGetSymbolAddress, taken once per device on the first call and
// kept in scratch_ptr.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[VOPP_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {nullptr};

vopp_status scratch_of(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(VOPP_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    scratch_ptr[dev] = ptr;
  }
  *out = scratch_ptr[dev];
  return VOPP_OK;
}
}  // namespace

extern "C" vopp_status vopp_plan_noalloc(const vopp_pomdp* p, const void* belief,
                                         int32_t n_belief, int32_t budget, int32_t depth,
                                         const vopp_params* prm, void* stream, double* result) {
  clear_error();
  vopp_status st = check_params(p, prm, budget, depth);
  if (st != VOPP_OK) return st;
  if (!belief || n_belief < 1) return fail(VOPP_E_INVALID, "empty belief");
  if (!result) return fail(VOPP_E_INVALID, "null result pointer");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device)
    return fail(VOPP_E_INVALID, "model lives on device %d, current is %d", p->device, dev);
  const WsSizes z = sizes_for(p, prm->n_particles, budget, depth, prm->schedule);
  const size_t need = bytes_for(z);
  if (need > (size_t)VOPP_NOALLOC_SCRATCH_BYTES)
    return fail(VOPP_E_INVALID,
                "the plan needs %zu bytes of tree memory; the allocation-free entry point "
                "holds %zu (use vopp_plan with a workspace)",
                need, (size_t)VOPP_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  st = scratch_of(dev, &base);
  if (st != VOPP_OK) return st;
  // A workspace record over the scratch: no pinned buffers, events or
  // profiling; nothing in it allocates.
  vopp_workspace w;
  w.z = z;
  w.device = dev;
  w.arena = base;
  w.bytes = need;
  double* unused_out = nullptr;
  carve_tree(base, z, w.tree, &w.carry_rng_dev, &w.step_base_dev, &unused_out);
  w.out_dev = result;
  PlanView P = make_view(p, &w, belief, n_belief, budget, depth, prm);
  P.clear_all = 1;
  int steps = 0;
  return enqueue_plan(p, &w, P, (hipStream_t)stream, &steps);
}

extern "C" vopp_status vopp_plan_anytime(const vopp_pomdp* p, const void* belief,
                                         int32_t n_belief, int32_t max_budget, int32_t depth,
                                         double time_ms, const vopp_params* prm,
                                         vopp_workspace* ws, void* stream, int32_t* action,
                                         double* values, double* v_root, vopp_stats* stats,
                                         int32_t* iterations) {
  clear_error();
  if (!(time_ms > 0.0) || !std::isfinite(time_ms))
    return fail(VOPP_E_INVALID, "time budget must be a positive number of milliseconds");
  return plan_common(p, belief, n_belief, max_budget, depth, prm, ws, stream, time_ms, action,
                     values, v_root, stats, iterations);
}

extern "C" vopp_status vopp_tree_dump(vopp_workspace* w, int32_t* b_parent, int32_t* b_obs,
                                      int32_t* b_depth, float* psi, float* b_V, int32_t* b_N,
                                      int32_t* a_parent, int32_t* a_act, double* a_C,
                                      int32_t* a_N) {
  clear_error();
  if (!w) return fail(VOPP_E_INVALID, "null workspace");
  if (w->n_prev_beliefs <= 0) return fail(VOPP_E_INVALID, "no plan has run in this workspace");
  const int A = w->last_A, ra = w->tree.ra, rs = dump_bytes(w->tree.ra);
  const int steps = w->last_steps, n_p = w->last_n_p;
  hipError_t e = hipDeviceSynchronize();
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  };
  // Beliefs with their depth: the root, then each level step's list (level d
  // creates depth d + 1).
  std::vector<int> list((size_t)steps * n_p);
  cp(list.data(), w->tree.list, list.size() * 4);
  std::vector<int> ids{0}, depth{0};
  if ((int)w->step_depth.size() != steps)
    return fail(VOPP_E_INTERNAL, "tree dump: %zu level-step depths for %d steps",
                w->step_depth.size(), steps);
  for (int t = 0; t < steps; ++t) {
    for (int j = 0; j < n_p; ++j)
      if (list[(size_t)t * n_p + j]) ids.push_back(1 + t * n_p + j);
    depth.resize(ids.size(), w->step_depth[t]);
  }
  if (e != hipSuccess) return hip_fail(e, "tree dump");
  const size_t nb = ids.size();
  if ((long long)nb != w->n_prev_beliefs)
    return fail(VOPP_E_INTERNAL, "tree dump: %zu listed beliefs, %d counted", nb,
                w->n_prev_beliefs);
  // Gather the records on the device, then copy them.
  std::vector<unsigned char> rec(nb * (size_t)rs);
  int* ids_dev = nullptr;
  unsigned char* rec_dev = nullptr;
  e = hipMalloc(&ids_dev, nb * 4);
  if (e == hipSuccess) e = hipMalloc(&rec_dev, nb * (size_t)rs);
  if (e == hipSuccess) e = hipMemcpy(ids_dev, ids.data(), nb * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_gather(w->tree, ids_dev, (int)nb, rec_dev, nullptr);
  cp(rec.data(), rec_dev, nb * (size_t)rs);
  if (ids_dev) (void)hipFree(ids_dev);
  if (rec_dev) (void)hipFree(rec_dev);
  if (e != hipSuccess) return hip_fail(e, "tree dump");
  // The packed copy of each belief (layout in vopp_device.hpp).
  struct Tail { float V; int Nb; int obs; int pad; unsigned long long parent; };
  auto meta = [&](size_t i) {
    return reinterpret_cast<const Tail*>(rec.data() + i * rs + dump_tail_off(ra));
  };
  auto nrow = [&](size_t i) {
    return reinterpret_cast<const int*>(rec.data() + i * rs + dump_n_off(ra));
  };
  auto crow = [&](size_t i) {
    return reinterpret_cast<const long long*>(rec.data() + i * rs + dump_c_off(ra));
  };
  auto prow = [&](size_t i) { return reinterpret_cast<const float*>(rec.data() + i * rs); };
  // Long rows: a belief other than the root holds (b, a) only where bit a
  // of its bitmap is set.
  auto valid = [&](size_t i, int a) {
    if (ra <= kMaxA || ids[i] == 0) return true;
    const uint32_t* bits =
        reinterpret_cast<const uint32_t*>(rec.data() + i * rs + dump_bits_off(ra));
    return ((bits[a >> 5] >> (a & 31)) & 1u) != 0;
  };
  // Canonical order: by depth, then (parent's position, action, observation);
  // action nodes by (parent's position, action).  It depends only on the
  // tree, not on the order in which episodes inserted it.
  int max_id = 0;
  for (int id : ids) max_id = std::max(max_id, id);
  std::vector<int> pos_of(max_id + 1, -1);
  std::vector<size_t> order(nb);
  for (size_t i = 0; i < nb; ++i) order[i] = i;
  pos_of[0] = 0;
  size_t lo = 1;
  for (int d = 1; lo < nb; ++d) {
    // Lists are per level step, so one depth is spread over several of them.
    std::vector<size_t> grp;
    for (size_t i = 0; i < nb; ++i)
      if (depth[i] == d) grp.push_back(i);
    auto key = [&](size_t i) {
      const unsigned long long par = meta(i)->parent;
      return std::make_tuple(pos_of[(int)(par >> kActBits)], (int)(par & kActMask), meta(i)->obs);
    };
    std::sort(grp.begin(), grp.end(), [&](size_t x, size_t y) { return key(x) < key(y); });
    for (size_t j = 0; j < grp.size(); ++j) {
      order[lo + j] = grp[j];
      pos_of[ids[grp[j]]] = (int)(lo + j);
    }
    lo += grp.size();
    if (grp.empty()) return fail(VOPP_E_INTERNAL, "tree dump: depth %d is empty", d);
  }
  std::vector<int> act_of(nb * (size_t)A, -1);
  size_t na = 0;
  for (size_t q = 0; q < nb; ++q) {
    const size_t i = order[q];
    for (int a = 0; a < A; ++a) {
      if (!valid(i, a)) continue;
      const int n = nrow(i)[a];
      if (n <= 0) continue;
      act_of[q * A + a] = (int)na;
      if (a_parent) a_parent[na] = (int32_t)q;
      if (a_act) a_act[na] = a;
      if (a_N) a_N[na] = n;
      if (a_C) a_C[na] = (double)crow(i)[a] * w->last_fix_inv64;
      ++na;
    }
  }
  if ((long long)na != w->n_prev_actions)
    return fail(VOPP_E_INTERNAL, "tree dump: %zu action nodes, %d counted", na,
                w->n_prev_actions);
  for (size_t q = 0; q < nb; ++q) {
    const size_t i = order[q];
    const Tail* m = meta(i);
    int par = -1;
    if (q > 0) {
      const int pq = pos_of[(int)(m->parent >> kActBits)];
      par = act_of[(size_t)pq * A + (int)(m->parent & kActMask)];
    }
    if (b_parent) b_parent[q] = par;
    if (b_obs) b_obs[q] = q > 0 ? m->obs : -1;
    if (b_depth) b_depth[q] = depth[i];
    if (b_V) b_V[q] = m->V;
    if (b_N) b_N[q] = m->Nb;
    if (psi)
      for (int j = 0; j < A; ++j) psi[q * A + j] = prow(i)[j];
  }
  return VOPP_OK;
}

extern "C" vopp_status vopp_level_counts(const vopp_workspace* w, int32_t* counts, int32_t cap,
                                         int32_t* n_steps) {
  clear_error();
  if (!w || !n_steps) return fail(VOPP_E_INVALID, "null argument");
  if (w->n_prev_beliefs <= 0) return fail(VOPP_E_INVALID, "no plan has run in this workspace");
  *n_steps = w->last_steps;
  const int n = std::min(cap, w->last_steps);
  if (counts && n > 0) {
    const size_t n_p = (size_t)w->last_n_p;
    std::vector<int> list((size_t)n * n_p);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
      e = hipMemcpy(list.data(), w->tree.list, list.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "level counts");
    for (int t = 0; t < n; ++t) {
      int c = 0;
      for (size_t j = 0; j < n_p; ++j) c += list[t * n_p + j] != 0;
      counts[t] = c;
    }
  }
  return VOPP_OK;
}

extern "C" vopp_status vopp_profile_enable(vopp_workspace* w, int32_t kind_mask) {
  clear_error();
  if (!w) return fail(VOPP_E_INVALID, "null workspace");
  w->prof_on = kind_mask != 0;
  w->prof_mask = (uint32_t)kind_mask;
  w->prof_used = 0;
  return VOPP_OK;
}

extern "C" vopp_status vopp_profile_reset(vopp_workspace* w) {
  clear_error();
  if (!w) return fail(VOPP_E_INVALID, "null workspace");
  for (int i = 0; i < VOPP_KERNEL_KINDS; ++i) { w->prof_ms[i] = 0.0; w->prof_count[i] = 0; }
  return VOPP_OK;
}

extern "C" vopp_status vopp_profile_read(const vopp_workspace* w, double* ms, int64_t* launches) {
  clear_error();
  if (!w || !ms) return fail(VOPP_E_INVALID, "null argument");
  for (int i = 0; i < VOPP_KERNEL_KINDS; ++i) {
    ms[i] = w->prof_ms[i];
    if (launches) launches[i] = w->prof_count[i];
  }
  return VOPP_OK;
}

// ---------------------------------------------------------------------------
// True environment and belief update (single episode).
// ---------------------------------------------------------------------------
namespace {

// Scratch layout: out record | env words | weights | propagated particles.
vopp_status filter_scratch(vopp_pomdp* p, int n, double** out, int** env,
                           unsigned long long** w, void** prop) {
  const size_t need = 4096 + (size_t)n * 8 + (size_t)n * 8 + 512;
  if (p->filt_bytes < need) {
    if (p->filt) (void)hipFree(p->filt);
    p->filt = nullptr;
    p->filt_bytes = 0;
    hipError_t e = hipMalloc(&p->filt, need);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(filter scratch)");
    p->filt_bytes = need;
  }
  char* base = (char*)p->filt;
  *out = (double*)base;
  *env = (int*)(base + 2048);
  *w = (unsigned long long*)(base + 4096);
  *prop = (void*)(base + 4096 + (size_t)n * 8);
  return VOPP_OK;
}

PlanView filter_view(const vopp_pomdp* p, double* out, int* env, unsigned long long* w,
                     void* prop, void* part, int n, uint64_t seed) {
  PlanView P;
  std::memset(&P, 0, sizeof(P));
  P.m = p->view;
  P.out = out;
  P.seed_lo = (uint32_t)seed;
  P.seed_hi = (uint32_t)(seed >> 32);
  P.f.part = part;
  P.f.prop = prop;
  P.f.w = w;
  P.f.M = n;
  P.f.env = env;
  P.f.env_seed_lo = (uint32_t)seed;
  P.f.env_seed_hi = (uint32_t)(seed >> 32);
  return P;
}

}  // namespace

extern "C" vopp_status vopp_env_step(const vopp_pomdp* p, void* state, int32_t action,
                                     uint64_t env_seed, uint32_t step, void* stream,
                                     int32_t* obs, float* reward, int32_t* terminal) {
  clear_error();
  if (!p || !state) return fail(VOPP_E_INVALID, "null argument");
  if (action < 0 || action >= p->nA) return fail(VOPP_E_INVALID, "action out of range");
  vopp_pomdp* mp = const_cast<vopp_pomdp*>(p);
  double* out;
  int* env;
  unsigned long long* w;
  void* prop;
  vopp_status st = filter_scratch(mp, 1, &out, &env, &w, &prop);
  if (st != VOPP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int words = p->kind == kTabular ? 1 : 2;
  int host_env[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double act = (double)action;
  hipError_t e = hipMemcpyAsync(env, state, words * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, &act, sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "env step set-up");
  if (p->kind == kTabular) {
    int sv = 0;
    e = hipMemcpy(&sv, env, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && (sv < 0 || sv >= p->view.nS))
      return fail(VOPP_E_INVALID, "state outside [0, nS)");
  }
  PlanView P = filter_view(p, out, env, w, prop, state, 1, env_seed);
  e = launch_env(P, (int)step, s);
  if (e == hipSuccess) e = hipMemcpyAsync(state, env, words * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(host_env, env, sizeof(host_env), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "env step");
  if (obs) *obs = host_env[2];
  if (reward) std::memcpy(reward, &host_env[4], 4);
  if (terminal) *terminal = host_env[5];
  return VOPP_OK;
}

extern "C" vopp_status vopp_belief_update(const vopp_pomdp* p, void* particles, int32_t n,
                                          int32_t action, int32_t obs, uint64_t seed,
                                          uint32_t step, void* stream,
                                          uint64_t* total_weight) {
  clear_error();
  if (!p || !particles) return fail(VOPP_E_INVALID, "null argument");
  if (n < 1 || n > (1 << 24)) return fail(VOPP_E_INVALID, "n must be in [1, 2^24]");
  if (action < 0 || action >= p->nA) return fail(VOPP_E_INVALID, "action out of range");
  if (obs < 0 || obs >= p->view.nO) return fail(VOPP_E_INVALID, "observation out of range");
  vopp_pomdp* mp = const_cast<vopp_pomdp*>(p);
  double* out;
  int* env;
  unsigned long long* w;
  void* prop;
  vopp_status st = filter_scratch(mp, n, &out, &env, &w, &prop);
  if (st != VOPP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  int host_env[8] = {0, 0, obs, action, 0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(env, host_env, sizeof(host_env), hipMemcpyHostToDevice, s);
  PlanView P = filter_view(p, out, env, w, prop, particles, n, seed);
  if (e == hipSuccess) e = launch_pf(P, (int)step, s);
  unsigned long long tot = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&tot, w + (n - 1), 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "belief update");
  if (total_weight) *total_weight = tot;
  return VOPP_OK;
}

// C ABI of the solver (declared in include/cdcs.h): setup packs one or more
// instances into concatenated device arrays, the iteration is a fixed
// sequence of kernel launches on the handle's stream, and results are read
// back in the canonical coordinates the header documents.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "device.h"
#include "plan.h"

using namespace cdcs;

// largest clique order the adjoint differentiates (Jacobi eigen-cache and
// Daleckii-Krein product in LDS)
constexpr int kAdjMax = 96;


namespace cdcs {
enum As { AS_QT = 0, AS_GT, AS_DEN2, AS_DIFF2, AS_NORM2, AS_BY, AS_EA, kNas = 8 };
struct AdjPlan {
  DevPlan d;
  double* as;
  double* mu_x;
  double* mu_s;
  double* mu_y;
  double* mu_v;
  double* mu_t;
  double* qx;
  const double* gx;
  const double* phi;
  const double* ev;
  const double* aphi;
  const double* eig;
  const int64_t* eig_off;
  double* dc;
  double* db;
};
void launch_adj_eig(const AdjPlan& ap, const int32_t* tasks, int32_t ntask, int kmax, hipStream_t st);
void launch_adj_iteration(const AdjPlan& ap, const int32_t* const* tasks, const int32_t* ntasks,
                          int final_pass, int use_g, hipStream_t st);
void launch_seg_dots(const double* w, const double* Vb, int64_t NF, int nk, const int64_t* seg, double* out,
                     int B, hipStream_t st);
void launch_flat_axpy_multi(double* w, const double* Vb, int64_t NF, int nk, const double* coef,
                            const int32_t* inst_of, int B, double sign, hipStream_t st);
void launch_flat_scale(double* out, const double* w, const double* sc, const int32_t* inst_of, int64_t NF,
                       hipStream_t st);
void launch_flat_sub(double* out, const double* a, const double* b, int64_t NF, hipStream_t st);
void launch_flat_sqrt(double* out, const double* a, int64_t n, hipStream_t st);
}  // namespace cdcs

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(CDCS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

enum Phase {
  PH_R0 = 0, PH_SPMV_A, PH_TRSV, PH_SPMV_AT, PH_SCALAR1, PH_UPDATE_E, PH_UPDATE_R,
  PH_CONE16, PH_CONE32, PH_CONE64, PH_CONE96, PH_LG_GATHER, PH_LG_TRD_SYMV, PH_LG_TRD_UPDATE, PH_LG_TRD_TRAIL,
  PH_LG_TRD_TAIL, PH_LG_EIG_PREP, PH_LG_EIG_BISECT, PH_LG_EIG_SINGLE, PH_LG_EIG_CLUSTER, PH_LG_BT_TFACTOR,
  PH_LG_BT_APPLY, PH_LG_RECON, PH_LG_PARTIALS, PH_SCALAR2, PH_SPLIT_R, PH_SPLIT_G, PH_SPLIT_X, PH_SPLIT_W,
  PH_SPLIT_UPDATE, PH_SPLIT_SCALAR, PH_LG_BAND_PANEL, PH_LG_BAND_TRAIL, PH_LG_BAND_CHASE, PH_LG_BAND_Q2, kNumPhases
};
const char* kPhaseNames[kNumPhases] = {
    "r0_scatter", "spmv_A", "trsv", "spmv_At", "scalar1", "update_x", "update_y",
    "cone_jacobi16", "cone_jacobi32", "cone_jacobi64", "cone_jacobi96", "large_gather", "trd_symv",
    "trd_update", "trd_trail", "trd_tail", "eig_prep", "eig_bisect", "eig_single", "eig_cluster", "bt_tfactor",
    "bt_apply", "large_recon", "large_partials", "scalar2", "split_scatter", "split_rhs", "split_x",
    "split_gather", "split_update", "split_scalar", "band_panel", "band_trail", "band_chase", "band_q2"};
// phase of each large-clique step (the tridiagonalisation is timed per launch kind)
const int kLargeStepPhase[kLargeSteps] = {PH_LG_GATHER, -1, -1, -1, PH_LG_RECON, PH_LG_PARTIALS};

}  // namespace

struct cdcs_handle {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream (default priority) for the large-clique eigensolver, which
  // runs beside the small-clique Jacobi kernels: both write disjoint cliques
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // one stream per Jacobi bucket after the first non-empty one, so that the
  // buckets run side by side (forked from and joined back into `stream`)
  hipStream_t jst[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_jjoin[3] = {nullptr, nullptr, nullptr};
  cdcs_settings set{};
  int32_t B = 0;
  std::vector<Instance> inst;
  std::vector<int64_t> ent_off, slot_off;
  std::vector<int32_t> row_off, clq_off;
  std::vector<void*> allocs;
  DevPlan d{};
  // cone work lists by kernel variant
  int32_t* tasks[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t ntasks[5] = {0, 0, 0, 0, 0};
  // the adjoint's Jacobi lists (every clique of up to kAdjMax vertices by
  // size: <= 16, 32, 64, 96; independent of settings.jacobi_max) and the
  // largest clique order
  int32_t* adj_tasks[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t adj_ntasks[4] = {0, 0, 0, 0};
  int32_t max_clique = 0;
  // Jacobi buckets: clique orders (host), tile variant, whether autotuned
  std::vector<int32_t> bucket_sizes[4];
  int32_t jvar[4] = {0, 0, 0, 0};
  int32_t jtuned[4] = {0, 0, 0, 0};
  int32_t kmax_large = 0;
  std::vector<int32_t> large_sizes;      // host copy of large task sizes (launch shapes)
  // timing
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<std::pair<int, size_t>> ev_used;   // (phase, pool index) since last harvest
  size_t ev_open = 0;                             // timers begun and not yet ended
  double phase_ms[kNumPhases] = {};
  int64_t phase_n[kNumPhases] = {};
  // graphs
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // adjoint buffers (allocated on the first cdcs_adjoint call)
  bool adj_ready = false;
  AdjPlan adj{};
  // batched GMRES workspace over flat vectors [x | s | y | v | tau]
  int64_t nf = 0;
  double* gm_V = nullptr;      // (kRestart + 1) * nf basis
  double* gm_w = nullptr;      // nf
  double* gm_mu = nullptr;     // nf
  double* gm_g = nullptr;      // nf
  double* gm_coef = nullptr;   // (kRestart + 1) * B
  double* gm_dots = nullptr;   // (kRestart + 1) * B
  double* gm_scale = nullptr;  // B
  int64_t* gm_seg = nullptr;   // 10 * B
  int32_t* gm_inst = nullptr;  // nf
  double* gm_dots2 = nullptr;  // (kRestart + 1) * B, the second Gram-Schmidt pass
  double* gm_nrm = nullptr;    // B
  double* gm_resid = nullptr;  // B
  int32_t* gm_reason = nullptr;  // B
  int32_t* gm_flags = nullptr; // 3 B + 1: jlim, done, nhist, alldone
  GmState gm_state{};          // Hessenberg, rotations, gamma, residual history (device)
  double setup_s = 0.0;
  // primal-only / dual-only ADMM (settings.method 1 or 2)
  SplitArgs sa{};
  // outcome of the last cdcs_adjoint per instance: final relative residual
  // ||g - (I - T'^T) mu|| / ||g|| and why GMRES stopped (0 tolerance met,
  // 1 stalled, 2 iteration limit)
  std::vector<double> adj_resid;
  std::vector<int32_t> adj_reason;
};

namespace {

template <typename T>
int dev_alloc(cdcs_handle* h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return set_error(CDCS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = (T*)q;
  return 0;
}

template <typename T>
int dev_upload(cdcs_handle* h, T** p, const std::vector<T>& v) {
  int rc = dev_alloc(h, p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

template <typename T>
int dev_zeros(cdcs_handle* h, T** p, size_t count) {
  int rc = dev_alloc(h, p, count);
  if (rc) return rc;
  HIPCHK(hipMemset(*p, 0, std::max<size_t>(count, 1) * sizeof(T)));
  return 0;
}

// Jacobi bucket of a clique of order K (0: <= 16, 1: <= 32, 2: <= 64), or 4
// (the tridiagonal path) above jmax, the largest order the Jacobi kernels
// take (settings.jacobi_max)
int bucket_of(int K, int jmax = kJacobiMax) {
  if (K > jmax) return 4;
  if (K <= 16) return 0;
  if (K <= 32) return 1;
  if (K <= 64) return 2;
  return 3;
}

// smallest clique order that takes the two-stage tridiagonalisation.  0 =
// automatic: 137 when the handle's largest clique has at least kBandAuto
// vertices (its two-stage chain then sets the pace, and the other cliques of
// 137 vertices or more ride in the same launches), otherwise none.  A lone
// clique of a few hundred vertices is reduced faster by the one-stage path
// (11 column steps and the LDS tail for the 147-vertex clique of the 40 x 50
// grid max-cut: 714 against 497 iterations/s); the estimates from the
// per-launch times cross near 300 vertices.
constexpr int kBandAuto = 320;
int band_min_of(const cdcs_handle* h) {
  if (h->set.band_min) return h->set.band_min;
  return (h->kmax_large >= kBandAuto) ? kBandMinDefault : 1025;
}

// largest clique order of the Jacobi kernels: 0 = 32, or 64 when the FP32 or
// warm-started Jacobi variants are on (they act on Jacobi cliques only);
// measured on max-cut G(2000, 6000): 82.9 against 81.0 iterations/s, on the
// uneven-clique workload 1412 against 581, on the 40 x 50 grid 774 against 593
int jacobi_max_of(const cdcs_settings& s) {
  if (s.jacobi_max) return s.jacobi_max;
  return (s.eig_fp32 || s.eig_warm) ? 64 : 32;
}

// record a phase launch between two events when timing is on
// event pair from the pool (not yet recorded)
size_t timer_alloc(cdcs_handle* h) {
  const size_t slot = h->ev_used.size() + h->ev_open;
  while (slot >= h->ev_pool.size()) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    h->ev_pool.push_back({a, b});
  }
  ++h->ev_open;
  return slot;
}

// the pair holds a measurement of phase ph once the stream reaches it
void timer_commit(cdcs_handle* h, size_t slot, int ph) {
  --h->ev_open;
  h->ev_used.push_back({ph, slot});
}

// event pair from the pool, start recorded on s
size_t timer_begin(cdcs_handle* h, hipStream_t s) {
  const size_t slot = timer_alloc(h);
  (void)hipEventRecord(h->ev_pool[slot].first, s);
  return slot;
}

void timer_end(cdcs_handle* h, size_t slot, int ph, hipStream_t s) {
  (void)hipEventRecord(h->ev_pool[slot].second, s);
  timer_commit(h, slot, ph);
}

struct PhaseTimer {
  cdcs_handle* h;
  int ph;
  size_t slot = 0;
  bool on;
  hipStream_t sm;
  PhaseTimer(cdcs_handle* hh, int p, hipStream_t s = nullptr)
      : h(hh), ph(p), on(hh->set.timing != 0 && p >= 0), sm(s ? s : hh->stream) {
    if (on) slot = timer_begin(h, sm);
  }
  ~PhaseTimer() {
    if (on) timer_end(h, slot, ph, sm);
  }
};

// times every launch of the tridiagonalisation step in its own phase with
// the kernel's own start and end (events passed to the launch)
struct TrdTimer {
  cdcs_handle* h;
  size_t slot;
  static void begin(void* c, int, hipEvent_t* e0, hipEvent_t* e1) {
    auto* t = static_cast<TrdTimer*>(c);
    t->slot = timer_alloc(t->h);
    *e0 = t->h->ev_pool[t->slot].first;
    *e1 = t->h->ev_pool[t->slot].second;
  }
  static void end(void* c, int kind) {
    auto* t = static_cast<TrdTimer*>(c);
    timer_commit(t->h, t->slot, kind < 10 ? PH_LG_TRD_SYMV + kind : PH_LG_BAND_PANEL + kind - 10);
  }
};

void harvest_timers(cdcs_handle* h) {
  for (auto& u : h->ev_used) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev_pool[u.second].first, h->ev_pool[u.second].second) == hipSuccess) {
      h->phase_ms[u.first] += ms;
      h->phase_n[u.first] += 1;
    }
  }
  h->ev_used.clear();
}

// one iteration of the primal-only (method 1) or dual-only (method 2) ADMM:
// scatter, right-hand side, the m x m solve (the same triangular-solve
// kernel, its solution written to y), x, projection argument, the clique
// projections (the conic-step kernels' stand-alone entry; buckets in
// sequence, the large cliques' chain beside them on the second stream),
// multiplier update, residuals
int launch_split_iteration(cdcs_handle* h, int32_t stop) {
  const DevPlan& d = h->d;
  const SplitArgs& a = h->sa;
  const int primal = h->set.method == 1;
  hipStream_t st = h->stream;
  DevPlan dy = d;
  dy.w = d.y;
  { PhaseTimer t(h, PH_SPLIT_R); launch_split_r(d, a, primal, st); }
  { PhaseTimer t(h, PH_SPLIT_G); launch_split_g(d, a, primal, st); }
  { PhaseTimer t(h, PH_TRSV); launch_trsv(dy, st); }
  { PhaseTimer t(h, PH_SPLIT_X); launch_split_x(d, a, primal, st); }
  { PhaseTimer t(h, PH_SPLIT_W); launch_split_w(d, a, primal, st); }
  const bool fork = h->ntasks[4] != 0;
  hipStream_t lst = st;
  if (fork) {
    HIPCHK(hipEventRecord(h->ev_fork, st));
    lst = h->aux;
    HIPCHK(hipStreamWaitEvent(lst, h->ev_fork, 0));
    PhaseTimer t(h, PH_LG_GATHER, lst);
    launch_psd_project_large(d.clq_size, d.clq_slot, h->tasks[4], d.big_size, h->large_sizes.data(), h->ntasks[4],
                             h->kmax_large, a.w, a.p, d.big_work, d.big_off, lst, band_min_of(h));
  }
  const int kmaxs[4] = {16, 32, 64, 96};
  for (int bk = 0; bk < 4; ++bk)
    if (h->ntasks[bk]) {
      PhaseTimer t(h, PH_CONE16 + bk);
      launch_psd_project(d.clq_size, d.clq_slot, h->tasks[bk], h->ntasks[bk], kmaxs[bk], a.w, a.p, st, h->jvar[bk],
                         h->set.eig_fp32);
    }
  if (fork) {
    HIPCHK(hipEventRecord(h->ev_join, lst));
    HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
  }
  { PhaseTimer t(h, PH_SPLIT_UPDATE); launch_split_update(d, a, primal, st); }
  { PhaseTimer t(h, PH_SPLIT_SCALAR); launch_split_scalar(d, a, h->set.eps_tol, h->set.max_iter, stop, st); }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return 0;
}

int launch_iteration(cdcs_handle* h, int32_t stop) {
  if (h->set.method != 0) return launch_split_iteration(h, stop);
  const DevPlan& d = h->d;
  hipStream_t st = h->stream;
  { PhaseTimer t(h, PH_R0); launch_r0(d, st); }
  { PhaseTimer t(h, PH_SPMV_A); launch_spmv_a(d, st); }
  { PhaseTimer t(h, PH_TRSV); launch_trsv(d, st); }
  { PhaseTimer t(h, PH_SPMV_AT); launch_spmv_at(d, st); }
  { PhaseTimer t(h, PH_SCALAR1); launch_scalar1(d, st); }
  { PhaseTimer t(h, PH_UPDATE_E); launch_update_e(d, st); }
  { PhaseTimer t(h, PH_UPDATE_R); launch_update_r(d, st); }
  const int kmaxs[4] = {16, 32, 64, 96};   // bucket orders (the last is empty while kJacobiMax = 64)
  int nsmall = 0;
  for (int bk = 0; bk < 4; ++bk) nsmall += h->ntasks[bk] ? 1 : 0;
  const bool fork = h->ntasks[4] && nsmall;
  // A large clique's chain of per-column launches (the columns above the 136
  // the LDS tail holds) is the critical path once it is long: beside it the
  // Jacobi buckets stay in sequence on `stream`, leaving compute units free
  // for the chain (random max-cut G(2000, 6000): 544 columns, ~10 ms per
  // iteration).  A chain of at most kLongChain columns takes about as long
  // as one Jacobi bucket or less (max-cut on the 40 x 50 periodic grid: 32
  // columns, ~0.35 ms, beside a 1.6 ms bucket of cliques up to 64), so the
  // buckets then run side by side.  The same fork and joins serve both.
  constexpr int32_t kLongChain = 128;
  const bool chain = h->ntasks[4] && h->kmax_large - 136 > kLongChain;
  if (fork || (nsmall > 1 && !chain)) HIPCHK(hipEventRecord(h->ev_fork, st));
  hipStream_t lst = st;
  if (fork) {
    lst = h->aux;
    HIPCHK(hipStreamWaitEvent(lst, h->ev_fork, 0));
  }
  if (h->ntasks[4]) {
    TrdTimer tt{h, 0};
    const LaunchHook hook{&TrdTimer::begin, &TrdTimer::end, &tt};
    for (int step = 0; step < kLargeSteps; ++step) {
      PhaseTimer t(h, kLargeStepPhase[step], lst);
      launch_cone_large_step(d, h->tasks[4], h->ntasks[4], h->kmax_large, h->large_sizes.data(), step, lst,
                             band_min_of(h),
                             h->set.timing ? &hook : nullptr);
    }
  }
  // Jacobi buckets: the first non-empty one on `stream` and the others each
  // on a stream of its own, unless a long per-column chain runs beside them
  const int nside = chain ? 0 : nsmall - 1;
  int side = 0;
  for (int bk = 0; bk < 4; ++bk)
    if (h->ntasks[bk]) {
      hipStream_t bs = st;
      if (bk > 0 && side < nside) {
        bs = h->jst[side];
        HIPCHK(hipStreamWaitEvent(bs, h->ev_fork, 0));
      }
      {
        PhaseTimer t(h, PH_CONE16 + bk, bs);
        launch_cone_jacobi(d, h->tasks[bk], h->ntasks[bk], kmaxs[bk], h->jvar[bk], h->set.eig_fp32, bs);
      }
      if (bs != st) {
        HIPCHK(hipEventRecord(h->ev_jjoin[side], bs));
        HIPCHK(hipStreamWaitEvent(st, h->ev_jjoin[side], 0));
        ++side;
      }
    }
  if (fork) {
    HIPCHK(hipEventRecord(h->ev_join, lst));
    HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
  }
  { PhaseTimer t(h, PH_SCALAR2); launch_scalar2(d, h->set.eps_tol, h->set.max_iter, stop, st); }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return 0;
}

// Autotuner: for every Jacobi bucket, time its two tile shapes (threads per
// clique) on synthetic symmetric blocks with the bucket's clique orders (at
// most kTuneBlocks of them, entries from a fixed integer hash in [-1, 1)) and
// keep the faster.  The stand-alone projection kernel is the proxy: it runs
// the same Jacobi as the fused cone kernel.
constexpr int kTuneBlocks = 1024;
constexpr int kTuneReps = 3;

int autotune(cdcs_handle* h) {
  hipStream_t st = h->stream;
  const int kmaxs[4] = {16, 32, 64, 96};   // bucket orders (the last is empty while kJacobiMax = 64)
  for (int bk = 0; bk < 4; ++bk) {
    const auto& all = h->bucket_sizes[bk];
    if (all.empty()) continue;
    const int nb = (int)std::min<size_t>(all.size(), kTuneBlocks);
    std::vector<int32_t> sz(all.begin(), all.begin() + nb), tk(nb);
    std::vector<int64_t> off(nb);
    int64_t tot = 0;
    for (int i = 0; i < nb; ++i) {
      tk[i] = i;
      off[i] = tot;
      tot += (int64_t)sz[i] * (sz[i] + 1) / 2;
    }
    std::vector<double> vals((size_t)tot);
    uint64_t x = 0x9E3779B97F4A7C15ull ^ (uint64_t)(bk + 1);
    for (auto& v : vals) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      v = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    int32_t *dsz = nullptr, *dtk = nullptr;
    int64_t* doff = nullptr;
    double *din = nullptr, *dout = nullptr;
    auto release = [&]() {
      (void)hipFree(dsz);
      (void)hipFree(dtk);
      (void)hipFree(doff);
      (void)hipFree(din);
      (void)hipFree(dout);
    };
    if (hipMalloc(&dsz, nb * 4) != hipSuccess || hipMalloc(&dtk, nb * 4) != hipSuccess ||
        hipMalloc(&doff, nb * 8) != hipSuccess || hipMalloc(&din, tot * 8) != hipSuccess ||
        hipMalloc(&dout, tot * 8) != hipSuccess) {
      release();
      return set_error(CDCS_E_NOMEM, "autotune: hipMalloc failed");
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      release();
      return set_error(CDCS_E_DEVICE, "autotune: hipEventCreate failed");
    }
    float best = 0.f;
    int bestv = 0;
    hipError_t e = hipMemcpyAsync(dsz, sz.data(), nb * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dtk, tk.data(), nb * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(doff, off.data(), nb * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(din, vals.data(), tot * 8, hipMemcpyHostToDevice, st);
    for (int v = 0; v < 2 && e == hipSuccess; ++v) {
      launch_psd_project(dsz, doff, dtk, nb, kmaxs[bk], din, dout, st, v, h->set.eig_fp32);   // warm-up
      (void)hipEventRecord(e0, st);
      for (int rep = 0; rep < kTuneReps; ++rep)
        launch_psd_project(dsz, doff, dtk, nb, kmaxs[bk], din, dout, st, v, h->set.eig_fp32);
      (void)hipEventRecord(e1, st);
      e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && (v == 0 || ms < best)) {
        best = ms;
        bestv = v;
      }
    }
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
    h->jvar[bk] = bestv;
    h->jtuned[bk] = 1;
  }
  return 0;
}

int capture_graph(cdcs_handle* h, int stop) {
  if (h->graph[stop]) return 0;
  hipGraph_t g;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  const int saved = h->set.timing;
  h->set.timing = 0;
  int rc = launch_iteration(h, stop);
  h->set.timing = saved;
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (rc) return rc;
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&h->graph[stop], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return 0;
}

int run_iterations(cdcs_handle* h, int32_t k, int32_t stop) {
  if (h->set.use_graph && !h->set.timing) {
    int rc = capture_graph(h, stop);
    if (rc) return rc;
    for (int32_t i = 0; i < k; ++i) HIPCHK(hipGraphLaunch(h->graph[stop], h->stream));
    return 0;
  }
  for (int32_t i = 0; i < k; ++i) {
    int rc = launch_iteration(h, stop);
    if (rc) return rc;
  }
  return 0;
}

int read_infos(cdcs_handle* h, cdcs_info* infos) {
  HIPCHK(hipStreamSynchronize(h->stream));
  harvest_timers(h);
  if (!infos) return 0;
  std::vector<double> sc((size_t)h->B * kNsc);
  std::vector<int32_t> st((size_t)h->B * kNst);
  HIPCHK(hipMemcpy(sc.data(), h->d.sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(st.data(), h->d.st, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < h->B; ++i) {
    const double* s = &sc[(size_t)i * kNsc];
    cdcs_info& o = infos[i];
    o.iter = st[(size_t)i * kNst + ST_ITER];
    o.status = st[(size_t)i * kNst + ST_STATUS];
    o.eps_p = s[SC_EPS_P];
    o.eps_d = s[SC_EPS_D];
    o.eps_g = s[SC_EPS_G];
    o.tau = s[SC_TAU];
    o.kappa = s[SC_KAPPA];
    o.cx = s[SC_CX];
    o.by = s[SC_BY];
    o.obj_p = s[SC_TAU] > 0 ? s[SC_CX] / s[SC_TAU] : NAN;
    o.obj_d = s[SC_TAU] > 0 ? s[SC_BY] / s[SC_TAU] : NAN;
  }
  return 0;
}

int pack_and_upload(cdcs_handle* h) {
  const int32_t B = h->B;
  auto& I = h->inst;
  h->ent_off.assign(B + 1, 0);
  h->slot_off.assign(B + 1, 0);
  h->row_off.assign(B + 1, 0);
  h->clq_off.assign(B + 1, 0);
  for (int32_t i = 0; i < B; ++i) {
    h->ent_off[i + 1] = h->ent_off[i] + I[i].nE;
    h->slot_off[i + 1] = h->slot_off[i] + I[i].ns;
    h->row_off[i + 1] = h->row_off[i] + I[i].m;
    h->clq_off[i + 1] = h->clq_off[i] + I[i].p;
  }
  const int64_t NE = h->ent_off[B], NS = h->slot_off[B];
  const int32_t M = h->row_off[B], P = h->clq_off[B];
  int64_t nnzA = 0;
  for (auto& in : I) nnzA += (int64_t)in.acol.size();
  if (NE >= INT32_MAX || NS >= INT32_MAX || nnzA >= INT32_MAX)
    return set_error(CDCS_E_ARG, "batch too large for 32-bit indices");
  DevPlan& d = h->d;
  d.B = B;
  d.M = M;
  d.NE = NE;
  d.NS = NS;
  d.P = P;
  // entry space
  std::vector<double> c(NE), pinv(NE), halfD(NE), ztx(NE), atzy(NE);
  std::vector<int32_t> slot2ent(NS), sptr(NE + 1, 0), slots(NS);
  for (int32_t i = 0; i < B; ++i) {
    const int64_t eo = h->ent_off[i], so = h->slot_off[i];
    for (int64_t e = 0; e < I[i].nE; ++e) {
      c[eo + e] = I[i].c[e];
      // self-dual: P^{-1} = 1 / (1 + D/2); primal/dual-only methods: D^{-1}
      pinv[eo + e] = h->set.method ? 1.0 / (double)I[i].D[e] : 1.0 / (1.0 + 0.5 * I[i].D[e]);
      halfD[eo + e] = 0.5 * I[i].D[e];
      ztx[eo + e] = I[i].zt_x[e];
      atzy[eo + e] = I[i].atzy[e];
    }
    for (int64_t s = 0; s < I[i].ns; ++s) {
      slot2ent[so + s] = (int32_t)(eo + I[i].slot2ent[s]);
      sptr[eo + I[i].slot2ent[s] + 1]++;
    }
  }
  for (int64_t e = 0; e < NE; ++e) sptr[e + 1] += sptr[e];
  {
    std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
    for (int64_t s = 0; s < NS; ++s) slots[fill[slot2ent[s]]++] = (int32_t)s;
  }
  int rc;
  if ((rc = dev_upload(h, (double**)&d.c, c)) || (rc = dev_upload(h, (double**)&d.pinv, pinv)) ||
      (rc = dev_upload(h, (double**)&d.halfD, halfD)) || (rc = dev_upload(h, (double**)&d.zt_x, ztx)) ||
      (rc = dev_upload(h, (double**)&d.atzy, atzy)) || (rc = dev_upload(h, (int32_t**)&d.ent_sptr, sptr)) ||
      (rc = dev_upload(h, (int32_t**)&d.ent_slots, slots)) ||
      (rc = dev_upload(h, (int32_t**)&d.slot2ent, slot2ent)) || (rc = dev_zeros(h, &d.x, NE)) ||
      (rc = dev_zeros(h, &d.hsum, NE)) || (rc = dev_zeros(h, &d.q, NE)) || (rc = dev_zeros(h, &d.px, NE)) ||
      (rc = dev_zeros(h, &d.atw, NE)) || (rc = dev_zeros(h, &d.s, NS)) || (rc = dev_zeros(h, &d.z, NS)) ||
      (rc = dev_zeros(h, &d.v, NS)))
    return rc;
  // row space and A, A^T
  std::vector<double> b(M), zty(M), aval(nnzA), atval(nnzA);
  std::vector<int32_t> aptr(M + 1, 0), acol(nnzA), atptr(NE + 1, 0), atrow(nnzA);
  {
    int64_t at = 0;
    for (int32_t i = 0; i < B; ++i) {
      const int32_t ro = h->row_off[i];
      const int64_t eo = h->ent_off[i];
      for (int32_t r = 0; r < I[i].m; ++r) {
        b[ro + r] = I[i].b[r];
        zty[ro + r] = I[i].zt_y[r];
        aptr[ro + r] = (int32_t)at;
        for (int32_t q = I[i].aptr[r]; q < I[i].aptr[r + 1]; ++q) {
          acol[at] = (int32_t)(eo + I[i].acol[q]);
          aval[at] = I[i].aval[q];
          atptr[acol[at] + 1]++;
          ++at;
        }
      }
    }
    aptr[M] = (int32_t)at;
    for (int64_t e = 0; e < NE; ++e) atptr[e + 1] += atptr[e];
    std::vector<int32_t> fill(atptr.begin(), atptr.end() - 1);
    for (int32_t r = 0; r < M; ++r)
      for (int32_t q = aptr[r]; q < aptr[r + 1]; ++q) {
        const int32_t pos = fill[acol[q]]++;
        atrow[pos] = r;
        atval[pos] = aval[q];
      }
  }
  if ((rc = dev_upload(h, (double**)&d.b, b)) || (rc = dev_upload(h, (double**)&d.zt_y, zty)) ||
      (rc = dev_upload(h, (int32_t**)&d.a_ptr, aptr)) || (rc = dev_upload(h, (int32_t**)&d.a_col, acol)) ||
      (rc = dev_upload(h, (double**)&d.a_val, aval)) || (rc = dev_upload(h, (int32_t**)&d.at_ptr, atptr)) ||
      (rc = dev_upload(h, (int32_t**)&d.at_row, atrow)) || (rc = dev_upload(h, (double**)&d.at_val, atval)) ||
      (rc = dev_zeros(h, &d.y, M)) || (rc = dev_zeros(h, &d.g, M)) || (rc = dev_zeros(h, &d.w, M)) ||
      (rc = dev_zeros(h, &d.trsv_z, M)))
    return rc;
  // relaxed steps 2-3: u_hat_x and the previous iterate's products
  d.alpha = h->set.alpha;
  d.relax = h->set.alpha != 1.0;
  d.xh = d.x;
  d.atyo = d.hvo = d.axo = nullptr;
  if (d.relax && ((rc = dev_zeros(h, &d.xh, NE)) || (rc = dev_zeros(h, &d.atyo, NE)) ||
                  (rc = dev_zeros(h, &d.hvo, NE)) || (rc = dev_zeros(h, &d.axo, M))))
    return rc;
  // factors
  std::vector<int32_t> fmode(B), perm(M, 0), lptr, lcol, uptr, ucol, flev_off(B + 1, 0), flev_ptr,
      flev_rows, blev_off(B + 1, 0), blev_ptr, blev_rows;
  std::vector<int64_t> fdoff(B, 0);
  std::vector<double> Ld, Ldt, Kinv, fdiag(M, 1.0), lval, uval;
  int32_t dense_m = 0;
  for (int32_t i = 0; i < B; ++i) {
    const Factor& f = I[i].fac;
    const int32_t ro = h->row_off[i];
    fmode[i] = f.dense ? (f.Kinv.empty() ? 0 : 2) : 1;
    if (f.dense) {
      fdoff[i] = (int64_t)Ld.size();
      Ld.insert(Ld.end(), f.Ld.begin(), f.Ld.end());
      Ldt.resize(Ld.size());
      for (int32_t c = 0; c < f.m; ++c)
        for (int32_t r = 0; r < f.m; ++r) Ldt[fdoff[i] + (size_t)r * f.m + c] = f.Ld[(size_t)c * f.m + r];
      dense_m = std::max(dense_m, f.m);
      Kinv.resize(Ld.size());
      if (!f.Kinv.empty()) std::copy(f.Kinv.begin(), f.Kinv.end(), Kinv.begin() + fdoff[i]);
      for (int32_t r = 0; r < f.m; ++r) lptr.push_back((int32_t)lcol.size());
      lptr.push_back((int32_t)lcol.size());
      for (int32_t r = 0; r < f.m; ++r) uptr.push_back((int32_t)ucol.size());
      uptr.push_back((int32_t)ucol.size());
    } else {
      for (int32_t r = 0; r < f.m; ++r) {
        perm[ro + r] = f.perm[r];
        fdiag[ro + r] = f.diag[r];
      }
      const int32_t lbase = (int32_t)lcol.size(), ubase = (int32_t)ucol.size();
      for (int32_t r = 0; r <= f.m; ++r) lptr.push_back(lbase + f.lptr[r]);
      for (int32_t r = 0; r <= f.m; ++r) uptr.push_back(ubase + f.uptr[r]);
      lcol.insert(lcol.end(), f.lcol.begin(), f.lcol.end());
      lval.insert(lval.end(), f.lval.begin(), f.lval.end());
      ucol.insert(ucol.end(), f.ucol.begin(), f.ucol.end());
      uval.insert(uval.end(), f.uval.begin(), f.uval.end());
      const int32_t fb = (int32_t)flev_rows.size(), bb = (int32_t)blev_rows.size();
      for (size_t l = 0; l + 1 < f.flev_ptr.size(); ++l) flev_ptr.push_back(fb + f.flev_ptr[l]);
      for (size_t l = 0; l + 1 < f.blev_ptr.size(); ++l) blev_ptr.push_back(bb + f.blev_ptr[l]);
      flev_rows.insert(flev_rows.end(), f.flev_rows.begin(), f.flev_rows.end());
      blev_rows.insert(blev_rows.end(), f.blev_rows.begin(), f.blev_rows.end());
    }
    flev_off[i + 1] = (int32_t)flev_ptr.size();
    blev_off[i + 1] = (int32_t)blev_ptr.size();
  }
  flev_ptr.push_back((int32_t)flev_rows.size());
  blev_ptr.push_back((int32_t)blev_rows.size());
  if ((rc = dev_upload(h, (int32_t**)&d.f_mode, fmode)) || (rc = dev_upload(h, (int64_t**)&d.f_dense_off, fdoff)) ||
      (rc = dev_upload(h, (double**)&d.f_Ld, Ld)) || (rc = dev_upload(h, (double**)&d.f_Ldt, Ldt)) ||
      (rc = dev_upload(h, (double**)&d.f_Kinv, Kinv)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_perm, perm)) ||
      (rc = dev_upload(h, (double**)&d.f_diag, fdiag)) || (rc = dev_upload(h, (int32_t**)&d.f_lptr, lptr)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_lcol, lcol)) || (rc = dev_upload(h, (double**)&d.f_lval, lval)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_uptr, uptr)) || (rc = dev_upload(h, (int32_t**)&d.f_ucol, ucol)) ||
      (rc = dev_upload(h, (double**)&d.f_uval, uval)) || (rc = dev_upload(h, (int32_t**)&d.f_flev_off, flev_off)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_flev_ptr, flev_ptr)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_flev_rows, flev_rows)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_blev_off, blev_off)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_blev_ptr, blev_ptr)) ||
      (rc = dev_upload(h, (int32_t**)&d.f_blev_rows, blev_rows)))
    return rc;
  // rows per thread of the dense sweeps (256 threads; the dense form has m <= 2048)
  d.trsv_rows = dense_m <= 256 ? 1 : dense_m <= 512 ? 2 : dense_m <= 1024 ? 4 : 8;
  if (dense_m > 2048) return set_error(CDCS_E_ARG, "dense factor of order > 2048");
  // blocks
  std::vector<int4> eblk, rblk;
  std::vector<int32_t> eblk_off(B + 1, 0), rblk_off(B + 1, 0);
  for (int32_t i = 0; i < B; ++i) {
    for (int64_t e = h->ent_off[i]; e < h->ent_off[i + 1]; e += kEntChunk)
      eblk.push_back(make_int4(i, (int)e, (int)std::min<int64_t>(e + kEntChunk, h->ent_off[i + 1]), 0));
    for (int32_t r = h->row_off[i]; r < h->row_off[i + 1]; r += kRowChunk)
      rblk.push_back(make_int4(i, r, std::min(r + kRowChunk, h->row_off[i + 1]), 0));
    eblk_off[i + 1] = (int32_t)eblk.size();
    rblk_off[i + 1] = (int32_t)rblk.size();
  }
  d.n_eblk = (int32_t)eblk.size();
  d.n_rblk = (int32_t)rblk.size();
  // A^T as sliced ELL over the entry blocks (k_spmv_at): per block, entries
  // sorted by nonzero count (descending, stable), chunks of 64 lanes, each
  // chunk column-interleaved and zero-padded (row 0, value 0) to its first
  // entry's count
  {
    std::vector<int32_t> choff(eblk.size()), chlen, sent, srow, order;
    std::vector<int64_t> chptr;
    std::vector<double> sval;
    int64_t pos = 0;
    auto cnt = [&](int32_t e) { return atptr[e + 1] - atptr[e]; };
    for (size_t bi = 0; bi < eblk.size(); ++bi) {
      const int32_t e0 = eblk[bi].y, e1 = eblk[bi].z;
      choff[bi] = (int32_t)chlen.size();
      order.resize(e1 - e0);
      std::iota(order.begin(), order.end(), e0);
      std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return cnt(a) > cnt(c); });
      for (int32_t c0 = 0; c0 < e1 - e0; c0 += 64) {
        const int32_t n = std::min<int32_t>(64, e1 - e0 - c0);
        const int32_t len = cnt(order[c0]);
        chptr.push_back(pos);
        chlen.push_back(len);
        for (int32_t l = 0; l < 64; ++l) sent.push_back(l < n ? order[c0 + l] : -1);
        for (int32_t k = 0; k < len; ++k)
          for (int32_t l = 0; l < 64; ++l) {
            int32_t r = 0;
            double v = 0.0;
            if (l < n && k < cnt(order[c0 + l])) {
              r = atrow[atptr[order[c0 + l]] + k];
              v = atval[atptr[order[c0 + l]] + k];
            }
            srow.push_back(r);
            sval.push_back(v);
          }
        pos += (int64_t)len * 64;
      }
    }
    if ((rc = dev_upload(h, (int32_t**)&d.at_choff, choff)) || (rc = dev_upload(h, (int64_t**)&d.at_chptr, chptr)) ||
        (rc = dev_upload(h, (int32_t**)&d.at_chlen, chlen)) || (rc = dev_upload(h, (int32_t**)&d.at_sent, sent)) ||
        (rc = dev_upload(h, (int32_t**)&d.at_srow, srow)) || (rc = dev_upload(h, (double**)&d.at_sval, sval)))
      return rc;
  }
  std::vector<int64_t> ent_off64(h->ent_off);
  if ((rc = dev_upload(h, (int4**)&d.eblk, eblk)) || (rc = dev_upload(h, (int4**)&d.rblk, rblk)) ||
      (rc = dev_upload(h, (int32_t**)&d.eblk_off, eblk_off)) ||
      (rc = dev_upload(h, (int32_t**)&d.rblk_off, rblk_off)) ||
      (rc = dev_upload(h, (int64_t**)&d.ent_off, ent_off64)) ||
      (rc = dev_upload(h, (int32_t**)&d.row_off, h->row_off)) ||
      (rc = dev_upload(h, (int32_t**)&d.clq_off, h->clq_off)) ||
      (rc = dev_zeros(h, &d.part_e, (size_t)d.n_eblk * 4)) ||
      (rc = dev_zeros(h, &d.part_r, (size_t)d.n_rblk * 4)) || (rc = dev_zeros(h, &d.part_c, (size_t)P * 2)))
    return rc;
  // cliques and cone work lists (bucketed by size, largest first within a bucket)
  std::vector<int32_t> csize(P), cinst(P);
  std::vector<int64_t> cslot(P);
  std::vector<std::vector<int32_t>> bk(5), abk(4);
  const int jmax = jacobi_max_of(h->set);
  h->max_clique = 0;
  for (int32_t i = 0; i < B; ++i)
    for (int32_t k = 0; k < I[i].p; ++k) {
      const int32_t g = h->clq_off[i] + k;
      csize[g] = I[i].csize[k];
      cinst[g] = i;
      cslot[g] = h->slot_off[i] + I[i].slot_off[k];
      bk[bucket_of(csize[g], jmax)].push_back(g);
      // the adjoint's eigen-cache runs Jacobi on every clique of up to
      // kAdjMax vertices, whichever path the forward iteration routes it to
      if (csize[g] <= kAdjMax) abk[bucket_of(csize[g], kAdjMax)].push_back(g);
      h->max_clique = std::max(h->max_clique, csize[g]);
    }
  for (auto& v : bk)
    std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b2) { return csize[a] > csize[b2]; });
  for (auto& v : abk)
    std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b2) { return csize[a] > csize[b2]; });
  for (int bkt = 0; bkt < 4; ++bkt) {
    h->adj_ntasks[bkt] = (int32_t)abk[bkt].size();
    if ((rc = dev_upload(h, &h->adj_tasks[bkt], abk[bkt]))) return rc;
  }
  if ((rc = dev_upload(h, (int32_t**)&d.clq_size, csize)) || (rc = dev_upload(h, (int32_t**)&d.clq_inst, cinst)) ||
      (rc = dev_upload(h, (int64_t**)&d.clq_slot, cslot)))
    return rc;
  // warm-started Jacobi: K^2 stored eigenvector entries per Jacobi clique
  d.warm_v = nullptr;
  d.warm_off = nullptr;
  if (h->set.eig_warm) {
    std::vector<int64_t> woff(P, 0);
    int64_t tot = 0;
    for (int32_t g = 0; g < P; ++g)
      if (csize[g] <= kJacobiMax) {
        woff[g] = tot;
        tot += (int64_t)csize[g] * csize[g];
      }
    const size_t esz = h->set.eig_fp32 ? sizeof(float) : sizeof(double);
    double* wv = nullptr;
    if ((rc = dev_zeros(h, &wv, (size_t)((tot * esz + sizeof(double) - 1) / sizeof(double)))) ||
        (rc = dev_upload(h, (int64_t**)&d.warm_off, woff)))
      return rc;
    d.warm_v = wv;
  }
  for (int bkt = 0; bkt < 5; ++bkt) {
    h->ntasks[bkt] = (int32_t)bk[bkt].size();
    if ((rc = dev_upload(h, &h->tasks[bkt], bk[bkt]))) return rc;
    if (bkt < 4) {
      h->bucket_sizes[bkt].clear();
      for (int32_t g : bk[bkt]) h->bucket_sizes[bkt].push_back(csize[g]);
    }
  }
  // large-clique workspace: one K x K (column-major) matrix + eigen data per task
  h->large_sizes.clear();
  std::vector<int64_t> boff;
  int64_t btot = 0;
  for (int32_t g : bk[4]) {
    const int64_t K = csize[g];
    h->large_sizes.push_back((int32_t)K);
    h->kmax_large = std::max<int32_t>(h->kmax_large, (int32_t)K);
    boff.push_back(btot);
    btot += large_work_size((int)K);
  }
  boff.push_back(btot);
  if ((rc = dev_zeros(h, &d.big_work, (size_t)btot)) || (rc = dev_upload(h, (int64_t**)&d.big_off, boff)) ||
      (rc = dev_upload(h, (int32_t**)&d.big_size, h->large_sizes)))
    return rc;
  // scalars and status
  std::vector<double> sc((size_t)B * kNsc, 0.0);
  for (int32_t i = 0; i < B; ++i) {
    double* s = &sc[(size_t)i * kNsc];
    // (the primal/dual-only methods keep tau = 1, kappa = 0: objectives are
    // c^T x and b^T y as they stand)
    s[SC_TAU] = 1.0;
    s[SC_KAPPA] = h->set.method ? 0.0 : 1.0;
    s[SC_DEN] = I[i].den;
    s[SC_CTZX] = I[i].ctzx;
    s[SC_BTZY] = I[i].btzy;
    s[SC_NB] = I[i].nb;
    s[SC_NC] = I[i].nc;
  }
  if ((rc = dev_upload(h, &d.sc, sc)) || (rc = dev_zeros(h, &d.st, (size_t)B * kNst))) return rc;
  if (h->set.method) {
    // slot blocks (never straddling an instance), projection buffers, partials
    std::vector<int4> sblk;
    std::vector<int32_t> sblk_off(B + 1, 0);
    for (int32_t i = 0; i < B; ++i) {
      for (int64_t q = h->slot_off[i]; q < h->slot_off[i + 1]; q += kSlotChunk)
        sblk.push_back(make_int4(i, (int)q, (int)std::min<int64_t>(q + kSlotChunk, h->slot_off[i + 1]), 0));
      sblk_off[i + 1] = (int32_t)sblk.size();
    }
    SplitArgs& a = h->sa;
    a.rho = h->set.rho;
    a.n_sblk = (int32_t)sblk.size();
    if ((rc = dev_upload(h, (int4**)&a.sblk, sblk)) || (rc = dev_upload(h, (int32_t**)&a.sblk_off, sblk_off)) ||
        (rc = dev_zeros(h, &a.w, NS)) || (rc = dev_zeros(h, &a.p, NS)) ||
        (rc = dev_zeros(h, &a.part_s, (size_t)std::max<int32_t>(a.n_sblk, 1) * kSplitParts)))
      return rc;
  }
  return 0;
}

bool valid_inst(const cdcs_handle* h, int32_t inst) { return h && inst >= 0 && inst < h->B; }

// ---------------------------------------------------------------------------
// the conic step on its own (cdcs_psd_project and its no-allocation variant)
// ---------------------------------------------------------------------------

// host plan: blocks split into the four Jacobi buckets and the large-clique
// list (largest first), with the large workspace offsets
struct ProjPlan {
  std::vector<int32_t> sizes;
  std::vector<int64_t> offs;
  std::vector<int32_t> bk[5];
  std::vector<int32_t> large_sizes;
  std::vector<int64_t> woff;
  int64_t wtot = 0;
  int32_t kmax_large = 0;
};

// device copies of the plan's arrays and the large workspace
struct ProjDev {
  int32_t* sizes = nullptr;
  int64_t* offs = nullptr;
  int32_t* tasks[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t* woff = nullptr;
  int32_t* lsz = nullptr;
  double* work = nullptr;
};

int plan_projection(int32_t count, const int32_t* sizes, const int64_t* offsets, ProjPlan* pl) {
  for (int32_t k = 0; k < count; ++k) {
    if (sizes[k] < 1 || sizes[k] > 1024 || offsets[k] < 0) return set_error(CDCS_E_ARG, "block size must be 1..1024");
    pl->bk[bucket_of(sizes[k])].push_back(k);
  }
  std::stable_sort(pl->bk[4].begin(), pl->bk[4].end(), [&](int32_t x, int32_t y) { return sizes[x] > sizes[y]; });
  for (int32_t k : pl->bk[4]) {
    pl->large_sizes.push_back(sizes[k]);
    pl->kmax_large = std::max(pl->kmax_large, sizes[k]);
    pl->woff.push_back(pl->wtot);
    pl->wtot += large_work_size(sizes[k]);
  }
  pl->woff.push_back(pl->wtot);
  pl->sizes.assign(sizes, sizes + count);
  pl->offs.assign(offsets, offsets + count);
  return 0;
}

void launch_projection(const ProjPlan& pl, const ProjDev& dv, const double* in, double* out, hipStream_t st) {
  const int kmaxs[4] = {16, 32, 64, 96};   // bucket orders (the last is empty while kJacobiMax = 64)
  for (int b = 0; b < 4; ++b)
    launch_psd_project(dv.sizes, dv.offs, dv.tasks[b], (int32_t)pl.bk[b].size(), kmaxs[b], in, out, st);
  if (!pl.bk[4].empty())
    launch_psd_project_large(dv.sizes, dv.offs, dv.tasks[4], dv.lsz, pl.large_sizes.data(),
                             (int32_t)pl.bk[4].size(), pl.kmax_large, in, out, dv.work, dv.woff, st);
}

__global__ void k_fill_zero(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

unsigned fill_blocks(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 2048); }

// Device scratch of cdcs_psd_project_noalloc: every GPU the library runs on
// holds one copy from module load until the process ends.  Host code never
// uses the array's name as an address (on the host it is only a stand-in
// for the symbol): scratch_base() looks its device address up once per
// device and every later use goes through that pointer.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

int scratch_base(unsigned char** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(CDCS_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(CDCS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}


}  // namespace

extern "C" {

void cdcs_default_settings(cdcs_settings* s) {
  if (!s) return;
  s->eps_tol = 1e-4;
  s->max_iter = 2000;
  s->check_every = 1;
  s->timing = 0;
  s->use_graph = 0;
  s->eig_fp32 = 0;
  s->autotune = 0;
  s->alpha = 1.0;
  s->eig_warm = 0;
  s->method = CDCS_METHOD_SELF_DUAL;
  s->rho = 1.0;
  s->jacobi_max = 0;
  s->band_min = 0;
}

int cdcs_abi_version(void) { return CDCS_ABI_VERSION; }

const char* cdcs_last_error(void) { return g_last_error.c_str(); }

void cdcs_destroy(cdcs_handle* h) {
  if (!h) return;
  if (h->aux) (void)hipStreamSynchronize(h->aux);
  for (int i = 0; i < 3; ++i)
    if (h->jst[i]) (void)hipStreamSynchronize(h->jst[i]);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (int i = 0; i < 2; ++i)
    if (h->graph[i]) (void)hipGraphExecDestroy(h->graph[i]);
  for (auto& e : h->ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  for (int i = 0; i < 3; ++i) {
    if (h->ev_jjoin[i]) (void)hipEventDestroy(h->ev_jjoin[i]);
    if (h->jst[i]) (void)hipStreamDestroy(h->jst[i]);
  }
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

int cdcs_setup_batch(int32_t count, const cdcs_problem* prob, const cdcs_settings* s, void* stream,
                     cdcs_handle** out) {
  if (!out) return set_error(CDCS_E_ARG, "null output handle");
  *out = nullptr;
  if (count < 1 || !prob) return set_error(CDCS_E_ARG, "need count >= 1 problems");
  cdcs_settings set;
  cdcs_default_settings(&set);
  if (s) set = *s;
  if (!(set.eps_tol > 0.0) || set.max_iter < 1 || set.check_every < 1)
    return set_error(CDCS_E_ARG, "settings: need eps_tol > 0, max_iter >= 1, check_every >= 1");
  if ((set.eig_fp32 != 0 && set.eig_fp32 != 1) || set.autotune < 0 || set.autotune > 2)
    return set_error(CDCS_E_ARG, "settings: eig_fp32 must be 0 or 1 and autotune 0, 1 or 2");
  if (!(set.alpha > 0.0 && set.alpha < 2.0))
    return set_error(CDCS_E_ARG, "settings: alpha must lie in (0, 2)");
  if (set.eig_warm != 0 && set.eig_warm != 1) return set_error(CDCS_E_ARG, "settings: eig_warm must be 0 or 1");
  if (set.method < CDCS_METHOD_SELF_DUAL || set.method > CDCS_METHOD_DUAL)
    return set_error(CDCS_E_ARG, "settings: method must be 0 (self-dual), 1 (primal) or 2 (dual)");
  if (set.method != CDCS_METHOD_SELF_DUAL && (!(set.rho > 0.0) || !std::isfinite(set.rho)))
    return set_error(CDCS_E_ARG, "settings: rho must be positive");
  if (set.jacobi_max != 0 && set.jacobi_max != 16 && set.jacobi_max != 32 && set.jacobi_max != 64)
    return set_error(CDCS_E_ARG, "settings: jacobi_max must be 0 (automatic), 16, 32 or 64");
  if (set.band_min != 0 && set.band_min < kBandMinDefault)
    return set_error(CDCS_E_ARG, "settings: band_min must be 0 or at least 137");
  if (set.method != CDCS_METHOD_SELF_DUAL && (set.alpha != 1.0 || set.eig_warm != 0))
    return set_error(CDCS_E_ARG, "settings: alpha and eig_warm apply to the self-dual method only");
  const auto t0 = std::chrono::steady_clock::now();
  cdcs_handle* h = new cdcs_handle();
  h->stream = (hipStream_t)stream;
  if (!h->stream) {
    // a stream of our own (default priority) so that the iteration can be captured
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return set_error(CDCS_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    h->own_stream = true;
  }
  bool made = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < 3 && made; ++i)
    made = hipStreamCreateWithFlags(&h->jst[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&h->ev_jjoin[i], hipEventDisableTiming) == hipSuccess;
  if (!made) {
    cdcs_destroy(h);
    return set_error(CDCS_E_DEVICE, "stream/event creation failed");
  }
  h->set = set;
  h->B = count;
  h->inst.resize(count);
  // host setup of independent instances in parallel
  std::vector<int> rcs(count, 0);
  std::vector<Error> errs(count);
  const int nthr = std::max(1, std::min<int>(count, (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
  std::vector<std::thread> pool;
  for (int t = 0; t < nthr; ++t)
    pool.emplace_back([&, t]() {
      for (int i = t; i < count; i += nthr) rcs[i] = build_instance(prob[i], h->inst[i], errs[i], set.method);
    });
  for (auto& th : pool) th.join();
  for (int i = 0; i < count; ++i)
    if (rcs[i]) {
      int rc = set_error(rcs[i], "instance " + std::to_string(i) + ": " + errs[i].msg);
      cdcs_destroy(h);
      return rc;
    }
  int rc = pack_and_upload(h);
  if (!rc && h->set.autotune == 1) rc = autotune(h);
  if (!rc && h->set.autotune == 2)
    for (int b = 0; b < 4; ++b) h->jvar[b] = 1;
  if (rc) {
    cdcs_destroy(h);
    return rc;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    cdcs_destroy(h);
    return set_error(CDCS_E_DEVICE, std::string("setup sync: ") + hipGetErrorString(e));
  }
  h->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return 0;
}

int cdcs_setup(const cdcs_problem* prob, const cdcs_settings* s, void* stream, cdcs_handle** out) {
  return cdcs_setup_batch(1, prob, s, stream, out);
}

int cdcs_iterate(cdcs_handle* h, int32_t k, cdcs_info* infos) {
  if (!h || k < 0) return set_error(CDCS_E_ARG, "bad handle or k");
  // exactly k iterations of every instance: nothing is frozen
  std::vector<int32_t> st((size_t)h->B * kNst);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(st.data(), h->d.st, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < h->B; ++i) st[(size_t)i * kNst + ST_FROZEN] = 0;
  HIPCHK(hipMemcpy(h->d.st, st.data(), st.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  int rc = run_iterations(h, k, 0);
  if (rc) return rc;
  return read_infos(h, infos);
}

int cdcs_solve(cdcs_handle* h, cdcs_info* infos) {
  if (!h) return set_error(CDCS_E_ARG, "null handle");
  std::vector<int32_t> st((size_t)h->B * kNst);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(st.data(), h->d.st, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < h->B; ++i) {
    int32_t* s = &st[(size_t)i * kNst];
    s[ST_FROZEN] = (s[ST_STATUS] != CDCS_RUNNING || s[ST_ITER] >= h->set.max_iter) ? 1 : 0;
    if (s[ST_STATUS] == CDCS_RUNNING && s[ST_ITER] >= h->set.max_iter) s[ST_STATUS] = CDCS_MAX_ITER;
  }
  HIPCHK(hipMemcpy(h->d.st, st.data(), st.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  for (;;) {
    bool all = true;
    int32_t maxit = 0;
    for (int32_t i = 0; i < h->B; ++i) {
      all = all && st[(size_t)i * kNst + ST_FROZEN];
      maxit = std::max(maxit, st[(size_t)i * kNst + ST_ITER]);
    }
    if (all) break;
    const int32_t chunk = std::min(h->set.check_every, std::max(1, h->set.max_iter - maxit));
    int rc = run_iterations(h, chunk, 1);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(st.data(), h->d.st, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  return read_infos(h, infos);
}

int cdcs_get_dims(const cdcs_handle* h, int32_t inst, int64_t dims[4]) {
  if (!valid_inst(h, inst) || !dims) return set_error(CDCS_E_ARG, "bad handle, instance or dims");
  dims[0] = h->inst[inst].nE;
  dims[1] = h->inst[inst].ns;
  dims[2] = h->inst[inst].m;
  dims[3] = h->inst[inst].p;
  return 0;
}

int cdcs_get_entries(const cdcs_handle* h, int32_t inst, int32_t* row, int32_t* col) {
  if (!valid_inst(h, inst)) return set_error(CDCS_E_ARG, "bad handle or instance");
  const Instance& I = h->inst[inst];
  if (row) std::memcpy(row, I.erow.data(), I.nE * sizeof(int32_t));
  if (col) std::memcpy(col, I.ecol.data(), I.nE * sizeof(int32_t));
  return 0;
}

namespace {

struct HostState {
  std::vector<double> x, s, y, v, z;
  double tau = 0, kappa = 0;
  int32_t status = 0, iter = 0;
};

int fetch_state(const cdcs_handle* h, int32_t inst, HostState& S) {
  const Instance& I = h->inst[inst];
  HIPCHK(hipStreamSynchronize(h->stream));
  const int64_t eo = h->ent_off[inst], so = h->slot_off[inst];
  const int32_t ro = h->row_off[inst];
  S.x.resize(I.nE);
  S.s.resize(I.ns);
  S.z.resize(I.ns);
  S.v.resize(I.ns);
  S.y.resize(I.m);
  HIPCHK(hipMemcpy(S.x.data(), h->d.x + eo, I.nE * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(S.s.data(), h->d.s + so, I.ns * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(S.z.data(), h->d.z + so, I.ns * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(S.v.data(), h->d.v + so, I.ns * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(S.y.data(), h->d.y + ro, I.m * sizeof(double), hipMemcpyDeviceToHost));
  double sc[kNsc];
  int32_t st[kNst];
  HIPCHK(hipMemcpy(sc, h->d.sc + (size_t)inst * kNsc, sizeof(sc), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(st, h->d.st + (size_t)inst * kNst, sizeof(st), hipMemcpyDeviceToHost));
  S.tau = sc[SC_TAU];
  S.kappa = sc[SC_KAPPA];
  S.status = st[ST_STATUS];
  S.iter = st[ST_ITER];
  return 0;
}

int put_out(const cdcs_handle* h, double* dst, const std::vector<double>& src, int32_t on_device) {
  if (!dst) return 0;
  if (on_device) {
    HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  } else {
    std::memcpy(dst, src.data(), src.size() * sizeof(double));
  }
  return 0;
}

}  // namespace

int cdcs_get_state(const cdcs_handle* h, int32_t inst, double* u, double* vt) {
  if (!valid_inst(h, inst)) return set_error(CDCS_E_ARG, "bad handle or instance");
  HostState S;
  int rc = fetch_state(h, inst, S);
  if (rc) return rc;
  const Instance& I = h->inst[inst];
  if (h->set.method != CDCS_METHOD_SELF_DUAL) {
    // primal/dual-only methods: u = (x, s or z, y), vt = lam (primal) or (lam, v) (dual)
    if (u) {
      double* p = u;
      std::memcpy(p, S.x.data(), I.nE * sizeof(double)); p += I.nE;
      std::memcpy(p, S.s.data(), I.ns * sizeof(double)); p += I.ns;
      std::memcpy(p, S.y.data(), I.m * sizeof(double));
    }
    if (vt) {
      std::memcpy(vt, S.z.data(), I.ns * sizeof(double));
      if (h->set.method == CDCS_METHOD_DUAL) std::memcpy(vt + I.ns, S.v.data(), I.ns * sizeof(double));
    }
    return 0;
  }
  if (u) {
    double* p = u;
    std::memcpy(p, S.x.data(), I.nE * sizeof(double)); p += I.nE;
    std::memcpy(p, S.s.data(), I.ns * sizeof(double)); p += I.ns;
    std::memcpy(p, S.y.data(), I.m * sizeof(double)); p += I.m;
    std::memcpy(p, S.v.data(), I.ns * sizeof(double)); p += I.ns;
    *p = S.tau;
  }
  if (vt) {
    double* p = vt;
    std::memset(p, 0, I.nE * sizeof(double)); p += I.nE;
    std::memcpy(p, S.z.data(), I.ns * sizeof(double)); p += I.ns;
    std::memset(p, 0, I.m * sizeof(double)); p += I.m;
    std::memset(p, 0, I.ns * sizeof(double)); p += I.ns;
    *p = S.kappa;
  }
  return 0;
}

int cdcs_set_state(cdcs_handle* h, int32_t inst, const double* u, const double* vt) {
  if (!valid_inst(h, inst) || !u || !vt) return set_error(CDCS_E_ARG, "bad handle, instance or state");
  const Instance& I = h->inst[inst];
  if (h->set.method != CDCS_METHOD_SELF_DUAL) {
    const int64_t eo = h->ent_off[inst], so = h->slot_off[inst];
    const int32_t ro = h->row_off[inst];
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(h->d.x + eo, u, I.nE * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d.s + so, u + I.nE, I.ns * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d.y + ro, u + I.nE + I.ns, I.m * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d.z + so, vt, I.ns * sizeof(double), hipMemcpyHostToDevice));
    if (h->set.method == CDCS_METHOD_DUAL)
      HIPCHK(hipMemcpy(h->d.v + so, vt + I.ns, I.ns * sizeof(double), hipMemcpyHostToDevice));
    int32_t st[kNst];
    HIPCHK(hipMemcpy(st, h->d.st + (size_t)inst * kNst, sizeof(st), hipMemcpyDeviceToHost));
    st[ST_STATUS] = CDCS_RUNNING;
    st[ST_FROZEN] = 0;
    HIPCHK(hipMemcpy(h->d.st + (size_t)inst * kNst, st, sizeof(st), hipMemcpyHostToDevice));
    return 0;
  }
  // h, r, w are identically zero along the iteration (step Step3); a state
  // with non-zero h, r or w is not one the method produces
  const double* hv = vt;
  const double* rv = vt + I.nE + I.ns;
  const double* wv = rv + I.m;
  for (int64_t e = 0; e < I.nE; ++e)
    if (hv[e] != 0.0) return set_error(CDCS_E_ARG, "h must be zero");
  for (int32_t r = 0; r < I.m; ++r)
    if (rv[r] != 0.0) return set_error(CDCS_E_ARG, "r must be zero");
  for (int64_t s = 0; s < I.ns; ++s)
    if (wv[s] != 0.0) return set_error(CDCS_E_ARG, "w must be zero");
  const int64_t eo = h->ent_off[inst], so = h->slot_off[inst];
  const int32_t ro = h->row_off[inst];
  HIPCHK(hipStreamSynchronize(h->stream));
  const double* p = u;
  HIPCHK(hipMemcpy(h->d.x + eo, p, I.nE * sizeof(double), hipMemcpyHostToDevice)); p += I.nE;
  HIPCHK(hipMemcpy(h->d.s + so, p, I.ns * sizeof(double), hipMemcpyHostToDevice)); p += I.ns;
  HIPCHK(hipMemcpy(h->d.y + ro, p, I.m * sizeof(double), hipMemcpyHostToDevice)); p += I.m;
  HIPCHK(hipMemcpy(h->d.v + so, p, I.ns * sizeof(double), hipMemcpyHostToDevice)); p += I.ns;
  const double tau = *p;
  HIPCHK(hipMemcpy(h->d.z + so, vt + I.nE, I.ns * sizeof(double), hipMemcpyHostToDevice));
  const double kappa = vt[I.nE + 2 * I.ns + I.m];
  double sc[kNsc];
  HIPCHK(hipMemcpy(sc, h->d.sc + (size_t)inst * kNsc, sizeof(sc), hipMemcpyDeviceToHost));
  sc[SC_TAU] = tau;
  sc[SC_KAPPA] = kappa;
  HIPCHK(hipMemcpy(h->d.sc + (size_t)inst * kNsc, sc, sizeof(sc), hipMemcpyHostToDevice));
  int32_t st[kNst];
  HIPCHK(hipMemcpy(st, h->d.st + (size_t)inst * kNst, sizeof(st), hipMemcpyDeviceToHost));
  st[ST_STATUS] = CDCS_RUNNING;
  st[ST_FROZEN] = 0;
  st[ST_WARM] = 0;   // stored eigenvectors belong to another iterate
  HIPCHK(hipMemcpy(h->d.st + (size_t)inst * kNst, st, sizeof(st), hipMemcpyHostToDevice));
  return 0;
}

int cdcs_get_solution(const cdcs_handle* h, int32_t inst, double* X, double* y, double* Z, int32_t on_device) {
  if (!valid_inst(h, inst)) return set_error(CDCS_E_ARG, "bad handle or instance");
  HostState S;
  int rc = fetch_state(h, inst, S);
  if (rc) return rc;
  if (S.status != CDCS_SOLVED || !(S.tau > 0)) return set_error(CDCS_E_STATE, "instance is not solved");
  const Instance& I = h->inst[inst];
  std::vector<double> xo(I.nE), yo(I.m), zo(I.nE, 0.0);
  for (int64_t e = 0; e < I.nE; ++e) xo[e] = S.x[e] / S.tau;
  for (int32_t r = 0; r < I.m; ++r) yo[r] = S.y[r] / S.tau;
  // Z = sum_k E_k^T Z_k E_k (Theorem 2) = H^T z / tau in svec coordinates;
  // the clique blocks Z_k are z (self-dual), the multiplier (primal-only
  // method) or the projected block (dual-only method)
  const std::vector<double>& zk = h->set.method == CDCS_METHOD_DUAL ? S.s : S.z;
  for (int64_t s = 0; s < I.ns; ++s) zo[I.slot2ent[s]] += zk[s];
  for (int64_t e = 0; e < I.nE; ++e) zo[e] /= S.tau;
  if ((rc = put_out(h, X, xo, on_device)) || (rc = put_out(h, y, yo, on_device)) || (rc = put_out(h, Z, zo, on_device)))
    return rc;
  return 0;
}

int cdcs_get_certificate(const cdcs_handle* h, int32_t inst, double* y_cert, double* X_cert, int32_t on_device) {
  if (!valid_inst(h, inst)) return set_error(CDCS_E_ARG, "bad handle or instance");
  if (h->set.method != CDCS_METHOD_SELF_DUAL)
    return set_error(CDCS_E_STATE, "the primal-only and dual-only methods give no infeasibility certificates");
  HostState S;
  int rc = fetch_state(h, inst, S);
  if (rc) return rc;
  const Instance& I = h->inst[inst];
  if (S.status == CDCS_PRIMAL_INFEASIBLE) {
    double by = 0.0;
    for (int32_t r = 0; r < I.m; ++r) by += I.b[r] * S.y[r];
    std::vector<double> yo(I.m);
    for (int32_t r = 0; r < I.m; ++r) yo[r] = S.y[r] / by;
    return put_out(h, y_cert, yo, on_device);
  }
  if (S.status == CDCS_DUAL_INFEASIBLE) {
    double cx = 0.0;
    for (int64_t e = 0; e < I.nE; ++e) cx += I.c[e] * S.x[e];
    std::vector<double> xo(I.nE);
    for (int64_t e = 0; e < I.nE; ++e) xo[e] = S.x[e] / (-cx);
    return put_out(h, X_cert, xo, on_device);
  }
  return set_error(CDCS_E_STATE, "instance is not infeasible");
}

namespace {

constexpr int kRestart = 20;

// point the adjoint plan's mu blocks at a flat vector
void adj_point(cdcs_handle* h, double* flat) {
  const int32_t B = h->B;
  const int64_t NE = h->ent_off[B], NS = h->slot_off[B];
  const int32_t M = h->row_off[B];
  h->adj.mu_x = flat;
  h->adj.mu_s = flat + NE;
  h->adj.mu_y = flat + NE + NS;
  h->adj.mu_v = flat + NE + NS + M;
  h->adj.mu_t = flat + NE + 2 * NS + M;
}

// data of the transposed solve (I - Q) q = mu that depends only on the problem:
// phi = F^{-1}(c + A^T b), A phi, e = c - A^T b, 1 + ||b||^2 + e^T phi
int adjoint_prepare(cdcs_handle* h) {
  if (h->adj_ready) return 0;
  const int32_t B = h->B;
  const int64_t NE = h->ent_off[B];
  const int32_t M = h->row_off[B], P = h->clq_off[B];
  std::vector<double> phi(NE), ev(NE), aphi(M), as((size_t)B * kNas, 0.0);
  for (int32_t i = 0; i < B; ++i) {
    const Instance& I = h->inst[i];
    const int64_t eo = h->ent_off[i];
    const int32_t ro = h->row_off[i];
    std::vector<double> atb(I.nE, 0.0), pinv(I.nE), q(I.nE), g(I.m, 0.0);
    for (int32_t r = 0; r < I.m; ++r)
      for (int32_t t = I.aptr[r]; t < I.aptr[r + 1]; ++t) atb[I.acol[t]] += I.aval[t] * I.b[r];
    for (int64_t e = 0; e < I.nE; ++e) {
      pinv[e] = 1.0 / (1.0 + 0.5 * I.D[e]);
      q[e] = pinv[e] * (I.c[e] + atb[e]);
    }
    for (int32_t r = 0; r < I.m; ++r)
      for (int32_t t = I.aptr[r]; t < I.aptr[r + 1]; ++t) g[r] += I.aval[t] * q[I.acol[t]];
    I.fac.solve(g);
    std::vector<double> atw(I.nE, 0.0);
    for (int32_t r = 0; r < I.m; ++r)
      for (int32_t t = I.aptr[r]; t < I.aptr[r + 1]; ++t) atw[I.acol[t]] += I.aval[t] * g[r];
    double etphi = 0.0, bb = 0.0;
    for (int64_t e = 0; e < I.nE; ++e) {
      phi[eo + e] = q[e] - pinv[e] * atw[e];
      ev[eo + e] = I.c[e] - atb[e];
      etphi += ev[eo + e] * phi[eo + e];
    }
    for (int32_t r = 0; r < I.m; ++r) {
      aphi[ro + r] = g[r];
      bb += I.b[r] * I.b[r];
    }
    as[(size_t)i * kNas + AS_DEN2] = 1.0 + bb + etphi;
  }
  AdjPlan& a = h->adj;
  a.d = h->d;
  int rc;
  int32_t* zst = nullptr;
  if ((rc = dev_zeros(h, &zst, (size_t)B * kNst))) return rc;
  a.d.st = zst;                          // the adjoint runs on every instance
  if ((rc = dev_upload(h, (double**)&a.phi, phi)) || (rc = dev_upload(h, (double**)&a.ev, ev)) ||
      (rc = dev_upload(h, (double**)&a.aphi, aphi)) || (rc = dev_upload(h, &a.as, as)) ||
      (rc = dev_zeros(h, &a.mu_x, NE)) || (rc = dev_zeros(h, &a.mu_s, h->slot_off[B])) ||
      (rc = dev_zeros(h, &a.mu_y, M)) || (rc = dev_zeros(h, &a.mu_v, h->slot_off[B])) ||
      (rc = dev_zeros(h, &a.mu_t, B)) || (rc = dev_zeros(h, &a.qx, NE)) ||
      (rc = dev_zeros(h, (double**)&a.gx, NE)) || (rc = dev_zeros(h, &a.dc, NE)) || (rc = dev_zeros(h, &a.db, M)))
    return rc;
  std::vector<int64_t> eoff(P);
  int64_t tot = 0;
  for (int32_t i = 0; i < B; ++i)
    for (int32_t k = 0; k < h->inst[i].p; ++k) {
      const int64_t K = h->inst[i].csize[k];
      eoff[h->clq_off[i] + k] = tot;
      tot += K * K + K;
    }
  if ((rc = dev_zeros(h, (double**)&a.eig, tot)) || (rc = dev_upload(h, (int64_t**)&a.eig_off, eoff))) return rc;
  const int64_t NS = h->slot_off[B];
  const int64_t nf = NE + 2 * NS + M + B;
  h->nf = nf;
  std::vector<int64_t> seg((size_t)10 * B);
  std::vector<int32_t> inst_of(nf);
  for (int32_t i = 0; i < B; ++i) {
    const int64_t lo[5] = {h->ent_off[i], NE + h->slot_off[i], NE + NS + h->row_off[i],
                           NE + NS + M + h->slot_off[i], NE + 2 * NS + M + i};
    const int64_t hi[5] = {h->ent_off[i + 1], NE + h->slot_off[i + 1], NE + NS + h->row_off[i + 1],
                           NE + NS + M + h->slot_off[i + 1], NE + 2 * NS + M + i + 1};
    for (int q = 0; q < 5; ++q) {
      seg[10 * i + 2 * q] = lo[q];
      seg[10 * i + 2 * q + 1] = hi[q];
      for (int64_t e = lo[q]; e < hi[q]; ++e) inst_of[e] = i;
    }
  }
  if ((rc = dev_zeros(h, &h->gm_V, (size_t)(kRestart + 1) * nf)) || (rc = dev_zeros(h, &h->gm_w, nf)) ||
      (rc = dev_zeros(h, &h->gm_mu, nf)) || (rc = dev_zeros(h, &h->gm_g, nf)) ||
      (rc = dev_zeros(h, &h->gm_coef, (size_t)(kRestart + 1) * B)) ||
      (rc = dev_zeros(h, &h->gm_dots, (size_t)(kRestart + 1) * B)) || (rc = dev_zeros(h, &h->gm_scale, B)) ||
      (rc = dev_upload(h, &h->gm_seg, seg)) || (rc = dev_upload(h, &h->gm_inst, inst_of)))
    return rc;
  GmState& g = h->gm_state;
  if ((rc = dev_zeros(h, &h->gm_dots2, (size_t)(kRestart + 1) * B)) || (rc = dev_zeros(h, &h->gm_nrm, B)) ||
      (rc = dev_zeros(h, &h->gm_resid, B)) || (rc = dev_zeros(h, &h->gm_reason, B)) ||
      (rc = dev_zeros(h, &h->gm_flags, (size_t)3 * B + 1)) ||
      (rc = dev_zeros(h, &g.H, (size_t)B * (kRestart + 1) * kRestart)) ||
      (rc = dev_zeros(h, &g.cs, (size_t)B * kRestart)) || (rc = dev_zeros(h, &g.sn, (size_t)B * kRestart)) ||
      (rc = dev_zeros(h, &g.gam, (size_t)B * (kRestart + 1))) ||
      (rc = dev_zeros(h, &g.hist, (size_t)B * kGmWindow)) || (rc = dev_zeros(h, &g.gnorm, B)))
    return rc;
  g.jlim = h->gm_flags;
  g.done = h->gm_flags + B;
  g.nhist = h->gm_flags + 2 * B;
  g.alldone = h->gm_flags + 3 * B;
  HIPCHK(hipDeviceSynchronize());
  h->adj_ready = true;
  return 0;
}

}  // namespace

int cdcs_adjoint(cdcs_handle* h, const double* dX, double* dC, double* db, int32_t on_device, int32_t max_iter,
                 double tol, int32_t* iters) {
  if (!h || !dX || max_iter < 1 || !(tol > 0.0)) return set_error(CDCS_E_ARG, "bad adjoint arguments");
  if (h->set.method != CDCS_METHOD_SELF_DUAL)
    return set_error(CDCS_E_ARG, "the adjoint differentiates the self-dual method's fixed point only");
  if (h->max_clique > kAdjMax) return set_error(CDCS_E_ARG, "the adjoint supports cliques of up to 96 vertices");
  const int32_t B = h->B;
  const int64_t NE = h->ent_off[B];
  const int32_t M = h->row_off[B];
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<double> sc((size_t)B * kNsc);
  std::vector<int32_t> stv((size_t)B * kNst);
  HIPCHK(hipMemcpy(sc.data(), h->d.sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(stv.data(), h->d.st, stv.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < B; ++i)
    if (stv[(size_t)i * kNst + ST_STATUS] != CDCS_SOLVED || !(sc[(size_t)i * kNsc + SC_TAU] > 0.0))
      return set_error(CDCS_E_STATE, "instance " + std::to_string(i) + " is not solved");
  int rc = adjoint_prepare(h);
  if (rc) return rc;
  AdjPlan& a = h->adj;
  // g = DPi dL/du with dL/dx = w / tau, dL/dtau = -w^T x / tau^2 (X = x / tau)
  std::vector<double> w(NE), x(NE), gx(NE);
  if (on_device) HIPCHK(hipMemcpy(w.data(), dX, NE * sizeof(double), hipMemcpyDeviceToHost));
  else std::memcpy(w.data(), dX, NE * sizeof(double));
  HIPCHK(hipMemcpy(x.data(), h->d.x, NE * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> as((size_t)B * kNas);
  HIPCHK(hipMemcpy(as.data(), a.as, as.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> mut(B);
  for (int32_t i = 0; i < B; ++i) {
    const double tau = sc[(size_t)i * kNsc + SC_TAU];
    double wx = 0.0;
    for (int64_t e = h->ent_off[i]; e < h->ent_off[i + 1]; ++e) {
      gx[e] = w[e] / tau;
      wx += w[e] * x[e];
    }
    as[(size_t)i * kNas + AS_GT] = -wx / (tau * tau);
    mut[i] = as[(size_t)i * kNas + AS_GT];
  }
  HIPCHK(hipMemcpy(const_cast<double*>(a.gx), gx.data(), NE * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(a.as, as.data(), as.size() * sizeof(double), hipMemcpyHostToDevice));
  // eigenpairs of the clique blocks at the solution
  const int kmaxs[4] = {16, 32, 64, 96};
  for (int bk = 0; bk < 4; ++bk) launch_adj_eig(a, h->adj_tasks[bk], h->adj_ntasks[bk], kmaxs[bk], h->stream);
  const int32_t* tl[4] = {h->adj_tasks[0], h->adj_tasks[1], h->adj_tasks[2], h->adj_tasks[3]};
  const int32_t nt[4] = {h->adj_ntasks[0], h->adj_ntasks[1], h->adj_ntasks[2], h->adj_ntasks[3]};
  hipStream_t st = h->stream;
  const int64_t nf = h->nf;
  const int64_t NS = h->slot_off[B];
  // right-hand side g = DPi dL/du (x block: w/tau, tau block: -w^T x/tau^2), mu = 0
  {
    std::vector<double> gflat(nf, 0.0);
    for (int64_t e = 0; e < NE; ++e) gflat[e] = gx[e];
    for (int32_t i = 0; i < B; ++i) gflat[NE + 2 * NS + M + i] = mut[i];
    HIPCHK(hipMemcpy(h->gm_g, gflat.data(), nf * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemsetAsync(h->gm_mu, 0, nf * sizeof(double), st));
  }
  // w = (I - T'^T) v : one operator application with g switched off leaves
  // v - (I - T'^T) v in w
  auto apply_op = [&](const double* v, double* w) -> int {
    HIPCHK(hipMemcpyAsync(w, v, nf * sizeof(double), hipMemcpyDeviceToDevice, st));
    adj_point(h, w);
    launch_adj_iteration(a, tl, nt, 0, 0, st);
    launch_flat_sub(w, v, w, nf, st);
    return 0;
  };
  // Restarted GMRES(kRestart) on (I - T'^T) mu = g, one Krylov basis per
  // instance, its bookkeeping on the device (k_gm_*): a cycle is a fixed
  // sequence of launches with no host round trip; the host reads one flag
  // per cycle (measured on the 64-SDP differentiated batch: backward 0.366 s
  // with the Hessenberg updates on the host, three round trips per step,
  // 0.273 s this way; capturing a cycle in a graph changed nothing).  The system is singular (the fixed points of the iteration
  // form a cone, not a single ray, when the clique decomposition of Z is not
  // unique) and consistent only up to the forward solve's accuracy, so an
  // instance also stops once its true residual has stalled (less than 10 %
  // reduction over the last 5 restarts).  A stopped instance keeps its mu
  // (zero update coefficients), so batched and single runs follow the same
  // arithmetic.
  GmState gs = h->gm_state;
  double* dots1 = h->gm_dots;
  double* dots2 = h->gm_dots2;
  double* nrm = h->gm_nrm;
  HIPCHK(hipMemsetAsync(h->gm_flags, 0, (size_t)(3 * B + 1) * sizeof(int32_t), st));   // jlim, done, nhist, alldone
  launch_seg_dots(h->gm_g, h->gm_g, nf, 1, h->gm_seg, nrm, B, st);
  launch_flat_sqrt(gs.gnorm, nrm, B, st);
  int32_t it = 0;
  const int32_t one = 1;
  while (it < max_iter) {
    // r = g - A mu into V_0, beta, stopping tests, V_0 = r / beta
    double* V0 = h->gm_V;
    if ((rc = apply_op(h->gm_mu, h->gm_w))) return rc;
    launch_flat_sub(V0, h->gm_g, h->gm_w, nf, st);
    launch_seg_dots(V0, V0, nf, 1, h->gm_seg, nrm, B, st);
    HIPCHK(hipMemcpyAsync(gs.alldone, &one, sizeof(int32_t), hipMemcpyHostToDevice, st));
    launch_gm_begin(gs, nrm, h->gm_scale, B, kRestart, tol, st);
    int32_t alldone = 0;
    HIPCHK(hipMemcpyAsync(&alldone, gs.alldone, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (alldone) break;
    // the rest of the cycle: steps 0..jn-1, then mu += V y with H y = gamma
    // over each instance's columns
    const int jn = std::min<int32_t>(kRestart, max_iter - it);
    launch_flat_scale(V0, V0, h->gm_scale, h->gm_inst, nf, st);
    for (int j = 0; j < jn; ++j) {
      double* Vj = h->gm_V + (size_t)j * nf;
      double* Vn = h->gm_V + (size_t)(j + 1) * nf;
      if ((rc = apply_op(Vj, h->gm_w))) return rc;
      // classical Gram-Schmidt, twice (the dots are the coefficients)
      launch_seg_dots(h->gm_w, h->gm_V, nf, j + 1, h->gm_seg, dots1, B, st);
      launch_flat_axpy_multi(h->gm_w, h->gm_V, nf, j + 1, dots1, h->gm_inst, B, -1.0, st);
      launch_seg_dots(h->gm_w, h->gm_V, nf, j + 1, h->gm_seg, dots2, B, st);
      launch_flat_axpy_multi(h->gm_w, h->gm_V, nf, j + 1, dots2, h->gm_inst, B, -1.0, st);
      launch_seg_dots(h->gm_w, h->gm_w, nf, 1, h->gm_seg, nrm, B, st);
      launch_gm_step(gs, dots1, dots2, nrm, h->gm_scale, B, kRestart, j, tol, st);
      launch_flat_scale(Vn, h->gm_w, h->gm_scale, h->gm_inst, nf, st);
    }
    launch_gm_solve(gs, h->gm_coef, B, kRestart, jn, st);
    launch_flat_axpy_multi(h->gm_mu, h->gm_V, nf, jn, h->gm_coef, h->gm_inst, B, 1.0, st);
    it += jn;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("adjoint launch: ") + hipGetErrorString(e));
  }
  // the final true residual of every instance (one more application)
  {
    double* V0 = h->gm_V;
    if ((rc = apply_op(h->gm_mu, h->gm_w))) return rc;
    launch_flat_sub(V0, h->gm_g, h->gm_w, nf, st);
    launch_seg_dots(V0, V0, nf, 1, h->gm_seg, nrm, B, st);
    launch_gm_final(gs, nrm, h->gm_resid, h->gm_reason, B, tol, st);
    h->adj_resid.assign(B, 0.0);
    h->adj_reason.assign(B, 0);
    HIPCHK(hipMemcpyAsync(h->adj_resid.data(), h->gm_resid, B * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h->adj_reason.data(), h->gm_reason, B * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  // nu = (I - Q)^{-1} mu and the data gradients
  adj_point(h, h->gm_mu);
  launch_adj_iteration(a, tl, nt, 1, 0, h->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("adjoint launch: ") + hipGetErrorString(e));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (iters) *iters = it;
  if (dC) HIPCHK(hipMemcpy(dC, a.dc, NE * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  if (db) HIPCHK(hipMemcpy(db, a.db, M * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return 0;
}

int cdcs_get_adjoint_info(const cdcs_handle* h, double* resid, int32_t* reason) {
  if (!h) return set_error(CDCS_E_ARG, "null handle");
  if (h->adj_resid.empty()) return set_error(CDCS_E_STATE, "no cdcs_adjoint call on this handle yet");
  for (int32_t i = 0; i < h->B; ++i) {
    if (resid) resid[i] = h->adj_resid[i];
    if (reason) reason[i] = h->adj_reason[i];
  }
  return 0;
}

int cdcs_get_tuning(const cdcs_handle* h, int32_t* out, int32_t cap) {
  if (!h || !out || cap < 16) return set_error(CDCS_E_ARG, "cdcs_get_tuning: need a handle and 16 outputs");
  const int kmaxs[4] = {16, 32, 64, 96};   // bucket orders (the last is empty while kJacobiMax = 64)
  for (int b = 0; b < 4; ++b) {
    out[4 * b + 0] = kmaxs[b];
    out[4 * b + 1] = jacobi_threads(kmaxs[b], h->jvar[b]);
    out[4 * b + 2] = h->ntasks[b];
    out[4 * b + 3] = h->jtuned[b];
  }
  return 4;
}

int cdcs_get_phase_times(const cdcs_handle* h, const char** names, double* ms, int64_t* launches, int32_t cap) {
  if (!h) return set_error(CDCS_E_ARG, "null handle");
  for (int i = 0; i < kNumPhases && i < cap; ++i) {
    if (names) names[i] = kPhaseNames[i];
    if (ms) ms[i] = h->phase_ms[i];
    if (launches) launches[i] = h->phase_n[i];
  }
  return kNumPhases;
}

int cdcs_reset_phase_times(cdcs_handle* h) {
  if (!h) return set_error(CDCS_E_ARG, "null handle");
  HIPCHK(hipStreamSynchronize(h->stream));
  harvest_timers(h);
  for (int i = 0; i < kNumPhases; ++i) {
    h->phase_ms[i] = 0.0;
    h->phase_n[i] = 0;
  }
  return 0;
}

int cdcs_psd_project(int32_t count, const int32_t* sizes, const int64_t* offsets, const double* in, double* out,
                     void* stream) {
  if (count < 0 || (count > 0 && (!sizes || !offsets || !in || !out)))
    return set_error(CDCS_E_ARG, "bad projection arguments");
  if (count == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  ProjPlan pl;
  int rc = plan_projection(count, sizes, offsets, &pl);
  if (rc) return rc;
  std::vector<void*> tmp;
  auto up = [&](const void* src, size_t bytes, void** dst) -> int {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return set_error(CDCS_E_NOMEM, "hipMalloc failed");
    tmp.push_back(p);
    if (bytes && src) {
      e = hipMemcpy(p, src, bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) return set_error(CDCS_E_DEVICE, "hipMemcpy failed");
    }
    *dst = p;
    return 0;
  };
  ProjDev dv;
  auto cleanup = [&]() {
    for (void* p : tmp) (void)hipFree(p);
  };
  if ((rc = up(pl.sizes.data(), pl.sizes.size() * 4, (void**)&dv.sizes)) ||
      (rc = up(pl.offs.data(), pl.offs.size() * 8, (void**)&dv.offs))) {
    cleanup();
    return rc;
  }
  for (int b = 0; b < 5; ++b)
    if ((rc = up(pl.bk[b].data(), pl.bk[b].size() * 4, (void**)&dv.tasks[b]))) {
      cleanup();
      return rc;
    }
  if (!pl.bk[4].empty()) {
    if ((rc = up(nullptr, (size_t)pl.wtot * 8, (void**)&dv.work)) ||
        (rc = up(pl.woff.data(), pl.woff.size() * 8, (void**)&dv.woff)) ||
        (rc = up(pl.large_sizes.data(), pl.large_sizes.size() * 4, (void**)&dv.lsz))) {
      cleanup();
      return rc;
    }
    hipLaunchKernelGGL(k_fill_zero, dim3(fill_blocks(pl.wtot)), dim3(256), 0, st, dv.work, pl.wtot);
  }
  launch_projection(pl, dv, in, out, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("projection: ") + hipGetErrorString(e));
  return 0;
}

int cdcs_psd_project_noalloc(int32_t count, const int32_t* sizes, const int64_t* offsets, const double* in,
                             double* out, void* stream) {
  if (count < 0 || (count > 0 && (!sizes || !offsets || !in || !out)))
    return set_error(CDCS_E_ARG, "bad projection arguments");
  if (count == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  ProjPlan pl;
  int rc = plan_projection(count, sizes, offsets, &pl);
  if (rc) return rc;
  // scratch layout: [sizes | offsets | task lists of the 5 buckets | large
  // work offsets | large sizes | (256-byte aligned) large workspace]
  size_t pos = 0;
  auto place = [&](size_t bytes, size_t align) {
    pos = (pos + align - 1) / align * align;
    const size_t at = pos;
    pos += bytes;
    return at;
  };
  const size_t o_sizes = place(pl.sizes.size() * 4, 8);
  const size_t o_offs = place(pl.offs.size() * 8, 8);
  size_t o_tasks[5];
  for (int b = 0; b < 5; ++b) o_tasks[b] = place(pl.bk[b].size() * 4, 8);
  const size_t o_woff = place(pl.woff.size() * 8, 8);
  const size_t o_lsz = place(pl.large_sizes.size() * 4, 8);
  const size_t meta_bytes = pos;
  const size_t o_work = place((size_t)pl.wtot * 8, 256);
  if (pos > kScratchBytes)
    return set_error(CDCS_E_ARG, "projection needs " + std::to_string(pos) +
                                     " bytes of device scratch; cdcs_psd_project_noalloc holds " +
                                     std::to_string(kScratchBytes) + " (use cdcs_psd_project)");
  unsigned char* base = nullptr;
  if ((rc = scratch_base(&base))) return rc;
  // stage the index arrays in one host buffer and copy them in one transfer
  std::vector<unsigned char> meta(meta_bytes);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(meta.data() + at, src, bytes);
  };
  put(o_sizes, pl.sizes.data(), pl.sizes.size() * 4);
  put(o_offs, pl.offs.data(), pl.offs.size() * 8);
  for (int b = 0; b < 5; ++b) put(o_tasks[b], pl.bk[b].data(), pl.bk[b].size() * 4);
  put(o_woff, pl.woff.data(), pl.woff.size() * 8);
  put(o_lsz, pl.large_sizes.data(), pl.large_sizes.size() * 4);
  HIPCHK(hipMemcpyAsync(base, meta.data(), meta_bytes, hipMemcpyHostToDevice, st));
  ProjDev dv;
  dv.sizes = (int32_t*)(base + o_sizes);
  dv.offs = (int64_t*)(base + o_offs);
  for (int b = 0; b < 5; ++b) dv.tasks[b] = (int32_t*)(base + o_tasks[b]);
  if (!pl.bk[4].empty()) {
    dv.woff = (int64_t*)(base + o_woff);
    dv.lsz = (int32_t*)(base + o_lsz);
    dv.work = (double*)(base + o_work);
    // the previous call's workspace contents are still there: start from zeros
    hipLaunchKernelGGL(k_fill_zero, dim3(fill_blocks(pl.wtot)), dim3(256), 0, st, dv.work, pl.wtot);
  }
  launch_projection(pl, dv, in, out, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(CDCS_E_DEVICE, std::string("projection: ") + hipGetErrorString(e));
  return 0;
}

}  // extern "C"

// Host side of the C ABI declared in include/dcax.h.
//
// All kernels are compiled into this one translation unit.  A handle holds a
// batch of walkers (independent Markov chains, possibly of different models
// and orders); every launch covers the whole batch, each kernel picking its
// walker's view by block index.  The host never reads device state inside a
// sweep: orders, window sizes, signs, cursors and counters live in one
// device control block per walker, kernels take their sizes from it, and
// grids are sized by host-side upper bounds.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_ext.h>
#include "dcax_dev.h"
#include "dcax_window.hip"
#include "dcax_refresh.hip"
#include "dcax_measure.hip"
#include "dcax_nfft.hip"
#include "dcax_dca.hip"
#include "dcax_g2.hip"

using namespace dcax;

// Staging for dcax_sweep_replay_static: replayed records, then their ratios,
// for at most DCAX_REPLAY_STATIC_MAX records, in a fixed device array rather
// than memory from the caller's allocator.  Each GPU holds its own copy until
// the process ends.  On the host the array's name is not a device address:
// host code uses the address hipGetSymbolAddress returns on each device.
constexpr size_t STATIC_REC_BYTES = sizeof(dcax_proposal) * (size_t)DCAX_REPLAY_STATIC_MAX;
constexpr size_t STATIC_SCRATCH_BYTES = STATIC_REC_BYTES + sizeof(double) * (size_t)DCAX_REPLAY_STATIC_MAX;
static_assert(STATIC_REC_BYTES % 256 == 0, "the ratios start 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

dcax_status fail(dcax_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) return fail(DCAX_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// Device address of `scratch` on the current device, looked up once per
// device (the walkers of several threads may be created at once).
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

void* static_scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) ptr = nullptr;
  g_scratch_addr[dev] = ptr;
  return ptr;
}

__global__ void k_fill_zero(double* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ------------------------------------------------------------- geometry
// Cluster sites and momenta from the superlattice vectors (enumeration rule
// in include/dcax.h).
struct Geometry {
  int Nc = 0;
  std::vector<int> sites;    // [Nc][2]
  std::vector<double> K;     // [Nc][2]
  std::vector<int> diff;     // [Nc][Nc]
};

bool canonical(long x, long y, const int* c, long& ox, long& oy) {
  const long a1x = c[0], a1y = c[1], a2x = c[2], a2y = c[3];
  const long D = a1x * a2y - a1y * a2x;
  if (D == 0) return false;
  const long ad = D > 0 ? D : -D, s = D > 0 ? 1 : -1;
  const long n0 = a2y * x - a2x * y, n1 = -a1y * x + a1x * y;
  long w0 = (s * n0) % ad, w1 = (s * n1) % ad;
  if (w0 < 0) w0 += ad;
  if (w1 < 0) w1 += ad;
  ox = (a1x * w0 + a2x * w1) / ad;
  oy = (a1y * w0 + a2y * w1) / ad;
  return true;
}

bool build_geometry(const int* c, Geometry& g) {
  const long a1x = c[0], a1y = c[1], a2x = c[2], a2y = c[3];
  const long D = a1x * a2y - a1y * a2x;
  if (D == 0) return false;
  const long ad = D > 0 ? D : -D;
  if (ad > 4096) return false;
  long xs[4] = {0, a1x, a2x, a1x + a2x}, ys[4] = {0, a1y, a2y, a1y + a2y};
  const long x0 = *std::min_element(xs, xs + 4) - 1, x1 = *std::max_element(xs, xs + 4) + 1;
  const long y0 = *std::min_element(ys, ys + 4) - 1, y1 = *std::max_element(ys, ys + 4) + 1;
  std::vector<std::pair<long, long>> reps;  // (y, x)
  for (long y = y0; y <= y1; ++y)
    for (long x = x0; x <= x1; ++x) {
      long ox, oy;
      canonical(x, y, c, ox, oy);
      reps.push_back({oy, ox});
    }
  std::sort(reps.begin(), reps.end());
  reps.erase(std::unique(reps.begin(), reps.end()), reps.end());
  if ((long)reps.size() != ad) return false;
  g.Nc = (int)ad;
  g.sites.resize(2 * ad);
  for (long i = 0; i < ad; ++i) {
    g.sites[2 * i] = (int)reps[i].second;
    g.sites[2 * i + 1] = (int)reps[i].first;
  }
  g.K.clear();
  for (long qy = 0; qy < ad; ++qy)
    for (long qx = 0; qx < ad; ++qx)
      if ((qx * a1x + qy * a1y) % ad == 0 && (qx * a2x + qy * a2y) % ad == 0) {
        g.K.push_back(2.0 * M_PI * (double)qx / (double)ad);
        g.K.push_back(2.0 * M_PI * (double)qy / (double)ad);
      }
  if ((long)g.K.size() != 2 * ad) return false;
  g.diff.resize(ad * ad);
  for (long i = 0; i < ad; ++i)
    for (long j = 0; j < ad; ++j) {
      long ox, oy;
      canonical(g.sites[2 * i] - g.sites[2 * j], g.sites[2 * i + 1] - g.sites[2 * j + 1], c, ox, oy);
      long idx = std::lower_bound(reps.begin(), reps.end(), std::make_pair(oy, ox)) - reps.begin();
      g.diff[i * ad + j] = (int)idx;
    }
  return true;
}

// ------------------------------------------------------------- G0 table
// T[d][l] = (1/Nc) sum_K cos(K . r_d) G0(K, tau_l), G0(K, tau) =
// -e^{-xi tau} / (1 + e^{-beta xi}) (overflow-safe form for xi < 0), with
// tau_l = l (beta / (n_tau - 1)) and the last point at beta.
__global__ void k_g0_table(double* table, int Nc, int n_tau, double beta, const int* sites, const double* K,
                           const double* xi) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int d = blockIdx.y;
  if (l >= n_tau) return;
  const double tau = (l == n_tau - 1) ? beta : (double)l * (beta / (double)(n_tau - 1));
  const double rx = sites[2 * d], ry = sites[2 * d + 1];
  double s = 0.0;
  for (int q = 0; q < Nc; ++q) {
    const double x = xi[q];
    const double g = (x >= 0.0) ? -exp(-x * tau) / (1.0 + exp(-beta * x))
                                : -exp(x * (beta - tau)) / (exp(beta * x) + 1.0);
    s += cos(K[2 * q] * rx + K[2 * q + 1] * ry) * g;
  }
  table[(size_t)d * n_tau + l] = s / (double)Nc;
}

template <typename T>
__global__ void k_set_cursor(const View<T>* __restrict__ vs, long long pos, long long end) {
  Ctl* c = vs[blockIdx.z].ctl;
  c->pos = pos;
  c->end = end;
}

// A sweep is max(k, 1) proposals rounded up to a multiple of k_s, with k the
// order at the sweep's start.
template <typename T>
__device__ void begin_sweep(const View<T>& w, Ctl* c) {
  long long L = c->sweep_len;
  if (L == 0) {
    // warm-up: the length follows the order; the mean order over the second
    // half (which holds at least the last warm-up sweep) becomes the frozen
    // length when the warm-up ends
    L = c->k > 1 ? c->k : 1;
    if (2 * c->n_sweeps >= w.warmup || c->n_sweeps + 1 == w.warmup) {
      c->warm_sum += (double)c->k;
      c->warm_n += 1;
    }
    if (c->n_sweeps + 1 >= w.warmup) {
      const long long mean = llround(c->warm_sum / (double)(c->warm_n > 0 ? c->warm_n : 1));
      c->sweep_len = mean > 1 ? mean : 1;
    }
  }
  c->end = c->pos + ((L + w.ks - 1) / w.ks) * w.ks;
  c->n_sweeps += 1;
}

template <typename T>
__global__ void k_begin_sweep(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  Ctl* c = w.ctl;
  if (c->status != 0) return;
  begin_sweep(w, c);
}

// Device-scheduled sweeps: each walker begins its next sweep as soon as the
// previous one has ended and been measured, independently of the others.
template <typename T>
__global__ void k_set_rounds(const View<T>* __restrict__ vs, long long n) {
  Ctl* c = vs[blockIdx.z].ctl;
  c->sweeps_left = n;
  c->meas_due = 0;
}

// no walker begins another sweep (a running one still ends and is measured)
template <typename T>
__global__ void k_stop_rounds(const View<T>* __restrict__ vs) {
  vs[blockIdx.z].ctl->sweeps_left = 0;
}

template <typename T>
__global__ void k_round_begin(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  Ctl* c = w.ctl;
  if (c->status != 0 || c->pos < c->end || c->meas_due || c->sweeps_left <= 0) return;
  begin_sweep(w, c);
  c->sweeps_left -= 1;
  c->meas_due = 1;
}

// closes the gated measurement of the walkers it covered
template <typename T>
__global__ void k_meas_done(const View<T>* __restrict__ vs) {
  Ctl* c = vs[blockIdx.z].ctl;
  if (!meas_skip(c, 1)) c->meas_due = 0;
}

template <typename T>
__global__ void k_refresh_begin(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  w.detsign[0] = 1.0;
  w.detsign[1] = 1.0;
  w.ctl->drift = 0.0;
  w.ctl->k_ref = w.ctl->k;
  w.ctl->hold = 0;         // a walker held by the drift control is released
}

// After dcax_set_config's refresh: the sign of the configuration is the sign
// of prod_sigma det N_sigma^{-1}, read off the Gauss-Jordan pivots.
template <typename T>
__global__ void k_set_sign(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  w.ctl->sign = w.detsign[0] * w.detsign[1];
}

}  // namespace

// One Markov chain of the batch.
struct WalkerHost {
  dcax_params p{};            // host pointers g0_tau / g0_Kw are cleared after creation
  bool has_g0Kw = false;
  Geometry geo;
  int ks = 0, cap = 0, ld = 0, max_order = 0, kpad_cap = 0;
  double gamma = 0.0;
  long long acc_off = 0;
  int nc_prefix = 0;
  bool latched = false;
  int k_host = 0;
  View<double> v64{};
  View<float> v32{};
};

struct dcax_walker_s {
  int W = 0;
  bool mixed = false;
  // two-particle measurement scratch (dcax_measure_G2), grown on demand
  G2Dev g2{};
  size_t g2_kpad = 0, g2_nw = 0, g2_nc = 0;
  int* g2_q = nullptr;          // [G2_Q_MAX] transfer momenta
  int* g2_dK = nullptr;         // [Nc][Nc] index of K_a - K_b
  int g2_dK_nc = 0;
  // probes of N against its definition (dcax_probe_N, drift_tol)
  double* probe_d = nullptr;   // [2 W] largest residual per walker and spin
  // work list of a measurement launch: [1 + W] count and walkers, [W + 1] item prefix sums
  int* meas_list_d = nullptr;
  long long* meas_pre_d = nullptr;
  long long probes = 0, probe_refreshes = 0;
  double last_probe = 0.0;
  long long held_since = -1;   // round at which the drift control first held a walker still held
  dcax_allocator alloc{};
  hipStream_t stream = nullptr;
  std::vector<WalkerHost> wk;
  std::vector<void*> blocks;
  Ctl* ctl_all = nullptr;      // [W] control blocks, contiguous
  std::vector<Ctl> h_ctl;      // host copy after the last synchronisation
  void* d_views = nullptr;     // [W] View<T> on the device
  // views of the walkers a partial rebuild covers (the drift control's), so
  // that its launches span only those walkers
  void* d_views_sel = nullptr; // [W] View<T>
  std::vector<char> views_sel_host;
  int ks_max = 0, cap_max = 0, nc_max = 0, nf_max = 0, kpad_max = 0, mo_max = 0;
  long long acc_total = 0;
  int nc_total = 0;
  // replay (single-walker handles)
  dcax_proposal* replay_d = nullptr;
  double* ratio_d = nullptr;
  long long replay_cap = 0;
  // the static staging of this walker's GPU (dcax_sweep_replay_static), and
  // the record buffer the device views currently point at
  void* static_scratch = nullptr;
  const dcax_proposal* views_replay = nullptr;
  long long sweeps_done = 0;
  double last_drift = 0.0, max_drift = 0.0;
  // sweeps replayed as hipGraphs (dcax_set_graphs).  Events recorded inside
  // a captured graph cannot be timed on this runtime (hipEventElapsedTime
  // rejects them), so a replayed sweep is timed as a whole from events
  // around its launch, and per-kernel times come from eager sweeps.
  bool use_graphs = false;
  int cand_variant = DCAX_VARIANT_AUTO, y_variant = DCAX_VARIANT_AUTO;   // dcax_set_variants
  hipStream_t gstream = nullptr;         // library stream the graphs run on
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  // rounds of device-scheduled sweeps, keyed by (order bound, windows,
  // delayed-NFFT half-width, accumulator, aux)
  std::map<std::tuple<int, int, int, double*, double*>, hipGraphExec_t> round_graphs;
  bool capturing = false;
  // the host copies of the control blocks match the device (nothing that
  // changes a walker has been enqueued since the last sync_all)
  bool fresh = false;
  long long rounds_done = 0;   // rounds of device-scheduled sweeps
  // live kernel timing (dcax_set_timing): every timing_every-th window
  bool timing = false;
  int timing_every = 1;
  long long win_seq = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pend_fold, pend_accept, pend_window, pend_cand, pend_y;
  double fold_s = 0.0, accept_s = 0.0, window_s = 0.0, cand_s = 0.0, y_s = 0.0;
  long long fold_launches = 0;

  // all device memory comes from the caller's allocator
  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    void* ptr = alloc.alloc(bytes, alloc.ctx);
    if (ptr) blocks.push_back(ptr);
    return ptr;
  }
  // drops every captured sweep graph (their launch shapes or events are stale)
  void clear_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    for (auto& kv : round_graphs) (void)hipGraphExecDestroy(kv.second);
    round_graphs.clear();
  }
  void release() {
    clear_graphs();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
    ev_in = ev_out = nullptr;
    gstream = nullptr;
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
    for (void* b : blocks) alloc.free(b, alloc.ctx);
    blocks.clear();
  }
  hipEvent_t ev() {
    hipEvent_t e = nullptr;
    if (!ev_pool.empty()) {
      e = ev_pool.back();
      ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  // called after the stream has been synchronised
  void drain_events() {
    auto drain = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& acc, long long* n) {
      for (auto& pr : v) {
        float ms = 0.f;
        if (pr.first && pr.second && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) acc += ms * 1e-3;
        if (n) ++*n;
        if (pr.first) ev_pool.push_back(pr.first);
        if (pr.second) ev_pool.push_back(pr.second);
      }
      v.clear();
    };
    drain(pend_fold, fold_s, &fold_launches);
    drain(pend_accept, accept_s, nullptr);
    drain(pend_window, window_s, nullptr);
    drain(pend_cand, cand_s, nullptr);
    drain(pend_y, y_s, nullptr);
  }
  void mark(std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, hipEvent_t a, hipEvent_t b) {
    if (timing && a && b) v.push_back({a, b});
  }
  // An event for a timed launch: attached to the kernel's own dispatch
  // (hipExtLaunchKernelGGL) rather than recorded as a separate stream
  // command, which would idle the queue between kernels.
  hipEvent_t tev(bool timed) { return timed ? ev() : nullptr; }
  // whether the next window is timed: a pseudo-random 1/timing_every share
  // (a fixed stride would always pick the same window of a sweep)
  bool timed_window() {
    if (!timing || capturing) return false;
    ++win_seq;
    if (timing_every == 1) return true;
    unsigned long long x = (unsigned long long)win_seq * 0x9E3779B97F4A7C15ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    return x % (unsigned long long)timing_every == 0;
  }
  template <typename T>
  const View<T>* views(int first = 0) const {
    return (const View<T>*)d_views + first;
  }
  int kmax_host() const {
    int k = 0;
    for (const auto& x : wk) k = std::max(k, x.k_host);
    return k;
  }
};

namespace {

template <typename T>
View<T>& hview(WalkerHost& x);
template <>
View<double>& hview<double>(WalkerHost& x) { return x.v64; }
template <>
View<float>& hview<float>(WalkerHost& x) { return x.v32; }

dcax_status validate(const dcax_params* p) {
  if (!p) return fail(DCAX_E_INVAL, "params is NULL");
  if (p->abi_version != DCAX_ABI_VERSION) return fail(DCAX_E_INVAL, "abi_version mismatch");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(DCAX_E_INVAL, "beta must be positive");
  if (!(p->U >= 0.0) || !std::isfinite(p->U)) return fail(DCAX_E_INVAL, "U must be >= 0");
  if (!(p->K_exp > 0.0) || !std::isfinite(p->K_exp)) return fail(DCAX_E_INVAL, "K_exp must be positive");
  if (!std::isfinite(p->t) || !std::isfinite(p->tp) || !std::isfinite(p->mu))
    return fail(DCAX_E_INVAL, "non-finite hopping or mu");
  if (p->n_tau < 2 || p->n_tau > (1 << 22)) return fail(DCAX_E_INVAL, "n_tau out of range");
  if (p->precision != DCAX_FP64 && p->precision != DCAX_FP32_MIXED) return fail(DCAX_E_INVAL, "unknown precision");
  if (p->submatrix_k < 1 || p->submatrix_k > KS_MAX) return fail(DCAX_E_INVAL, "submatrix_k must be in 1..64");
  if (p->refresh_every < 0) return fail(DCAX_E_INVAL, "refresh_every must be >= 0");
  if (p->max_order < 1 || p->max_order > 32768) return fail(DCAX_E_INVAL, "max_order must be in 1..32768");
  if (p->n_freq < 0 || p->n_freq > 65536) return fail(DCAX_E_INVAL, "n_freq out of range");
  if (p->warmup_sweeps < 0) return fail(DCAX_E_INVAL, "warmup_sweeps must be >= 0");
  if (p->sweep_length < 0) return fail(DCAX_E_INVAL, "sweep_length must be >= 0");
  if (p->n_spin_tables < 0 || p->n_spin_tables > 2) return fail(DCAX_E_INVAL, "n_spin_tables must be 0, 1 or 2");
  if (p->n_spin_tables > 0 && !p->g0_tau) return fail(DCAX_E_INVAL, "n_spin_tables > 0 needs g0_tau");
  if (p->n_spin_tables == 0 && (p->g0_tau || p->g0_Kw)) return fail(DCAX_E_INVAL, "g0_tau or g0_Kw given with n_spin_tables = 0");
  if (p->reserved != 0 || p->reserved2 != 0) return fail(DCAX_E_INVAL, "reserved fields must be 0");
  if (!(p->flip_share >= 0.0 && p->flip_share < 1.0)) return fail(DCAX_E_INVAL, "flip_share must be in [0, 1)");
  if (p->touched_twice != 0 && p->touched_twice != 1) return fail(DCAX_E_INVAL, "touched_twice must be 0 or 1");
  if (!(p->drift_tol >= 0.0) || !std::isfinite(p->drift_tol)) return fail(DCAX_E_INVAL, "drift_tol must be finite and >= 0");
  Geometry g;
  if (!build_geometry(p->cluster, g)) return fail(DCAX_E_INVAL, "degenerate or too large cluster");
  if (p->n_freq > 0 && g.Nc > MEAS_NC_MAX)
    return fail(DCAX_E_INVAL, "the measurement supports clusters of at most 256 sites");
  return DCAX_OK;
}

dcax_status check_latched(dcax_walker w) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  for (const auto& x : w->wk)
    if (x.latched) return fail(DCAX_E_STATE, "a walker holds a latched error; call dcax_set_config on it");
  return DCAX_OK;
}

// Copies every control block to the host and checks the latched statuses.
dcax_status sync_all(dcax_walker w) {
  HIPCHK(hipMemcpyAsync(w->h_ctl.data(), w->ctl_all, sizeof(Ctl) * w->W, hipMemcpyDeviceToHost, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  w->drain_events();
  dcax_status st = DCAX_OK;
  for (int i = 0; i < w->W; ++i) {
    const Ctl& h = w->h_ctl[i];
    w->wk[i].k_host = h.k;
    if (h.status != ST_OK && st == DCAX_OK) {
      w->wk[i].latched = true;
      switch (h.status) {
        case ST_NUMERIC: st = fail(DCAX_E_NUMERIC, "non-finite ratio or zero pivot (walker " + std::to_string(i) + ")"); break;
        case ST_CAPACITY: st = fail(DCAX_E_CAPACITY, "expansion order would exceed max_order (walker " + std::to_string(i) + ")"); break;
        case ST_TRACE: st = fail(DCAX_E_TRACE, "replay names a vertex id that is not present"); break;
        default: st = fail(DCAX_E_NUMERIC, "latched device error"); break;
      }
    } else if (h.status != ST_OK) {
      w->wk[i].latched = true;
    }
  }
  w->fresh = true;
  return st;
}

// Workgroups per walker and spin along a kernel's tile dimension.  The
// kernels stride over their tiles by the device-side order, so any count
// covers the work; the tiles of one walker are latency-bound chains, so a
// launch keeps all of them in flight (idle workgroups of small walkers cost
// little) up to a ceiling on the launch size.
static int spread(int tiles, int W, int units, long long budget = 1ll << 21) {
  const long long g = std::max<long long>(1, budget / ((long long)W * units));
  return (int)std::max<long long>(1, std::min<long long>(tiles, g));
}
// Gated measurements cover the few walkers whose sweep has just ended: a
// launch sized for every walker would spend its time dispatching workgroups
// that return at once, so the measurement grids stay within this budget.
constexpr long long MEAS_BUDGET = 1ll << 15;
// workgroups of the persistent measurement contraction (8 per compute unit)
constexpr long long MEAS_BLOCKS = 2048;
// orders from which a single walker's device-scheduled rounds carry spare
// windows (below it an empty window's ~10 launches are a visible share of a
// full one)
constexpr int SPARE_MIN_ORDER = 512;

template <typename T>
void enqueue_window(dcax_walker w, int kb, bool replay) {
  w->fresh = false;
  const bool timed = w->timed_window();
  const View<T>* vs = w->views<T>();
  hipStream_t s = w->stream;
  const int W = w->W;
  const int ks = w->ks_max;
  const int kx = std::min(kb + ks, w->cap_max);
  const int kb1 = std::max(kb, 1);
  hipEvent_t e_w0 = w->tev(timed);
  if (replay) hipExtLaunchKernelGGL(k_prep_replay<T>, dim3(1, 1, W), dim3(WG), 0, s, e_w0, nullptr, 0, vs);
  else hipExtLaunchKernelGGL(k_prep_rng<T>, dim3(1, 1, W), dim3(PW), 0, s, e_w0, nullptr, 0, vs);
  const int ne = std::min(2 * ks, KS_MAX);   // elements: candidates, targets, second attempts
  const int gx = spread(cdiv(kb1, WG), W, 1);
  hipLaunchKernelGGL(k_gather<T>, dim3(gx, spread(ne, W, gx), W), dim3(WG), 0, s, vs);
  // Candidate rows: 16 wavefronts per workgroup for few workgroups and for
  // large orders (long column segments per workgroup stream best), 4 for
  // large batches of small walkers.  Y columns: 8 wavefronts while the row
  // tiles are few; in FP64, from a few hundred tiles on (a single walker of
  // order ~5000) the 4-wavefront form streams N faster, in FP32 only from
  // the batch bound on.
  // With many workgroups (batches) the FP32 products run on 64-wide tiles of
  // N staged in LDS, whose small operand is then read once per 64 columns or
  // rows (measured on 32 walkers of order 6000: 7.5 -> 4.8 ms and 5.6 ->
  // 4.2 ms per launch; in FP64 the split-inner-dimension forms stay faster,
  // 8.0 and 8.4 ms against 13.5 and 12.8 ms).
  const int g16 = spread(cdiv(kb1, 16), W, 2);
  const int g64 = spread(cdiv(kb1, 64), W, 2);
  const bool big = sizeof(T) == 4 && (long long)g64 * 2 * W >= 1024;
  const int cv = w->cand_variant != DCAX_VARIANT_AUTO ? w->cand_variant
      : big ? DCAX_VARIANT_TILED : ((long long)g16 * 2 * W < 4096 || kb1 >= 1024) ? DCAX_VARIANT_WIDE
      : DCAX_VARIANT_NARROW;
  const int yv = w->y_variant != DCAX_VARIANT_AUTO ? w->y_variant
      : big ? DCAX_VARIANT_TILED : ((long long)g16 * 2 * W < (sizeof(T) == 8 ? 512 : 4096)) ? DCAX_VARIANT_WIDE
      : DCAX_VARIANT_NARROW;
  const bool tiled = cv == DCAX_VARIANT_TILED, wide = cv == DCAX_VARIANT_WIDE;
  hipEvent_t e_c0 = w->tev(timed), e_c1 = w->tev(timed);
  if (tiled) hipExtLaunchKernelGGL(k_cand_xt<T>, dim3(g64, 2, W), dim3(256), 0, s, e_c0, e_c1, 0, vs);
  else if (wide) hipExtLaunchKernelGGL((k_cand_x<T, 16>), dim3(g16, 2, W), dim3(1024), 0, s, e_c0, e_c1, 0, vs);
  else hipExtLaunchKernelGGL((k_cand_x<T, 4>), dim3(g16, 2, W), dim3(256), 0, s, e_c0, e_c1, 0, vs);
  w->mark(w->pend_cand, e_c0, e_c1);
  // Gram: a workgroup per row for few walkers, the matrix-core form for
  // batches (a workgroup per 16 candidates)
  if ((long long)ne * 2 * W < 4096) hipLaunchKernelGGL((k_gram_rows<T, 16>), dim3(ne, 2, W), dim3(1024), 0, s, vs);
  else hipLaunchKernelGGL((k_gram<T, 4>), dim3(cdiv(ks, 16), 2, W), dim3(256), 0, s, vs);
  hipEvent_t e_a0 = w->tev(timed), e_a1 = w->tev(timed);
  hipExtLaunchKernelGGL(k_accept<T>, dim3(1, 1, W), dim3(AW), 0, s, e_a0, e_a1, 0, vs);
  w->mark(w->pend_accept, e_a0, e_a1);
  hipEvent_t e_y0 = w->tev(timed), e_y1 = w->tev(timed);
  if (yv == DCAX_VARIANT_TILED) hipExtLaunchKernelGGL(k_ygemm_t<T>, dim3(g64, 2, W), dim3(256), 0, s, e_y0, e_y1, 0, vs);
  else if (yv == DCAX_VARIANT_WIDE) hipExtLaunchKernelGGL((k_ygemm<T, 8>), dim3(g16, 2, W), dim3(512), 0, s, e_y0, e_y1, 0, vs);
  else hipExtLaunchKernelGGL((k_ygemm<T, 4>), dim3(g16, 2, W), dim3(256), 0, s, e_y0, e_y1, 0, vs);
  w->mark(w->pend_y, e_y0, e_y1);
  hipLaunchKernelGGL(k_fold_prep<T>, dim3(spread(cdiv(kx, 64), W, 2), 2, W), dim3(WG), 0, s, vs);
  hipEvent_t e_f0 = w->tev(timed), e_f1 = w->tev(timed);
  const int ft = cdiv(kx, 64);
  hipExtLaunchKernelGGL(k_fold<T>, dim3(spread(ft * ft, W, 2), 1, 2 * W), dim3(WG), 0, s, e_f0, e_f1, 0, vs);
  w->mark(w->pend_fold, e_f0, e_f1);
  hipEvent_t e_w1 = w->tev(timed);
  hipExtLaunchKernelGGL(k_compact_move<T>, dim3(spread(cdiv(kx, WG), W, 2), 1, 2 * W), dim3(WG), 0, s, nullptr, e_w1,
                        0, vs);
  w->mark(w->pend_window, e_w0, e_w1);
}

// FP64 refresh of N for walkers [first, first + n); nothing is read back.
template <typename T>
void enqueue_refresh_vs(dcax_walker w, const View<T>* vs, int n, int kmax, bool measure) {
  w->fresh = false;
  hipStream_t s = w->stream;
  hipLaunchKernelGGL(k_refresh_begin<T>, dim3(1, 1, n), dim3(1), 0, s, vs);
  if (kmax == 0) return;
  hipLaunchKernelGGL(k_build_ninv<T>, dim3(cdiv(kmax, WG), kmax, n), dim3(WG), 0, s, vs);
  // panel width: see dcax_refresh.hip (wide panels pay off from three
  // rebuilt walkers on)
  const bool one = kmax <= PANEL_ROWS;
  const int pw = (one || n < 3) ? NB_ONE : NB;
  for (int p0 = 0; p0 < kmax; p0 += pw) {
    if (one)
      hipLaunchKernelGGL(k_gj_panel<T>, dim3(2, 1, n), dim3(cdiv(kmax, 64) * 64), 0, s, vs, p0);
    else if (pw == NB)
      for (int c = 0; c <= std::min(NB, kmax - p0); ++c)
        hipLaunchKernelGGL((k_gj_col<T, NB>), dim3(cdiv(kmax, WG), 2, n), dim3(WG), 0, s, vs, p0, c);
    else
      for (int c = 0; c <= std::min(NB_ONE, kmax - p0); ++c)
        hipLaunchKernelGGL((k_gj_col<T, NB_ONE>), dim3(cdiv(kmax, WG), 2, n), dim3(WG), 0, s, vs, p0, c);
    hipLaunchKernelGGL(k_gj_prep<T>, dim3(cdiv(kmax, WG), 2, n), dim3(WG), 0, s, vs, p0, pw);
    hipLaunchKernelGGL(k_gj_update<T>, dim3(cdiv(kmax, 64), cdiv(kmax, 64), 2 * n), dim3(WG), 0, s, vs, p0, pw);
  }
  hipLaunchKernelGGL(k_gj_perm<T>, dim3(2, 1, n), dim3(64), 0, s, vs);
  hipLaunchKernelGGL(k_refresh_store<T>, dim3(cdiv(kmax, WG), kmax, 2 * n), dim3(WG), 0, s, vs, measure ? 1 : 0);
  if (measure) hipLaunchKernelGGL(k_drift<T>, dim3(1, 1, n), dim3(WG), 0, s, vs);
}

template <typename T>
void enqueue_refresh(dcax_walker w, int first, int n, int kmax, bool measure) {
  enqueue_refresh_vs<T>(w, w->views<T>(first), n, kmax, measure);
}

// FP64 rebuild of the listed walkers only: their views are copied into a
// separate array, so every launch of the sequence spans just them (a masked
// sequence over the whole batch would dispatch mostly idle workgroups).
template <typename T>
void enqueue_refresh_some(dcax_walker w, const std::vector<int>& idx, int kmax) {
  const int n = (int)idx.size();
  if (n == 0) return;
  w->views_sel_host.resize(sizeof(View<T>) * n);
  View<T>* h = (View<T>*)w->views_sel_host.data();
  for (int j = 0; j < n; ++j) h[j] = hview<T>(w->wk[idx[j]]);
  (void)hipMemcpyAsync(w->d_views_sel, h, sizeof(View<T>) * n, hipMemcpyHostToDevice, w->stream);
  enqueue_refresh_vs<T>(w, (const View<T>*)w->d_views_sel, n, kmax, true);
}

dcax_status refresh_all(dcax_walker w, double* drift) {
  dcax_status st = sync_all(w);
  if (st != DCAX_OK) return st;
  const int kmax = w->kmax_host();
  if (w->mixed) enqueue_refresh<float>(w, 0, w->W, kmax, true);
  else enqueue_refresh<double>(w, 0, w->W, kmax, true);
  HIPCHK(hipGetLastError());
  st = sync_all(w);
  if (st != DCAX_OK) return st;
  double d = 0.0;
  for (const Ctl& h : w->h_ctl) d = std::max(d, h.drift);
  if (drift) *drift = d;
  return DCAX_OK;
}

// Largest sampled residual of N against N^{-1} = e^V - g (e^V - 1) per
// walker (k_probe), into res[W]; synchronises.
dcax_status probe_all(dcax_walker w, std::vector<double>& res) {
  const unsigned long long salt = 0x9E3779B97F4A7C15ULL * (unsigned long long)(++w->probes) ^ w->wk[0].p.seed;
  if (w->mixed)
    hipLaunchKernelGGL(k_probe<float>, dim3(1, 2, w->W), dim3(WG), 0, w->stream, w->views<float>(), salt, w->probe_d,
                       0.0);
  else
    hipLaunchKernelGGL(k_probe<double>, dim3(1, 2, w->W), dim3(WG), 0, w->stream, w->views<double>(), salt,
                       w->probe_d, 0.0);
  HIPCHK(hipGetLastError());
  std::vector<double> h(2 * w->W);
  HIPCHK(hipMemcpyAsync(h.data(), w->probe_d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  res.assign(w->W, 0.0);
  double m = 0.0;
  for (int i = 0; i < w->W; ++i) {
    const double a = h[2 * i], b = h[2 * i + 1];
    res[i] = (a != a || b != b) ? a + b : std::max(a, b);
    m = (res[i] != res[i] || res[i] > m) ? res[i] : m;
  }
  w->last_probe = m;
  return DCAX_OK;
}

// The drift control of drift_tol (walker 0's parameter): probe every walker
// and rebuild N in FP64 for those whose residual exceeds the tolerance.
dcax_status probe_and_refresh(dcax_walker w) {
  const double tol = w->wk[0].p.drift_tol;
  if (!(tol > 0.0)) return DCAX_OK;
  dcax_status st = sync_all(w);
  if (st != DCAX_OK) return st;
  std::vector<double> res;
  st = probe_all(w, res);
  if (st != DCAX_OK) return st;
  int nflag = 0, kflag = 0;
  std::vector<int> flag(w->W, 0), idx;
  for (int i = 0; i < w->W; ++i)
    if (!(res[i] <= tol)) {
      flag[i] = 1;
      ++nflag;
      idx.push_back(i);
      kflag = std::max(kflag, w->wk[i].k_host);
    }
  if (nflag == 0) return DCAX_OK;
  w->probe_refreshes += nflag;
  // one refresh launch sequence over the flagged walkers only (its column
  // steps are launch-latency-bound, so it costs about what one walker's does)
  if (w->mixed) enqueue_refresh_some<float>(w, idx, kflag);
  else enqueue_refresh_some<double>(w, idx, kflag);
  HIPCHK(hipGetLastError());
  w->fresh = false;
  st = sync_all(w);
  if (st != DCAX_OK) return st;
  for (int i = 0; i < w->W; ++i)
    if (flag[i]) w->max_drift = std::max(w->max_drift, w->h_ctl[i].drift);
  return DCAX_OK;
}

// The work list of a measurement launch and the site-sorted copy of M.
template <typename T>
void enqueue_sorted_copy(dcax_walker w, int gated) {
  const View<T>* vs = w->views<T>();
  hipStream_t s = w->stream;
  const int W = w->W;
  const int kb1 = std::max(std::min(w->kpad_max, w->kmax_host() + 16 * w->nc_max), 1);
  hipLaunchKernelGGL(k_meas_sort<T>, dim3(1, 1, W), dim3(WG), 0, s, vs, gated);
  hipLaunchKernelGGL(k_meas_list<T>, dim3(1), dim3(64), 0, s, vs, W, gated, w->meas_list_d, w->meas_pre_d);
  if (kb1 <= MCOPY_ROWS) {      // every walker's padded order fits the LDS column
    hipLaunchKernelGGL(k_meas_copy<T>, dim3(std::min(kb1, 1024), W), dim3(WG), 0, s, vs, w->meas_list_d);
  } else {
    const long long mb = MEAS_BUDGET;
    const int cx = spread(cdiv(kb1, WG), W, 1, mb);
    hipLaunchKernelGGL(k_meas_copy_wide<T>, dim3(cx, spread(cdiv(kb1, MCOLS), W, cx, mb), W), dim3(WG), 0, s, vs,
                       gated);
  }
}

template <typename T>
void enqueue_measure(dcax_walker w, double* acc, double* aux, int gated) {
  const View<T>* vs = w->views<T>();
  hipStream_t s = w->stream;
  const int W = w->W;
  hipLaunchKernelGGL(k_meas_diag<T>, dim3(2, 1, W), dim3(WG), 0, s, vs, aux, gated);
  const int nf = w->nf_max;
  if (nf == 0) {
    if (gated) hipLaunchKernelGGL(k_meas_done<T>, dim3(1, 1, W), dim3(1), 0, s, vs);
    return;
  }
  const int ncm = w->nc_max;
  const int kb = std::min(w->kpad_max, w->kmax_host() + 16 * ncm);
  const int kb1 = std::max(kb, 1);
  enqueue_sorted_copy<T>(w, gated);
  const long long mb = MEAS_BUDGET;
  const int px = cdiv(nf, WG);
  hipLaunchKernelGGL(k_meas_phase<T>, dim3(px, spread(cdiv(kb1, MCOLS), W, px, mb), W), dim3(WG), 0, s, vs, gated);
  // the contraction: a persistent grid over the work items of the walkers
  // this launch covers, listed on the device
  long long items = 0;
  for (const auto& x : w->wk) items += meas_items(x.geo.Nc, x.p.n_freq);
  const int nbk = (int)std::min<long long>(MEAS_BLOCKS, (std::max(1ll, (items + WG / 64 - 1) / (WG / 64)) + XCDS - 1) / XCDS * XCDS);
  hipLaunchKernelGGL(k_meas_block<T>, dim3(nbk), dim3(WG), 0, s, vs, w->meas_list_d, w->meas_pre_d);
  hipLaunchKernelGGL(k_meas_K<T>, dim3(px, spread(ncm, W, 2 * px, mb), 2 * W), dim3(WG), 0, s, vs, acc, gated);
  if (gated) hipLaunchKernelGGL(k_meas_done<T>, dim3(1, 1, W), dim3(1), 0, s, vs);
}

// Checks shared by the delayed-NFFT entry points.
dcax_status nfft_check(dcax_walker w, int32_t half_width) {
  if (half_width < 2 || half_width > NFFT_MSP_MAX) return fail(DCAX_E_INVAL, "half_width must be in [2, 16]");
  for (const auto& x : w->wk) {
    const int nf = x.p.n_freq;
    if (nf < 1) return fail(DCAX_E_INVAL, "the NFFT measurement needs n_freq >= 1");
    if (4 * nf > NFFT_L_MAX) return fail(DCAX_E_INVAL, "the NFFT grid holds at most 2048 frequencies");
    if (2 * half_width > 4 * nf) return fail(DCAX_E_INVAL, "half_width wider than the grid");
  }
  return DCAX_OK;
}

// The delayed-NFFT measurement: aux terms, the site sort and sorted copy of M
// shared with the direct measurement, then the gridding.  gated: only the
// walkers whose sweep has ended (device-scheduled sweeps).
template <typename T>
void enqueue_nfft(dcax_walker w, int half_width, double* grid, double* aux, int gated) {
  const View<T>* vs = w->views<T>();
  hipStream_t s = w->stream;
  const int W = w->W;
  hipLaunchKernelGGL(k_meas_diag<T>, dim3(2, 1, W), dim3(WG), 0, s, vs, aux, gated);
  const int ncm = w->nc_max;
  const int kb = std::min(w->kpad_max, w->kmax_host() + 16 * ncm);
  const int kb1 = std::max(kb, 1);
  enqueue_sorted_copy<T>(w, gated);
  // rows split over groups of sites until the launch has ~1024 workgroups
  const int groups = (int)std::max<long long>(1, std::min<long long>(ncm, 1024 / (2ll * ncm * W)));
  const size_t lds = sizeof(double) * 4 * (size_t)w->nf_max;
  hipLaunchKernelGGL(k_nfft_grid<T>, dim3(ncm * groups, 2, W), dim3(WG), lds, s, vs, half_width, groups, grid,
                     gated);
  if (gated) hipLaunchKernelGGL(k_meas_done<T>, dim3(1, 1, W), dim3(1), 0, s, vs);
}

// One sweep's kernels (sweep start plus nwin windows with growing bounds).
void enqueue_sweep(dcax_walker w, int kb, int nwin) {
  w->fresh = false;
  if (w->mixed) hipLaunchKernelGGL(k_begin_sweep<float>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<float>());
  else hipLaunchKernelGGL(k_begin_sweep<double>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<double>());
  for (int i = 0; i < nwin; ++i) {
    kb = std::min(w->mo_max, kb + w->ks_max);
    if (w->mixed) enqueue_window<float>(w, kb, false);
    else enqueue_window<double>(w, kb, false);
  }
}

// Captures what `enqueue` puts on the walker's stream as a graph on the
// library's own stream.
template <typename F>
dcax_status capture_graph(dcax_walker w, F enqueue, hipGraphExec_t* exec) {
  if (!w->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&w->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming));
  }
  hipStream_t user = w->stream;
  HIPCHK(hipStreamBeginCapture(w->gstream, hipStreamCaptureModeThreadLocal));
  w->stream = w->gstream;
  w->capturing = true;
  enqueue();
  w->capturing = false;
  w->stream = user;
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamEndCapture(w->gstream, &graph));
  const hipError_t ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ie);
  return DCAX_OK;
}

// Launches a captured graph on the library's stream, ordered after and
// before the caller's stream by events (timed as a whole when timing is on).
dcax_status launch_graph(dcax_walker w, hipGraphExec_t exec) {
  HIPCHK(hipEventRecord(w->ev_in, w->stream));
  HIPCHK(hipStreamWaitEvent(w->gstream, w->ev_in, 0));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (w->timing) {
    t0 = w->ev();
    if (t0) HIPCHK(hipEventRecord(t0, w->gstream));
  }
  HIPCHK(hipGraphLaunch(exec, w->gstream));
  if (w->timing) {
    t1 = w->ev();
    if (t1) HIPCHK(hipEventRecord(t1, w->gstream));
    w->mark(w->pend_window, t0, t1);
  }
  HIPCHK(hipEventRecord(w->ev_out, w->gstream));
  HIPCHK(hipStreamWaitEvent(w->stream, w->ev_out, 0));
  return DCAX_OK;
}

// Replays the sweep as a hipGraph captured once per (order bound, window
// count).
dcax_status launch_sweep_graph(dcax_walker w, int kb, int nwin) {
  w->fresh = false;
  const int kq = std::min(w->mo_max, ((kb + 63) / 64) * 64);
  const auto key = std::make_pair(kq, nwin);
  auto it = w->graphs.find(key);
  if (it == w->graphs.end()) {
    hipGraphExec_t exec = nullptr;
    dcax_status st = capture_graph(w, [&] { enqueue_sweep(w, kq, nwin); }, &exec);
    if (st != DCAX_OK) return st;
    it = w->graphs.emplace(key, exec).first;
  }
  return launch_graph(w, it->second);
}

dcax_status sweep_rng(dcax_walker w, int n_sweeps) {
  // every call that changes a walker ends with a sync; only work that leaves
  // the walkers alone (a measurement) may be in flight here
  dcax_status st = DCAX_OK;
  if (!w->fresh) {
    st = sync_all(w);
    if (st != DCAX_OK) return st;
  }
  for (int sw = 0; sw < n_sweeps; ++sw) {
    int nwin = 1, kb = 0;
    for (int i = 0; i < w->W; ++i) {
      const auto& x = w->wk[i];
      const long long L = w->h_ctl[i].sweep_len > 0 ? w->h_ctl[i].sweep_len : std::max(x.k_host, 1);
      nwin = std::max(nwin, (int)std::min<long long>((L + x.ks - 1) / x.ks, 1 << 20));
      kb = std::max(kb, x.k_host);
    }
    if (w->use_graphs) {
      st = launch_sweep_graph(w, kb, nwin);
      if (st != DCAX_OK) return st;
    } else {
      enqueue_sweep(w, kb, nwin);
    }
    HIPCHK(hipGetLastError());
    st = sync_all(w);
    if (st != DCAX_OK) return st;
    // windows closed early by a carried removal leave proposals of the sweep
    for (;;) {
      bool left = false;
      for (const Ctl& h : w->h_ctl) left |= h.pos < h.end;
      if (!left) break;
      const int kb2 = std::min(w->mo_max, w->kmax_host() + w->ks_max);
      if (w->mixed) enqueue_window<float>(w, kb2, false);
      else enqueue_window<double>(w, kb2, false);
      st = sync_all(w);
      if (st != DCAX_OK) return st;
    }
    ++w->sweeps_done;
    const int re = w->wk[0].p.refresh_every;
    if (re > 0 && w->sweeps_done % re == 0) {
      double d = 0.0;
      st = refresh_all(w, &d);
      if (st != DCAX_OK) return st;
      w->last_drift = d;
      w->max_drift = std::max(w->max_drift, d);
    } else {
      st = probe_and_refresh(w);
      if (st != DCAX_OK) return st;
    }
  }
  return DCAX_OK;
}

template <typename T>
size_t walker_bytes(const WalkerHost& x) {
  const size_t ks = KS_MAX, cap = x.cap, ld = x.ld, Nc = x.geo.Nc, kp = x.kpad_cap;
  const size_t nf = std::max(x.p.n_freq, 1);
  size_t b = 0;
  auto add = [&](size_t n) { b += (n + 255) & ~size_t(255); };
  add(sizeof(int) * Nc * Nc);                    // diff
  const size_t nt = x.p.n_spin_tables == 2 ? 2 : 1;
  add(sizeof(double) * nt * Nc * x.p.n_tau);     // table(s)
  if (x.p.g0_Kw) add(sizeof(double) * 2 * nt * Nc * nf);  // caller's G0(K, i w_n)
  add(sizeof(int) * 2 * Nc);                     // sites
  add(sizeof(double) * 2 * Nc);                  // K
  add(sizeof(double) * Nc);                      // xi
  add(sizeof(int) * cap);                        // v_site
  add(sizeof(double) * cap);                     // v_tau
  add(sizeof(int) * cap);                        // v_s
  add(sizeof(long long) * cap);                  // v_id
  for (int sp = 0; sp < 2; ++sp) add(sizeof(T) * ld * cap);  // N
  add(sizeof(WinProp) * KS_MAX);
  for (int i = 0; i < 9; ++i) add(sizeof(int) * KS_MAX);    // el_*, cand_el, S, ins_el, el_row, el_flip
  add(sizeof(double) * KS_MAX);                  // el_tau
  add(sizeof(long long) * KS_MAX);               // cand_id
  add(sizeof(int) * cap);                        // remap
  add(sizeof(int) * (2 * KS_MAX + 1));           // moves
  for (size_t sp = 0; sp < nt; ++sp) {
    add(sizeof(T) * ks * cap);                   // gcol
    add(sizeof(double) * KS_MAX * KS_MAX);       // gCC
  }
  for (int sp = 0; sp < 2; ++sp) {
    add(sizeof(T) * ks * cap);                   // W
    add(sizeof(T) * KS_MAX * cap);               // R
    add(sizeof(double) * KS_MAX * KS_MAX);       // gram
    add(sizeof(double) * KS_MAX * KS_MAX);       // ginv
    add(sizeof(T) * ks * cap);                   // Y
    add(sizeof(T) * KS_MAX * cap);               // A
    add(sizeof(T) * KS_MAX * cap);               // B
    add(sizeof(double) * cap * cap);             // M
    add(sizeof(double) * cap * NB);              // P
    add(sizeof(double) * cap * NB);              // Tm
    add(sizeof(int) * cap);                      // ipiv
    add(sizeof(int) * cap);                      // perm
    add(sizeof(double) * gjc_len(cap));          // gjc
    add(sizeof(T) * kp * kp);                    // m_Ms
    add(sizeof(double) * 2 * Nc * Nc * nf);      // m_Mab
  }
  add(sizeof(double) * 2 * 2 * (size_t)cdiv(cap, WG) * cap);  // blkmax
  add(sizeof(double) * 2);                       // detsign
  add(sizeof(int) * kp);                         // m_order
  add(sizeof(int) * (Nc + 1));                   // m_off
  add(sizeof(T) * 2 * kp * nf);                  // m_E
  return b + 256;
}

// Carves one walker's device memory out of a single allocation and fills its view.
template <typename T>
void wire_walker(dcax_walker w, WalkerHost& x, int wid, char* base, Ctl* ctl) {
  View<T>& v = hview<T>(x);
  std::memset(&v, 0, sizeof(v));
  auto take = [&](size_t bytes) {
    char* p = base;
    base += (bytes + 255) & ~size_t(255);
    return (void*)p;
  };
  const size_t ks = KS_MAX, cap = x.cap, ld = x.ld, Nc = x.geo.Nc, kp = x.kpad_cap;
  const size_t nf = std::max(x.p.n_freq, 1);
  v.Nc = (int)Nc;
  v.n_tau = x.p.n_tau;
  v.ks = x.ks;
  v.cap = x.cap;
  v.ld = x.ld;
  v.max_order = x.max_order;
  v.warmup = x.p.warmup_sweeps;
  v.beta = x.p.beta;
  v.h = x.p.beta / (double)(x.p.n_tau - 1);
  v.gamma = x.gamma;
  v.K_exp = x.p.K_exp;
  for (int sp = 0; sp < 2; ++sp) {
    const double sig = sp == 0 ? 1.0 : -1.0;
    v.ev[sp][0] = std::exp(sig * x.gamma);
    v.ev[sp][1] = std::exp(-sig * x.gamma);
  }
  v.seed = x.p.seed;
  v.flip_share = x.p.flip_share;
  v.neglect = x.p.touched_twice;
  v.diff = (const int*)take(sizeof(int) * Nc * Nc);
  const int nt = x.p.n_spin_tables == 2 ? 2 : 1;
  v.spin_tables = nt;
  v.ext_g0 = x.p.n_spin_tables > 0 ? 1 : 0;
  v.table[0] = (const double*)take(sizeof(double) * nt * Nc * x.p.n_tau);
  v.table[1] = v.table[0] + (nt == 2 ? Nc * (size_t)x.p.n_tau : 0);
  v.g0Kw = x.p.g0_Kw ? (const double*)take(sizeof(double) * 2 * nt * Nc * nf) : nullptr;
  v.sites = (const int*)take(sizeof(int) * 2 * Nc);
  v.Kp = (const double*)take(sizeof(double) * 2 * Nc);
  v.xi = (const double*)take(sizeof(double) * Nc);
  v.ctl = ctl;
  v.v_site = (int*)take(sizeof(int) * cap);
  v.v_tau = (double*)take(sizeof(double) * cap);
  v.v_s = (int*)take(sizeof(int) * cap);
  v.v_id = (long long*)take(sizeof(long long) * cap);
  for (int sp = 0; sp < 2; ++sp) v.N[sp] = (T*)take(sizeof(T) * ld * cap);
  v.wp = (WinProp*)take(sizeof(WinProp) * KS_MAX);
  v.el_site = (int*)take(sizeof(int) * KS_MAX);
  v.el_s = (int*)take(sizeof(int) * KS_MAX);
  v.el_slot = (int*)take(sizeof(int) * KS_MAX);
  v.el_flip = (int*)take(sizeof(int) * KS_MAX);
  v.el_cand = (int*)take(sizeof(int) * KS_MAX);
  v.el_row = (int*)take(sizeof(int) * KS_MAX);
  v.cand_el = (int*)take(sizeof(int) * KS_MAX);
  v.S = (int*)take(sizeof(int) * KS_MAX);
  v.ins_el = (int*)take(sizeof(int) * KS_MAX);
  v.el_tau = (double*)take(sizeof(double) * KS_MAX);
  v.cand_id = (long long*)take(sizeof(long long) * KS_MAX);
  v.remap = (int*)take(sizeof(int) * cap);
  v.moves = (int*)take(sizeof(int) * (2 * KS_MAX + 1));
  for (int sp = 0; sp < nt; ++sp) {
    v.gcol[sp] = (T*)take(sizeof(T) * ks * cap);
    v.gCC[sp] = (double*)take(sizeof(double) * KS_MAX * KS_MAX);
  }
  if (nt == 1) {
    v.gcol[1] = v.gcol[0];
    v.gCC[1] = v.gCC[0];
  }
  for (int sp = 0; sp < 2; ++sp) {
    v.W[sp] = (T*)take(sizeof(T) * ks * cap);
    v.R[sp] = (T*)take(sizeof(T) * KS_MAX * cap);
    v.gram[sp] = (double*)take(sizeof(double) * KS_MAX * KS_MAX);
    v.ginv[sp] = (double*)take(sizeof(double) * KS_MAX * KS_MAX);
    v.Y[sp] = (T*)take(sizeof(T) * ks * cap);
    v.A[sp] = (T*)take(sizeof(T) * KS_MAX * cap);
    v.B[sp] = (T*)take(sizeof(T) * KS_MAX * cap);
    v.M[sp] = (double*)take(sizeof(double) * cap * cap);
    v.P[sp] = (double*)take(sizeof(double) * cap * NB);
    v.Tm[sp] = (double*)take(sizeof(double) * cap * NB);
    v.ipiv[sp] = (int*)take(sizeof(int) * cap);
    v.perm[sp] = (int*)take(sizeof(int) * cap);
    v.gjc[sp] = (double*)take(sizeof(double) * gjc_len(cap));
    v.m_Ms[sp] = (T*)take(sizeof(T) * kp * kp);
    v.m_Mab[sp] = (double*)take(sizeof(double) * 2 * Nc * Nc * nf);
  }
  v.blkmax = (double*)take(sizeof(double) * 2 * 2 * (size_t)cdiv(cap, WG) * cap);
  v.detsign = (double*)take(sizeof(double) * 2);
  v.n_freq = x.p.n_freq;
  v.kpad_cap = x.kpad_cap;
  v.m_order = (int*)take(sizeof(int) * kp);
  v.m_off = (int*)take(sizeof(int) * (Nc + 1));
  v.m_E = (T*)take(sizeof(T) * 2 * kp * nf);
  v.ratio_out = w->ratio_d;
  v.replay = w->replay_d;
  v.acc_off = x.acc_off;
  v.nc_prefix = x.nc_prefix;
  v.wid = wid;
}

template <typename T>
dcax_status create_walkers(dcax_walker w) {
  w->ctl_all = (Ctl*)w->dalloc(sizeof(Ctl) * w->W);
  w->probe_d = (double*)w->dalloc(sizeof(double) * 2 * w->W);
  w->meas_list_d = (int*)w->dalloc(sizeof(int) * (w->W + 1));
  w->meas_pre_d = (long long*)w->dalloc(sizeof(long long) * (w->W + 1));
  if (!w->ctl_all || !w->probe_d || !w->meas_list_d || !w->meas_pre_d)
    return fail(DCAX_E_NOMEM, "device allocation failed");
  for (int i = 0; i < w->W; ++i) {
    WalkerHost& x = w->wk[i];
    char* base = (char*)w->dalloc(walker_bytes<T>(x));
    if (!base) return fail(DCAX_E_NOMEM, "device allocation failed (walker " + std::to_string(i) + ")");
    wire_walker<T>(w, x, i, base, w->ctl_all + i);
  }
  w->d_views = w->dalloc(sizeof(View<T>) * w->W);
  w->d_views_sel = w->dalloc(sizeof(View<T>) * w->W);
  if (!w->d_views || !w->d_views_sel) return fail(DCAX_E_NOMEM, "device allocation failed");
  std::vector<View<T>> hv(w->W);
  for (int i = 0; i < w->W; ++i) hv[i] = hview<T>(w->wk[i]);
  HIPCHK(hipMemcpyAsync(w->d_views, hv.data(), sizeof(View<T>) * w->W, hipMemcpyHostToDevice, w->stream));
  // model tables and the G0(r, tau) table of each walker
  for (int i = 0; i < w->W; ++i) {
    WalkerHost& x = w->wk[i];
    View<T>& v = hview<T>(x);
    const int Nc = x.geo.Nc;
    std::vector<double> xi(Nc);
    for (int q = 0; q < Nc; ++q) {
      const double cx = std::cos(x.geo.K[2 * q]), cy = std::cos(x.geo.K[2 * q + 1]);
      xi[q] = -2.0 * x.p.t * (cx + cy) - 4.0 * x.p.tp * cx * cy - x.p.mu;
    }
    HIPCHK(hipMemcpyAsync((void*)v.diff, x.geo.diff.data(), sizeof(int) * Nc * Nc, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync((void*)v.sites, x.geo.sites.data(), sizeof(int) * 2 * Nc, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync((void*)v.Kp, x.geo.K.data(), sizeof(double) * 2 * Nc, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync((void*)v.xi, xi.data(), sizeof(double) * Nc, hipMemcpyHostToDevice, w->stream));
    if (x.p.n_spin_tables == 0) {
      hipLaunchKernelGGL(k_g0_table, dim3(cdiv(x.p.n_tau, WG), Nc), dim3(WG), 0, w->stream, (double*)v.table[0], Nc,
                         x.p.n_tau, x.p.beta, v.sites, v.Kp, v.xi);
      HIPCHK(hipGetLastError());
    } else {
      // the caller's propagator, copied before this call returns (it syncs)
      const size_t nt = (size_t)v.spin_tables;
      HIPCHK(hipMemcpyAsync((void*)v.table[0], x.p.g0_tau, sizeof(double) * nt * Nc * x.p.n_tau,
                            hipMemcpyHostToDevice, w->stream));
      if (x.p.g0_Kw)
        HIPCHK(hipMemcpyAsync((void*)v.g0Kw, x.p.g0_Kw, sizeof(double) * 2 * nt * Nc * std::max(x.p.n_freq, 1),
                              hipMemcpyHostToDevice, w->stream));
    }
  }
  std::vector<Ctl> h(w->W);
  std::memset(h.data(), 0, sizeof(Ctl) * w->W);
  for (int i = 0; i < w->W; ++i) {
    h[i].sign = 1.0;
    h[i].carry_id = -1;
    h[i].sweep_len = w->wk[i].p.sweep_length;
  }
  HIPCHK(hipMemcpyAsync(w->ctl_all, h.data(), sizeof(Ctl) * w->W, hipMemcpyHostToDevice, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  // the caller's buffers are not referenced after creation
  for (auto& x : w->wk) {
    x.has_g0Kw = x.p.g0_Kw != nullptr;
    x.p.g0_tau = nullptr;
    x.p.g0_Kw = nullptr;
  }
  return DCAX_OK;
}

// Replay buffers are shared by the views; (re)point them after a reallocation.
// One round of device-scheduled sweeps: walkers between sweeps begin their
// next one, nwin windows run, and the walkers whose sweep has ended are
// measured (gated measurement).
template <typename T>
void enqueue_round(dcax_walker w, int kb, int nwin, double* acc, double* aux, int nfft_hw) {
  w->fresh = false;
  hipLaunchKernelGGL(k_round_begin<T>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<T>());
  for (int i = 0; i < nwin; ++i) enqueue_window<T>(w, kb, false);
  // drift control: each walker whose sweep has just ended is probed before
  // its measurement, and held for a rebuild if N has drifted too far
  const double tol = w->wk[0].p.drift_tol;
  if (tol > 0.0)
    hipLaunchKernelGGL(k_probe<T>, dim3(1, 2, w->W), dim3(WG), 0, w->stream, w->views<T>(),
                       0xD1B54A32D192ED03ULL ^ w->wk[0].p.seed, w->probe_d, tol);
  if (nfft_hw > 0) enqueue_nfft<T>(w, nfft_hw, acc, aux, 1);
  else enqueue_measure<T>(w, acc, aux, 1);
}

// After a round: rebuild the walkers the sweep-end probe held (one masked
// refresh for all of them), then take their pending measurements.  A rebuild
// pass costs about the same for one walker as for many (its column steps are
// launch-latency-bound), while a held walker only sits out the rounds (the
// batch's launches shrink with it), so in a batch the pass waits until an
// eighth of the walkers are held or the first of them has waited `wait`
// rounds (a sweep: 32 walkers of 8x8 make 57.6k accepted updates/s with a
// quarter sweep, 59.9k with a sweep); force releases at once.
// Synchronises.
template <typename T>
dcax_status release_held(dcax_walker w, double* acc, double* aux, int nfft_hw, long long wait, bool force) {
  dcax_status st = sync_all(w);
  if (st != DCAX_OK) return st;
  ++w->probes;
  int nheld = 0, kheld = 0;
  for (int i = 0; i < w->W; ++i)
    if (w->h_ctl[i].hold) {
      ++nheld;
      kheld = std::max(kheld, w->h_ctl[i].k);
    }
  if (nheld == 0) {
    w->held_since = -1;
    return DCAX_OK;
  }
  if (w->held_since < 0) w->held_since = w->rounds_done;
  if (!force && nheld < std::max(1, w->W / 8) && w->rounds_done - w->held_since < wait) return DCAX_OK;
  w->held_since = -1;
  std::vector<double> h(2 * w->W);
  HIPCHK(hipMemcpy(h.data(), w->probe_d, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
  double m = 0.0;
  for (int i = 0; i < w->W; ++i)
    if (w->h_ctl[i].hold)
      for (int sp = 0; sp < 2; ++sp) m = (h[2 * i + sp] > m || h[2 * i + sp] != h[2 * i + sp]) ? h[2 * i + sp] : m;
  w->last_probe = m;
  w->probe_refreshes += nheld;
  std::vector<int> idx;
  for (int i = 0; i < w->W; ++i)
    if (w->h_ctl[i].hold) idx.push_back(i);
  enqueue_refresh_some<T>(w, idx, kheld);     // releases them (clears hold)
  if (nfft_hw > 0) enqueue_nfft<T>(w, nfft_hw, acc, aux, 1);
  else enqueue_measure<T>(w, acc, aux, 1);
  HIPCHK(hipGetLastError());
  std::vector<int> was(w->W);
  for (int i = 0; i < w->W; ++i) was[i] = w->h_ctl[i].hold;
  st = sync_all(w);
  if (st != DCAX_OK) return st;
  for (int i = 0; i < w->W; ++i)
    if (was[i]) w->max_drift = std::max(w->max_drift, w->h_ctl[i].drift);
  return DCAX_OK;
}

// Sweeps of every walker, each followed by its measurement, scheduled on the
// device: a walker starts its next sweep as soon as the previous one has been
// measured, so walkers of different sweep lengths in one batch do not wait
// for the longest.  With free_rounds == 0 every walker makes n sweeps; with
// free_rounds > 0 every walker sweeps for that many rounds and then finishes
// the sweep it is in (short walkers make more sweeps than long ones).
// Kernel grids follow the order seen at the last sync (the kernels stride
// over the device-side order); the host syncs only to refresh, and at the
// end to check that every walker has finished (rounds lost to windows closed
// early are made up).  nfft_hw > 0: the measurement is the delayed-NFFT
// gridding into acc (a grid) with that kernel half-width.
dcax_status sweep_rounds(dcax_walker w, int n, double* acc, double* aux, long long free_rounds = 0,
                         int nfft_hw = 0) {
  dcax_status st = DCAX_OK;
  if (!w->fresh) {
    st = sync_all(w);
    if (st != DCAX_OK) return st;
  }
  if (n == 0 && free_rounds == 0) return DCAX_OK;
  w->fresh = false;
  const long long each = free_rounds > 0 ? (1ll << 60) : (long long)n;
  if (w->mixed) hipLaunchKernelGGL(k_set_rounds<float>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<float>(), each);
  else hipLaunchKernelGGL(k_set_rounds<double>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<double>(), each);
  // windows per sweep of each walker; a single walker runs one sweep per
  // round, a batch ROUND_WINDOWS windows per round
  long long nw_max = 1, nw_sum = 0;
  for (int i = 0; i < w->W; ++i) {
    const auto& x = w->wk[i];
    const long long L = w->h_ctl[i].sweep_len > 0 ? w->h_ctl[i].sweep_len : std::max(x.k_host, 1);
    const long long nw = std::max<long long>(1, (L + x.ks - 1) / x.ks);
    nw_max = std::max(nw_max, nw);
    nw_sum += nw;
  }
  constexpr int ROUND_WINDOWS = 4;
  const int R = (w->W == 1) ? (int)std::min<long long>(nw_max, 1 << 20) : (int)std::min<long long>(nw_max, ROUND_WINDOWS);
  const long long rounds_per_sweep = (nw_max + R - 1) / R;
  // refresh every refresh_every sweeps of the average walker
  const int re = w->wk[0].p.refresh_every;
  const long long nw_mean = std::max<long long>(1, (nw_sum + w->W - 1) / w->W);
  const long long refresh_rounds = re > 0 ? std::max<long long>(1, re * ((nw_mean + R - 1) / R)) : 0;
  long long planned = free_rounds > 0 ? free_rounds : (long long)n * rounds_per_sweep;
  for (int pass = 0;; ++pass) {
    if (pass > 64) return fail(DCAX_E_STATE, "device-scheduled sweeps made no progress");
    const int kb = std::min(w->mo_max, w->kmax_host() + 2 * w->ks_max);
    // A single walker runs one sweep per round.  A window closed early by a
    // carried removal makes its sweep need one window more, and a sweep left
    // unfinished would cost a whole round of empty windows, so at large
    // orders (where an empty window's launches cost little beside a full
    // one) the round carries spare windows in proportion to the observed
    // share of such windows; unused spares find the sweep complete and exit.
    int spare = 0;
    if (w->W == 1 && kb >= SPARE_MIN_ORDER) {
      const Ctl& h = w->h_ctl[0];
      const double expect = h.n_windows > 0 ? (double)R * (double)h.n_abort / (double)h.n_windows : 0.0;
      if (expect > 0.0) spare = (int)std::ceil(expect + 2.0 * std::sqrt(expect) + 1.0);
    }
    hipGraphExec_t rg = nullptr;
    if (w->use_graphs) {
      // one round as a hipGraph, captured once per (order bound, windows,
      // measurement buffers) and replayed for every round of this pass
      const auto key = std::make_tuple(kb, R + spare, nfft_hw, acc, aux);
      auto it = w->round_graphs.find(key);
      if (it == w->round_graphs.end()) {
        hipGraphExec_t exec = nullptr;
        st = capture_graph(w, [&] {
          if (w->mixed) enqueue_round<float>(w, kb, R + spare, acc, aux, nfft_hw);
          else enqueue_round<double>(w, kb, R + spare, acc, aux, nfft_hw);
        }, &exec);
        if (st != DCAX_OK) return st;
        it = w->round_graphs.emplace(key, exec).first;
      }
      rg = it->second;
    }
    for (long long r = 0; r < planned; ++r) {
      if (rg) {
        w->fresh = false;
        st = launch_graph(w, rg);
        if (st != DCAX_OK) return st;
      } else if (w->mixed) {
        enqueue_round<float>(w, kb, R + spare, acc, aux, nfft_hw);
      } else {
        enqueue_round<double>(w, kb, R + spare, acc, aux, nfft_hw);
      }
      HIPCHK(hipGetLastError());
      ++w->rounds_done;
      if (refresh_rounds > 0 && w->rounds_done % refresh_rounds == 0) {
        double d = 0.0;
        st = refresh_all(w, &d);
        if (st != DCAX_OK) return st;
        w->last_drift = d;
        w->max_drift = std::max(w->max_drift, d);
        // walkers the probe held are rebuilt too: take their measurements
        if (w->wk[0].p.drift_tol > 0.0) {
          if (nfft_hw > 0) {
            if (w->mixed) enqueue_nfft<float>(w, nfft_hw, acc, aux, 1);
            else enqueue_nfft<double>(w, nfft_hw, acc, aux, 1);
          } else if (w->mixed) {
            enqueue_measure<float>(w, acc, aux, 1);
          } else {
            enqueue_measure<double>(w, acc, aux, 1);
          }
          HIPCHK(hipGetLastError());
        }
      } else if (w->wk[0].p.drift_tol > 0.0) {
        const long long wait = std::max<long long>(1, rounds_per_sweep);
        const bool last = r + 1 == planned;
        st = w->mixed ? release_held<float>(w, acc, aux, nfft_hw, wait, last)
                      : release_held<double>(w, acc, aux, nfft_hw, wait, last);
        if (st != DCAX_OK) return st;
      }
    }
    if (free_rounds > 0 && pass == 0) {
      if (w->mixed) hipLaunchKernelGGL(k_stop_rounds<float>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<float>());
      else hipLaunchKernelGGL(k_stop_rounds<double>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<double>());
    }
    st = sync_all(w);
    if (st != DCAX_OK) return st;
    // rounds the slowest walker still needs: the rest of its sweep (or the
    // pending measurement, which closes a round), then its whole sweeps; a
    // sweep that windows closed early stretch is topped up by another pass
    long long need = 0;
    for (int i = 0; i < w->W; ++i) {
      const Ctl& h = w->h_ctl[i];
      const auto& x = w->wk[i];
      const long long L = h.sweep_len > 0 ? h.sweep_len : std::max(x.k_host, 1);
      const long long nw = std::max<long long>(1, (L + x.ks - 1) / x.ks);
      long long r = h.sweeps_left * ((nw + R - 1) / R);
      if (h.pos < h.end) r += ((h.end - h.pos + x.ks - 1) / x.ks + R - 1) / R;
      else if (h.meas_due) r += 1;
      need = std::max(need, r);
    }
    if (need == 0) break;
    planned = need;
  }
  if (free_rounds == 0) w->sweeps_done += n;
  return DCAX_OK;
}

template <typename T>
dcax_status repoint_replay(dcax_walker w, dcax_proposal* rec, double* rat) {
  std::vector<View<T>> hv(w->W);
  for (int i = 0; i < w->W; ++i) {
    View<T>& v = hview<T>(w->wk[i]);
    v.replay = rec;
    v.ratio_out = rat;
    hv[i] = v;
  }
  HIPCHK(hipMemcpyAsync(w->d_views, hv.data(), sizeof(View<T>) * w->W, hipMemcpyHostToDevice, w->stream));
  return DCAX_OK;
}

template <typename T>
const View<T>& view0(dcax_walker w, int i) { return hview<T>(w->wk[i]); }

template <typename T>
dcax_status upload_views(dcax_walker w) {
  std::vector<View<T>> hv(w->W);
  for (int i = 0; i < w->W; ++i) hv[i] = hview<T>(w->wk[i]);
  HIPCHK(hipMemcpyAsync(w->d_views, hv.data(), sizeof(View<T>) * w->W, hipMemcpyHostToDevice, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  return DCAX_OK;
}

dcax_status set_ks(dcax_walker w, int walker, int ks) {
  for (int i = 0; i < w->W; ++i) {
    if (walker >= 0 && i != walker) continue;
    w->wk[i].ks = ks;
    w->wk[i].v64.ks = ks;
    w->wk[i].v32.ks = ks;
  }
  w->ks_max = 0;
  for (const auto& x : w->wk) w->ks_max = std::max(w->ks_max, x.ks);
  w->clear_graphs();
  return w->mixed ? upload_views<float>(w) : upload_views<double>(w);
}

}  // namespace

// ================================================================= C ABI
extern "C" {

const char* dcax_last_error(void) { return g_err.c_str(); }

dcax_status dcax_cluster(const dcax_params* p, int32_t* n_sites, int32_t* sites, double* momenta) {
  if (!p || !n_sites) return fail(DCAX_E_INVAL, "NULL argument");
  Geometry g;
  if (!build_geometry(p->cluster, g)) return fail(DCAX_E_INVAL, "degenerate or too large cluster");
  *n_sites = g.Nc;
  if (sites) std::copy(g.sites.begin(), g.sites.end(), sites);
  if (momenta) std::copy(g.K.begin(), g.K.end(), momenta);
  return DCAX_OK;
}

dcax_status dcax_walker_create(const dcax_params* p, int32_t n_walkers, const dcax_allocator* a, void* stream,
                               dcax_walker* out) {
  if (!out) return fail(DCAX_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(DCAX_E_INVAL, "params is NULL");
  if (n_walkers < 1 || n_walkers > 32767) return fail(DCAX_E_INVAL, "n_walkers must be in 1..32767");
  for (int i = 0; i < n_walkers; ++i) {
    dcax_status st = validate(p + i);
    if (st != DCAX_OK) return fail(st, "walker " + std::to_string(i) + ": " + g_err);
    if (p[i].precision != p[0].precision) return fail(DCAX_E_INVAL, "all walkers of a batch share one precision");
  }
  if (!a || !a->alloc || !a->free) return fail(DCAX_E_INVAL, "an allocator with alloc and free is required");
  dcax_walker w = new dcax_walker_s();
  w->W = n_walkers;
  w->alloc = *a;
  w->stream = (hipStream_t)stream;
  w->mixed = p[0].precision == DCAX_FP32_MIXED;
  w->wk.resize(n_walkers);
  w->h_ctl.resize(n_walkers);
  long long acc = 0;
  int ncp = 0;
  for (int i = 0; i < n_walkers; ++i) {
    WalkerHost& x = w->wk[i];
    x.p = p[i];
    build_geometry(p[i].cluster, x.geo);
    x.ks = p[i].submatrix_k;
    x.max_order = p[i].max_order;
    x.cap = ((p[i].max_order + KS_MAX + 63) / 64) * 64;
    x.ld = x.cap;
    x.kpad_cap = x.cap + 16 * x.geo.Nc;
    x.gamma = std::acosh(1.0 + p[i].U * p[i].beta * (double)x.geo.Nc / (2.0 * p[i].K_exp));
    x.acc_off = acc;
    x.nc_prefix = ncp;
    acc += 4LL * x.geo.Nc * std::max(p[i].n_freq, 1);
    ncp += x.geo.Nc;
    w->ks_max = std::max(w->ks_max, x.ks);
    w->cap_max = std::max(w->cap_max, x.cap);
    w->nc_max = std::max(w->nc_max, x.geo.Nc);
    w->nf_max = std::max(w->nf_max, p[i].n_freq);
    w->kpad_max = std::max(w->kpad_max, x.kpad_cap);
    w->mo_max = std::max(w->mo_max, x.max_order);
  }
  w->acc_total = acc;
  w->nc_total = ncp;
  w->static_scratch = static_scratch_of_current_device();
  dcax_status st = w->mixed ? create_walkers<float>(w) : create_walkers<double>(w);
  if (st != DCAX_OK) {
    (void)hipStreamSynchronize(w->stream);
    w->release();
    delete w;
    return st;
  }
  *out = w;
  return DCAX_OK;
}

dcax_status dcax_walker_destroy(dcax_walker w) {
  if (!w) return DCAX_OK;
  (void)hipStreamSynchronize(w->stream);
  w->release();
  delete w;
  return DCAX_OK;
}

dcax_status dcax_set_config(dcax_walker w, int32_t walker, const dcax_vertex* v, int32_t k) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (walker < 0 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  WalkerHost& x = w->wk[walker];
  if (k < 0 || k > x.max_order || (k > 0 && !v)) return fail(DCAX_E_INVAL, "bad configuration size");
  std::vector<int> site(k), s(k);
  std::vector<double> tau(k);
  std::vector<long long> id(k);
  long long next_id = 0;
  for (int i = 0; i < k; ++i) {
    if (v[i].site < 0 || v[i].site >= x.geo.Nc) return fail(DCAX_E_INVAL, "vertex site out of range");
    if (v[i].aux_spin != 1 && v[i].aux_spin != -1) return fail(DCAX_E_INVAL, "aux_spin must be +1 or -1");
    if (!(v[i].tau >= 0.0 && v[i].tau < x.p.beta)) return fail(DCAX_E_INVAL, "tau must be in [0, beta)");
    if (v[i].id < 0) return fail(DCAX_E_INVAL, "vertex ids must be >= 0");
    site[i] = v[i].site;
    s[i] = v[i].aux_spin;
    tau[i] = v[i].tau;
    id[i] = v[i].id;
    next_id = std::max(next_id, (long long)v[i].id + 1);
  }
  {
    std::vector<long long> sid(id);
    std::sort(sid.begin(), sid.end());
    if (std::adjacent_find(sid.begin(), sid.end()) != sid.end()) return fail(DCAX_E_INVAL, "duplicate vertex ids");
  }
  int* vs_ = w->mixed ? x.v32.v_site : x.v64.v_site;
  double* vt = w->mixed ? x.v32.v_tau : x.v64.v_tau;
  int* vsp = w->mixed ? x.v32.v_s : x.v64.v_s;
  long long* vid = w->mixed ? x.v32.v_id : x.v64.v_id;
  if (k > 0) {
    HIPCHK(hipMemcpyAsync(vs_, site.data(), sizeof(int) * k, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync(vt, tau.data(), sizeof(double) * k, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync(vsp, s.data(), sizeof(int) * k, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync(vid, id.data(), sizeof(long long) * k, hipMemcpyHostToDevice, w->stream));
  }
  Ctl h;
  std::memset(&h, 0, sizeof(h));
  h.k = k;
  h.next_id = next_id;
  h.sign = 1.0;
  h.carry_id = -1;
  h.sweep_len = x.p.sweep_length;
  w->fresh = false;
  HIPCHK(hipMemcpyAsync(w->ctl_all + walker, &h, sizeof(Ctl), hipMemcpyHostToDevice, w->stream));
  if (w->mixed) {
    enqueue_refresh<float>(w, walker, 1, k, false);
    hipLaunchKernelGGL(k_set_sign<float>, dim3(1), dim3(1), 0, w->stream, w->views<float>(walker));
  } else {
    enqueue_refresh<double>(w, walker, 1, k, false);
    hipLaunchKernelGGL(k_set_sign<double>, dim3(1), dim3(1), 0, w->stream, w->views<double>(walker));
  }
  HIPCHK(hipGetLastError());
  x.latched = false;
  return sync_all(w);
}

}  // extern "C"

namespace {

// Host checks of replay records (argument errors, nothing enqueued).
dcax_status check_replay(dcax_walker w, const dcax_proposal* replay, int64_t n_replay) {
  if (w->W != 1) return fail(DCAX_E_INVAL, "replay needs a single-walker handle");
  if (n_replay < 0) return fail(DCAX_E_INVAL, "n_replay < 0");
  const WalkerHost& x = w->wk[0];
  for (int64_t i = 0; i < n_replay; ++i) {
    const dcax_proposal& r = replay[i];
    if (r.kind < 0 || r.kind > 2) return fail(DCAX_E_INVAL, "replay kind must be 0, 1 or 2");
    if (r.accepted != 0 && r.accepted != 1) return fail(DCAX_E_INVAL, "replay accepted must be 0 or 1");
    if (r.kind == 0) {
      if (r.site < 0 || r.site >= x.geo.Nc) return fail(DCAX_E_INVAL, "replay site out of range");
      if (r.aux_spin != 1 && r.aux_spin != -1) return fail(DCAX_E_INVAL, "replay aux_spin must be +1 or -1");
      if (!(r.tau >= 0.0 && r.tau < x.p.beta)) return fail(DCAX_E_INVAL, "replay tau outside [0, beta)");
      if (r.accepted && r.id < 0) return fail(DCAX_E_INVAL, "accepted insertion needs an id >= 0");
    } else if (r.id < 0 && r.accepted) {
      return fail(DCAX_E_INVAL, "a removal or flip without target cannot be accepted");
    }
  }
  return DCAX_OK;
}

// Replays n_replay records staged at rec (device) with forced decisions; the
// ratios land at rat (device, cleared first) and are copied to ratio_out.
dcax_status replay_staged(dcax_walker w, const dcax_proposal* replay, int64_t n_replay, double* ratio_out,
                          dcax_proposal* rec, double* rat) {
  if (w->views_replay != rec) {
    dcax_status st = w->mixed ? repoint_replay<float>(w, rec, rat) : repoint_replay<double>(w, rec, rat);
    if (st != DCAX_OK) return st;
    w->views_replay = rec;
  }
  const WalkerHost& x = w->wk[0];
  HIPCHK(hipMemcpyAsync(rec, replay, sizeof(dcax_proposal) * n_replay, hipMemcpyHostToDevice, w->stream));
  hipLaunchKernelGGL(k_fill_zero, dim3(std::min(cdiv(n_replay, WG), 256)), dim3(WG), 0, w->stream, rat,
                     (long long)n_replay);
  if (w->mixed) hipLaunchKernelGGL(k_set_cursor<float>, dim3(1), dim3(1), 0, w->stream, w->views<float>(), 0LL, (long long)n_replay);
  else hipLaunchKernelGGL(k_set_cursor<double>, dim3(1), dim3(1), 0, w->stream, w->views<double>(), 0LL, (long long)n_replay);
  // A window that ends before a second change of one spin (flip then
  // removal, insertion then flip) leaves records for more windows than
  // ceil(n / k_s): enqueue what the records left need, until none are left.
  long long left = n_replay;
  for (;;) {
    const long long nwin = (left + x.ks - 1) / x.ks;
    int kb = x.k_host;
    for (long long i = 0; i < nwin; ++i) {
      kb = std::min(x.max_order, kb + x.ks);
      if (w->mixed) enqueue_window<float>(w, kb, true);
      else enqueue_window<double>(w, kb, true);
    }
    HIPCHK(hipGetLastError());
    dcax_status st = sync_all(w);
    if (st != DCAX_OK) return st;
    left = w->h_ctl[0].end - w->h_ctl[0].pos;
    if (left <= 0) break;
  }
  if (ratio_out) HIPCHK(hipMemcpyAsync(ratio_out, rat, sizeof(double) * n_replay, hipMemcpyDeviceToHost, w->stream));
  return sync_all(w);
}

}  // namespace

extern "C" {

dcax_status dcax_sweep(dcax_walker w, int32_t n_sweeps, const dcax_proposal* replay, int64_t n_replay,
                       double* ratio_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (replay) {
    st = check_replay(w, replay, n_replay);
    if (st != DCAX_OK || n_replay == 0) return st;
    if (n_replay > w->replay_cap) {
      const long long cap = std::max<long long>(n_replay, 4096);
      w->replay_d = (dcax_proposal*)w->dalloc(sizeof(dcax_proposal) * cap);
      w->ratio_d = (double*)w->dalloc(sizeof(double) * cap);
      if (!w->replay_d || !w->ratio_d) return fail(DCAX_E_NOMEM, "replay buffer allocation failed");
      w->replay_cap = cap;
    }
    return replay_staged(w, replay, n_replay, ratio_out, w->replay_d, w->ratio_d);
  }
  if (n_sweeps < 0) return fail(DCAX_E_INVAL, "n_sweeps < 0");
  return sweep_rng(w, n_sweeps);
}

dcax_status dcax_sweep_replay_static(dcax_walker w, const dcax_proposal* replay, int64_t n_replay,
                                     double* ratio_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (!replay) return fail(DCAX_E_INVAL, "replay is NULL");
  if (n_replay > DCAX_REPLAY_STATIC_MAX)
    return fail(DCAX_E_INVAL, "n_replay exceeds DCAX_REPLAY_STATIC_MAX (" + std::to_string(DCAX_REPLAY_STATIC_MAX) +
                                  " records)");
  st = check_replay(w, replay, n_replay);
  if (st != DCAX_OK || n_replay == 0) return st;
  if (!w->static_scratch) return fail(DCAX_E_HIP, "the static replay staging has no device address on this GPU");
  dcax_proposal* rec = (dcax_proposal*)w->static_scratch;
  double* rat = (double*)((char*)w->static_scratch + STATIC_REC_BYTES);
  return replay_staged(w, replay, n_replay, ratio_out, rec, rat);
}

dcax_status dcax_sweep_measure(dcax_walker w, int32_t n_sweeps, double* acc_dev, double* aux_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (n_sweeps < 0) return fail(DCAX_E_INVAL, "n_sweeps < 0");
  if (!aux_dev || (!acc_dev && w->nf_max > 0)) return fail(DCAX_E_INVAL, "NULL accumulator");
  return sweep_rounds(w, n_sweeps, acc_dev, aux_dev);
}

dcax_status dcax_sweep_measure_nfft(dcax_walker w, int32_t n_sweeps, int32_t half_width, double* grid_dev,
                                    double* aux_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (n_sweeps < 0) return fail(DCAX_E_INVAL, "n_sweeps < 0");
  if (!grid_dev || !aux_dev) return fail(DCAX_E_INVAL, "NULL accumulator");
  st = nfft_check(w, half_width);
  if (st != DCAX_OK) return st;
  return sweep_rounds(w, n_sweeps, grid_dev, aux_dev, 0, half_width);
}

dcax_status dcax_run_rounds(dcax_walker w, int32_t n_rounds, double* acc_dev, double* aux_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (n_rounds < 0) return fail(DCAX_E_INVAL, "n_rounds < 0");
  if (!aux_dev || (!acc_dev && w->nf_max > 0)) return fail(DCAX_E_INVAL, "NULL accumulator");
  if (n_rounds == 0) return DCAX_OK;
  return sweep_rounds(w, 0, acc_dev, aux_dev, n_rounds);
}

dcax_status dcax_refresh(dcax_walker w, double* drift_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  return refresh_all(w, drift_out);
}

dcax_status dcax_measure_G(dcax_walker w, double* acc_dev, double* aux_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (!aux_dev || (!acc_dev && w->nf_max > 0)) return fail(DCAX_E_INVAL, "NULL accumulator");
  if (w->mixed) enqueue_measure<float>(w, acc_dev, aux_dev, 0);
  else enqueue_measure<double>(w, acc_dev, aux_dev, 0);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_measure_nfft(dcax_walker w, int32_t half_width, double* grid_dev, double* aux_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (!grid_dev || !aux_dev) return fail(DCAX_E_INVAL, "NULL accumulator");
  st = nfft_check(w, half_width);
  if (st != DCAX_OK) return st;
  if (w->mixed) enqueue_nfft<float>(w, half_width, grid_dev, aux_dev, 0);
  else enqueue_nfft<double>(w, half_width, grid_dev, aux_dev, 0);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_nfft_transform(dcax_walker w, int32_t half_width, const double* grid_dev, double* acc_dev) {
  if (!w || !grid_dev || !acc_dev) return fail(DCAX_E_INVAL, "NULL argument");
  dcax_status st = nfft_check(w, half_width);
  if (st != DCAX_OK) return st;
  const int nf = w->nf_max, ncm = w->nc_max, W = w->W;
  if (w->mixed) {
    hipLaunchKernelGGL(k_nfft_rows<float>, dim3(cdiv(nf, WG), ncm, 2 * W), dim3(WG), 0, w->stream,
                       w->views<float>(), half_width, grid_dev);
    hipLaunchKernelGGL(k_nfft_K<float>, dim3(cdiv(nf, WG), ncm, 2 * W), dim3(WG), 0, w->stream, w->views<float>(),
                       acc_dev);
  } else {
    hipLaunchKernelGGL(k_nfft_rows<double>, dim3(cdiv(nf, WG), ncm, 2 * W), dim3(WG), 0, w->stream,
                       w->views<double>(), half_width, grid_dev);
    hipLaunchKernelGGL(k_nfft_K<double>, dim3(cdiv(nf, WG), ncm, 2 * W), dim3(WG), 0, w->stream, w->views<double>(),
                       acc_dev);
  }
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_finalize_G(dcax_walker w, const double* acc_dev, const double* aux_dev, double* Giw_dev,
                            int32_t n_tau_out, double* Gtau_dev) {
  if (!w || !acc_dev || !aux_dev || !Giw_dev) return fail(DCAX_E_INVAL, "NULL argument");
  if (n_tau_out < 0 || n_tau_out == 1 || (n_tau_out > 0 && !Gtau_dev)) return fail(DCAX_E_INVAL, "bad n_tau_out");
  for (const auto& x : w->wk)
    if (x.p.n_spin_tables > 0 && !x.has_g0Kw && x.p.n_freq > 0)
      return fail(DCAX_E_INVAL, "a walker was given g0_tau without g0_Kw: G0(K, i w_n) is unknown");
  const int nx = std::max(w->nf_max, n_tau_out);
  if (nx == 0) return DCAX_OK;
  double* gt = n_tau_out > 0 ? Gtau_dev : nullptr;
  if (w->mixed)
    hipLaunchKernelGGL(k_finalize<float>, dim3(cdiv(nx, WG), w->nc_max, 2 * w->W), dim3(WG), 0, w->stream,
                       w->views<float>(), acc_dev, aux_dev, Giw_dev, n_tau_out, gt);
  else
    hipLaunchKernelGGL(k_finalize<double>, dim3(cdiv(nx, WG), w->nc_max, 2 * w->W), dim3(WG), 0, w->stream,
                       w->views<double>(), acc_dev, aux_dev, Giw_dev, n_tau_out, gt);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_get_order(dcax_walker w, int32_t walker, int32_t* k) {
  if (!w || !k) return fail(DCAX_E_INVAL, "NULL argument");
  if (walker < 0 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  dcax_status st = sync_all(w);
  *k = w->h_ctl[walker].k;
  return st;
}

dcax_status dcax_get_config(dcax_walker w, int32_t walker, dcax_vertex* out, int32_t cap, int32_t* k) {
  if (!w || !k) return fail(DCAX_E_INVAL, "NULL argument");
  if (walker < 0 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  dcax_status st = sync_all(w);
  if (st == DCAX_E_HIP) return st;
  const int n = w->h_ctl[walker].k;
  *k = n;
  if (!out) return st;
  if (cap < n) return fail(DCAX_E_INVAL, "output too small");
  const WalkerHost& x = w->wk[walker];
  std::vector<int> site(n), s(n);
  std::vector<double> tau(n);
  std::vector<long long> id(n);
  const bool mx = w->mixed;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(site.data(), mx ? x.v32.v_site : x.v64.v_site, sizeof(int) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(tau.data(), mx ? x.v32.v_tau : x.v64.v_tau, sizeof(double) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(s.data(), mx ? x.v32.v_s : x.v64.v_s, sizeof(int) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(id.data(), mx ? x.v32.v_id : x.v64.v_id, sizeof(long long) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
  }
  for (int i = 0; i < n; ++i) {
    out[i].id = id[i];
    out[i].site = site[i];
    out[i].aux_spin = s[i];
    out[i].tau = tau[i];
  }
  return st;
}

dcax_status dcax_copy_N(dcax_walker w, int32_t walker, int32_t spin, double* host, int64_t ld, int64_t* ids_host) {
  if (!w || !host || (spin != 0 && spin != 1)) return fail(DCAX_E_INVAL, "bad argument");
  if (walker < 0 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  dcax_status st = sync_all(w);
  if (st == DCAX_E_HIP) return st;
  const int k = w->h_ctl[walker].k;
  if (ld < k) return fail(DCAX_E_INVAL, "ld < k");
  if (k == 0) return st;
  const WalkerHost& x = w->wk[walker];
  const bool mx = w->mixed;
  std::vector<long long> id(k);
  HIPCHK(hipMemcpyAsync(id.data(), mx ? x.v32.v_id : x.v64.v_id, sizeof(long long) * k, hipMemcpyDeviceToHost, w->stream));
  std::vector<double> Nh((size_t)k * k);
  if (mx) {
    std::vector<float> Nf((size_t)x.ld * k);
    HIPCHK(hipMemcpyAsync(Nf.data(), x.v32.N[spin], sizeof(float) * (size_t)x.ld * k, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) Nh[i + (size_t)j * k] = Nf[i + (size_t)j * x.ld];
  } else {
    std::vector<double> Nd((size_t)x.ld * k);
    HIPCHK(hipMemcpyAsync(Nd.data(), x.v64.N[spin], sizeof(double) * (size_t)x.ld * k, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) Nh[i + (size_t)j * k] = Nd[i + (size_t)j * x.ld];
  }
  std::vector<int> o(k);
  for (int i = 0; i < k; ++i) o[i] = i;
  std::sort(o.begin(), o.end(), [&](int a, int b) { return id[a] < id[b]; });
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) host[(size_t)a * ld + b] = Nh[o[a] + (size_t)o[b] * k];
  if (ids_host)
    for (int a = 0; a < k; ++a) ids_host[a] = id[o[a]];
  return st;
}

static_assert(sizeof(dcax_stats::fold_rank_hist) == sizeof(int64_t) * FOLD_RANK_BINS,
              "fold-rank histogram bins of the ABI and of the control block differ");

dcax_status dcax_get_stats(dcax_walker w, int32_t walker, dcax_stats* out) {
  if (!w || !out) return fail(DCAX_E_INVAL, "NULL argument");
  if (walker < -1 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  dcax_status st = sync_all(w);
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < w->W; ++i) {
    if (walker >= 0 && i != walker) continue;
    const Ctl& h = w->h_ctl[i];
    out->proposals += h.n_prop;
    out->accepted_insertions += h.n_acc_ins;
    out->accepted_removals += h.n_acc_rem;
    out->accepted_flips += h.n_acc_flip;
    out->neglected += h.n_neglect;
    out->windows += h.n_windows;
    out->flips_folded += h.sum_m;
    out->decision_mismatches += h.n_mismatch;
    out->fold_flops += h.fold_flops;
    out->fold_bytes += h.fold_bytes;
    out->cand_flops += h.cand_flops;
    out->cand_bytes += h.cand_bytes;
    out->y_flops += h.y_flops;
    out->y_bytes += h.y_bytes;
    out->aborted_windows += h.n_abort;
    for (int b = 0; b < FOLD_RANK_BINS; ++b) out->fold_rank_hist[b] += h.m_hist[b];
  }
  out->sign = w->h_ctl[walker >= 0 ? walker : 0].sign;
  out->sweeps = w->sweeps_done;
  out->fold_seconds = w->fold_s;
  out->fold_launches = w->fold_launches;
  out->windows_enqueued = w->win_seq;
  out->accept_seconds = w->accept_s;
  out->window_seconds = w->window_s;
  out->cand_seconds = w->cand_s;
  out->y_seconds = w->y_s;
  out->last_drift = w->last_drift;
  out->max_drift = w->max_drift;
  out->probes = w->probes;
  out->probe_refreshes = w->probe_refreshes;
  out->last_probe = w->last_probe;
  return st;
}

dcax_status dcax_probe_N(dcax_walker w, double* residual_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  st = sync_all(w);
  if (st != DCAX_OK) return st;
  std::vector<double> res;
  st = probe_all(w, res);
  if (st != DCAX_OK) return st;
  if (residual_out) std::copy(res.begin(), res.end(), residual_out);
  return DCAX_OK;
}

dcax_status dcax_set_submatrix_k(dcax_walker w, int32_t walker, int32_t ks) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (walker < -1 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  if (ks < 1 || ks > KS_MAX) return fail(DCAX_E_INVAL, "submatrix_k must be in 1..64");
  dcax_status st = sync_all(w);
  if (st != DCAX_OK) return st;
  return set_ks(w, walker, ks);
}

}  // extern "C"

namespace {

// Accepted updates per second of sweeps_per_trial generator sweeps of the
// whole batch, timed with HIP events.
dcax_status trial_rate(dcax_walker w, int sweeps_per_trial, double* rate) {
  dcax_status st = sync_all(w);
  if (st != DCAX_OK) return st;
  long long a0 = 0;
  for (const Ctl& h : w->h_ctl) a0 += h.n_acc_ins + h.n_acc_rem;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, w->stream));
  st = sweep_rng(w, sweeps_per_trial);
  if (st != DCAX_OK) return st;
  HIPCHK(hipEventRecord(e1, w->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st = sync_all(w);
  if (st != DCAX_OK) return st;
  long long a1 = 0;
  for (const Ctl& h : w->h_ctl) a1 += h.n_acc_ins + h.n_acc_rem;
  *rate = ms > 0.f ? (double)(a1 - a0) / (ms * 1e-3) : 0.0;
  return DCAX_OK;
}

}  // namespace

extern "C" {

dcax_status dcax_autotune(dcax_walker w, int32_t sweeps_per_trial, int32_t* chosen_ks, double* rate_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (sweeps_per_trial < 1) return fail(DCAX_E_INVAL, "sweeps_per_trial must be >= 1");
  static const int cand[] = {8, 16, 24, 32, 48, 64};
  int best = w->ks_max;
  double best_rate = -1.0;
  for (int ks : cand) {
    st = set_ks(w, -1, ks);
    if (st != DCAX_OK) return st;
    double rate = 0.0;
    st = trial_rate(w, sweeps_per_trial, &rate);
    if (st != DCAX_OK) return st;
    if (rate > best_rate) {
      best_rate = rate;
      best = ks;
    }
  }
  st = set_ks(w, -1, best);
  if (st != DCAX_OK) return st;
  // then the kernel forms of the two candidate products, one after the other
  static const int forms[] = {DCAX_VARIANT_TILED, DCAX_VARIANT_WIDE, DCAX_VARIANT_NARROW};
  for (int which = 0; which < 2; ++which) {
    int best_form = forms[0];
    double best_form_rate = -1.0;
    for (int f : forms) {
      if (which == 0) w->cand_variant = f;
      else w->y_variant = f;
      w->clear_graphs();
      double rate = 0.0;
      st = trial_rate(w, sweeps_per_trial, &rate);
      if (st != DCAX_OK) return st;
      if (rate > best_form_rate) {
        best_form_rate = rate;
        best_form = f;
      }
    }
    best_rate = std::max(best_rate, best_form_rate);
    if (which == 0) w->cand_variant = best_form;
    else w->y_variant = best_form;
    w->clear_graphs();
  }
  if (chosen_ks) *chosen_ks = best;
  if (rate_out) *rate_out = best_rate;
  return DCAX_OK;
}

dcax_status dcax_get_variants(dcax_walker w, int32_t* cand_rows, int32_t* y_columns) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (cand_rows) *cand_rows = w->cand_variant;
  if (y_columns) *y_columns = w->y_variant;
  return DCAX_OK;
}

dcax_status dcax_set_graphs(dcax_walker w, int32_t on) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  dcax_status st = sync_all(w);
  w->use_graphs = on != 0;
  if (!w->use_graphs) w->clear_graphs();
  return st;
}

dcax_status dcax_set_variants(dcax_walker w, int32_t cand_rows, int32_t y_columns) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (cand_rows < DCAX_VARIANT_AUTO || cand_rows > DCAX_VARIANT_NARROW || y_columns < DCAX_VARIANT_AUTO ||
      y_columns > DCAX_VARIANT_NARROW)
    return fail(DCAX_E_INVAL, "unknown kernel variant");
  dcax_status st = sync_all(w);
  w->cand_variant = cand_rows;
  w->y_variant = y_columns;
  w->clear_graphs();       // captured sweeps hold the previous kernels
  return st;
}

dcax_status dcax_set_timing(dcax_walker w, int32_t on) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (on < 0) return fail(DCAX_E_INVAL, "on must be >= 0");
  dcax_status st = sync_all(w);  // drains pending events
  if (w->timing != (on != 0)) w->clear_graphs();
  w->timing = on != 0;
  w->timing_every = on > 0 ? on : 1;
  return st;
}

dcax_status dcax_copy_g0_table(dcax_walker w, int32_t walker, double* host) {
  if (!w || !host) return fail(DCAX_E_INVAL, "NULL argument");
  if (walker < 0 || walker >= w->W) return fail(DCAX_E_INVAL, "walker index out of range");
  const WalkerHost& x = w->wk[walker];
  const double* t = w->mixed ? x.v32.table[0] : x.v64.table[0];
  HIPCHK(hipMemcpyAsync(host, t, sizeof(double) * (size_t)x.geo.Nc * x.p.n_tau, hipMemcpyDeviceToHost, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  return DCAX_OK;
}

}  // extern "C"

// ------------------------------------------------------------- DCA loop
// The self-consistency loop of Sec. 2.1 around a walker handle: the patch
// quadrature is built here, every numerical step runs in the kernels of
// dcax_dca.hip (enqueued on the handle's stream).
struct dcax_dca_s {
  dcax_dca_params p{};
  Geometry geo;
  int P = 0;                       // quadrature points of one patch
  dcax_allocator alloc{};
  hipStream_t stream = nullptr;
  std::vector<void*> blocks;
  DcaDev dev{};
  double* g0 = nullptr;            // [n_spin][Nc][n_cg] complex: the last G0cal of dcax_dca_iterate
  double* gk_tau = nullptr;        // [n_spin][Nc][n_tau] G0cal(K, tau)
  double* tab = nullptr;           // [n_spin][Nc][n_tau] G0cal(r, tau)
  double* G = nullptr;             // [n_spin][Nc][n_freq] complex
  unsigned long long* maxchg = nullptr;
  double* acc = nullptr;           // walker accumulators for dcax_dca_iterate
  double* aux = nullptr;
  long long acc_cap = 0, aux_cap = 0;

  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    void* ptr = alloc.alloc(bytes, alloc.ctx);
    if (ptr) blocks.push_back(ptr);
    return ptr;
  }
  void release() {
    for (void* b : blocks) alloc.free(b, alloc.ctx);
    blocks.clear();
  }
};

namespace {

dcax_status dca_validate(const dcax_dca_params* p) {
  if (p->abi_version != DCAX_ABI_VERSION) return fail(DCAX_E_INVAL, "abi_version mismatch");
  Geometry g;
  if (!build_geometry(p->cluster, g)) return fail(DCAX_E_INVAL, "degenerate or too large cluster");
  if (g.Nc > 1024) return fail(DCAX_E_INVAL, "the DCA loop takes clusters of at most 1024 sites");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(DCAX_E_INVAL, "beta must be positive");
  if (!std::isfinite(p->t) || !std::isfinite(p->tp) || !std::isfinite(p->mu) || !std::isfinite(p->h))
    return fail(DCAX_E_INVAL, "t, tp, mu and h must be finite");
  if (p->n_spin != 1 && p->n_spin != 2) return fail(DCAX_E_INVAL, "n_spin must be 1 or 2");
  if (p->h != 0.0 && p->n_spin != 2) return fail(DCAX_E_INVAL, "a field h != 0 needs n_spin = 2");
  if (p->n_freq < 1) return fail(DCAX_E_INVAL, "n_freq must be >= 1");
  if (p->n_cg < p->n_freq || p->n_cg > (1 << 20)) return fail(DCAX_E_INVAL, "n_cg must be in n_freq .. 2^20");
  if (p->n_tau < 2) return fail(DCAX_E_INVAL, "n_tau must be >= 2");
  if (p->patch_points < 1 || p->patch_points > 256) return fail(DCAX_E_INVAL, "patch_points must be in 1..256");
  if (p->reserved != 0) return fail(DCAX_E_INVAL, "reserved must be 0");
  return DCAX_OK;
}

// Offsets k~ and weights of the standard patch around K = 0 (quadrature rule
// in include/dcax.h).
void patch_quadrature(const int* c, int L, std::vector<double>& kt, std::vector<double>& wt) {
  const double a1x = c[0], a1y = c[1], a2x = c[2], a2y = c[3];
  const double det = a1x * a2y - a1y * a2x;
  const double b1x = 2.0 * M_PI * a2y / det, b1y = -2.0 * M_PI * a2x / det;
  const double b2x = -2.0 * M_PI * a1y / det, b2y = 2.0 * M_PI * a1x / det;
  kt.clear();
  wt.clear();
  for (int j = 0; j < L; ++j)
    for (int i = 0; i < L; ++i) {
      const double fi = (i + 0.5) / L - 0.5, fj = (j + 0.5) / L - 0.5;
      const double ux = fi * b1x + fj * b2x, uy = fi * b1y + fj * b2y;
      double vx[25], vy[25], nv[25], best = 0.0;
      int q = 0;
      for (int n1 = -2; n1 <= 2; ++n1)
        for (int n2 = -2; n2 <= 2; ++n2, ++q) {
          vx[q] = ux + n1 * b1x + n2 * b2x;
          vy[q] = uy + n1 * b1y + n2 * b2y;
          nv[q] = vx[q] * vx[q] + vy[q] * vy[q];
          if (q == 0 || nv[q] < best) best = nv[q];
        }
      int cnt = 0;
      for (q = 0; q < 25; ++q) cnt += nv[q] <= best + 1e-12;
      for (q = 0; q < 25; ++q)
        if (nv[q] <= best + 1e-12) {
          kt.push_back(vx[q]);
          kt.push_back(vy[q]);
          wt.push_back(1.0 / cnt);
        }
    }
}

dcax_status dca_launch_cg(dcax_dca d, const double* sigma, double* gbar, double* g0) {
  hipLaunchKernelGGL(k_dca_coarse_grain, dim3(cdiv(d->p.n_cg, WG), d->geo.Nc, d->p.n_spin), dim3(WG), 0, d->stream,
                     d->dev, sigma, gbar, g0);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dca_launch_tables(dcax_dca d, const double* g0, double* tab) {
  hipLaunchKernelGGL(k_dca_K_tau, dim3(cdiv(d->p.n_tau, WG), d->geo.Nc, d->p.n_spin), dim3(WG), 0, d->stream, d->dev,
                     g0, d->gk_tau);
  hipLaunchKernelGGL(k_dca_table, dim3(cdiv(d->p.n_tau, WG), d->geo.Nc, d->p.n_spin), dim3(WG), 0, d->stream, d->dev,
                     (const double*)d->gk_tau, tab);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dca_launch_sigma(dcax_dca d, const double* g0, const double* G, const double* s_old, double alpha,
                             double* s_new, double* max_change) {
  // the maximum starts at +0.0 (all bits clear), written by a kernel
  hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(WG), 0, d->stream, (double*)d->maxchg, 1LL);
  hipLaunchKernelGGL(k_dca_sigma, dim3(cdiv(d->p.n_freq, WG), d->geo.Nc, d->p.n_spin), dim3(WG), 0, d->stream,
                     d->dev, g0, G, s_old, alpha, s_new, d->maxchg);
  HIPCHK(hipGetLastError());
  if (max_change) {
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, d->maxchg, sizeof(bits), hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
    double v;
    std::memcpy(&v, &bits, sizeof(v));
    *max_change = v;
  }
  return DCAX_OK;
}

// The walkers of a handle fit a DCA handle: same cluster, beta, n_tau,
// n_freq, one table per spin block, and G0(K, i w_n) memory.
dcax_status dca_fits(dcax_dca d, dcax_walker w) {
  for (int i = 0; i < w->W; ++i) {
    const WalkerHost& x = w->wk[i];
    if (std::memcmp(x.p.cluster, d->p.cluster, sizeof(int32_t) * 4) != 0 || x.p.beta != d->p.beta ||
        x.p.n_tau != d->p.n_tau || x.p.n_freq != d->p.n_freq)
      return fail(DCAX_E_INVAL, "walker " + std::to_string(i) + " differs from the DCA handle in cluster, beta, "
                                "n_tau or n_freq");
    if (x.p.n_spin_tables != d->p.n_spin || !x.has_g0Kw)
      return fail(DCAX_E_INVAL, "walker " + std::to_string(i) + " needs g0_tau and g0_Kw with n_spin_tables = n_spin");
  }
  return DCAX_OK;
}

dcax_status set_g0_all(dcax_walker w, const double* tab, int nt, const double* g0kw, int stride) {
  const WalkerHost& x0 = w->wk[0];
  const int Nc = x0.geo.Nc, n_tau = x0.p.n_tau, nf = x0.p.n_freq;
  for (int i = 0; i < w->W; ++i) {
    const WalkerHost& x = w->wk[i];
    if (x.geo.Nc != Nc || x.p.n_tau != n_tau || x.p.n_freq != nf)
      return fail(DCAX_E_INVAL, "the walkers of the handle differ in Nc, n_tau or n_freq");
    if (x.p.n_spin_tables != nt) return fail(DCAX_E_INVAL, "n_spin_tables differs from the walkers' tables");
    if (g0kw && !x.has_g0Kw) return fail(DCAX_E_INVAL, "the walkers were created without g0_Kw");
  }
  if (g0kw && stride < nf) return fail(DCAX_E_INVAL, "g0_Kw_stride < n_freq");
  dcax_status st = sync_all(w);
  if (st != DCAX_OK) return st;
  for (int i = 0; i < w->W; ++i) {
    const WalkerHost& x = w->wk[i];
    const double* vt = w->mixed ? x.v32.table[0] : x.v64.table[0];
    const double* vk = w->mixed ? x.v32.g0Kw : x.v64.g0Kw;
    HIPCHK(hipMemcpyAsync((void*)vt, tab, sizeof(double) * nt * Nc * n_tau, hipMemcpyDeviceToDevice, w->stream));
    if (g0kw && nf > 0)
      HIPCHK(hipMemcpy2DAsync((void*)vk, sizeof(double) * 2 * nf, g0kw, sizeof(double) * 2 * stride,
                              sizeof(double) * 2 * nf, (size_t)nt * Nc, hipMemcpyDeviceToDevice, w->stream));
  }
  // N of the current configurations under the new propagator, and their signs
  const int kmax = w->kmax_host();
  w->fresh = false;
  if (w->mixed) {
    enqueue_refresh<float>(w, 0, w->W, kmax, false);
    hipLaunchKernelGGL(k_set_sign<float>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<float>());
  } else {
    enqueue_refresh<double>(w, 0, w->W, kmax, false);
    hipLaunchKernelGGL(k_set_sign<double>, dim3(1, 1, w->W), dim3(1), 0, w->stream, w->views<double>());
  }
  HIPCHK(hipGetLastError());
  return sync_all(w);
}

}  // namespace

extern "C" {

dcax_status dcax_dca_create(const dcax_dca_params* p, const dcax_allocator* a, void* stream, dcax_dca* out) {
  if (!out) return fail(DCAX_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(DCAX_E_INVAL, "params is NULL");
  dcax_status st = dca_validate(p);
  if (st != DCAX_OK) return st;
  if (!a || !a->alloc || !a->free) return fail(DCAX_E_INVAL, "an allocator with alloc and free is required");
  dcax_dca d = new dcax_dca_s();
  d->p = *p;
  d->alloc = *a;
  d->stream = (hipStream_t)stream;
  build_geometry(p->cluster, d->geo);
  const int Nc = d->geo.Nc, L = p->patch_points;
  std::vector<double> kt, wt;
  patch_quadrature(p->cluster, L, kt, wt);
  d->P = (int)wt.size();
  std::vector<double> eps((size_t)Nc * d->P), epsbar(Nc, 0.0), epsvar(Nc, 0.0), Kr((size_t)Nc * Nc);
  for (int K = 0; K < Nc; ++K)
    for (int q = 0; q < d->P; ++q) {
      const double kx = d->geo.K[2 * K] + kt[2 * q], ky = d->geo.K[2 * K + 1] + kt[2 * q + 1];
      const double cx = std::cos(kx), cy = std::cos(ky);
      eps[(size_t)K * d->P + q] = -2.0 * p->t * (cx + cy) - 4.0 * p->tp * cx * cy;
    }
  for (int r = 0; r < Nc; ++r)
    for (int K = 0; K < Nc; ++K)
      Kr[(size_t)r * Nc + K] = (double)d->geo.sites[2 * r] * d->geo.K[2 * K] +
                               (double)d->geo.sites[2 * r + 1] * d->geo.K[2 * K + 1];
  const int ns = p->n_spin;
  double* e_d = (double*)d->dalloc(sizeof(double) * eps.size());
  double* w_d = (double*)d->dalloc(sizeof(double) * wt.size());
  double* eb_d = (double*)d->dalloc(sizeof(double) * 2 * Nc);      // means, then variances
  double* kr_d = (double*)d->dalloc(sizeof(double) * Kr.size());
  d->g0 = (double*)d->dalloc(sizeof(double) * 2 * ns * Nc * (size_t)p->n_cg);
  d->gk_tau = (double*)d->dalloc(sizeof(double) * ns * Nc * (size_t)p->n_tau);
  d->tab = (double*)d->dalloc(sizeof(double) * ns * Nc * (size_t)p->n_tau);
  d->G = (double*)d->dalloc(sizeof(double) * 2 * ns * Nc * (size_t)p->n_freq);
  d->maxchg = (unsigned long long*)d->dalloc(sizeof(unsigned long long));
  if (!e_d || !w_d || !eb_d || !kr_d || !d->g0 || !d->gk_tau || !d->tab || !d->G || !d->maxchg) {
    d->release();
    delete d;
    return fail(DCAX_E_NOMEM, "device allocation failed");
  }
  // patch means and variances (two passes) of eps, from the eps values the
  // kernels use: the first two moments of G0cal's tail
  for (int K = 0; K < Nc; ++K) {
    double s = 0.0, v = 0.0;
    for (int q = 0; q < d->P; ++q) s += wt[q] * eps[(size_t)K * d->P + q];
    epsbar[K] = s / ((double)L * L);
    for (int q = 0; q < d->P; ++q) {
      const double e = eps[(size_t)K * d->P + q] - epsbar[K];
      v += wt[q] * e * e;
    }
    epsvar[K] = v / ((double)L * L);
  }
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, d->stream);
  };
  if (up(e_d, eps.data(), sizeof(double) * eps.size()) != hipSuccess ||
      up(w_d, wt.data(), sizeof(double) * wt.size()) != hipSuccess ||
      up(eb_d, epsbar.data(), sizeof(double) * Nc) != hipSuccess ||
      up(eb_d + Nc, epsvar.data(), sizeof(double) * Nc) != hipSuccess ||
      up(kr_d, Kr.data(), sizeof(double) * Kr.size()) != hipSuccess ||
      hipStreamSynchronize(d->stream) != hipSuccess) {
    d->release();
    delete d;
    return fail(DCAX_E_HIP, "copying the patch tables failed");
  }
  d->dev = DcaDev{Nc, d->P, p->n_freq, p->n_cg, p->n_tau, ns, p->beta, p->mu, p->h, 1.0 / ((double)L * L),
                  e_d, w_d, eb_d, eb_d + Nc, kr_d};
  *out = d;
  return DCAX_OK;
}

dcax_status dcax_dca_destroy(dcax_dca d) {
  if (!d) return DCAX_OK;
  (void)hipStreamSynchronize(d->stream);
  d->release();
  delete d;
  return DCAX_OK;
}

dcax_status dcax_dca_coarse_grain(dcax_dca d, const double* sigma_dev, double* gbar_dev, double* g0_dev) {
  if (!d || !sigma_dev || !g0_dev) return fail(DCAX_E_INVAL, "NULL argument");
  return dca_launch_cg(d, sigma_dev, gbar_dev, g0_dev);
}

dcax_status dcax_dca_g0_tables(dcax_dca d, const double* g0_dev, double* g0_tau_dev) {
  if (!d || !g0_dev || !g0_tau_dev) return fail(DCAX_E_INVAL, "NULL argument");
  return dca_launch_tables(d, g0_dev, g0_tau_dev);
}

dcax_status dcax_dca_cluster_G(dcax_dca d, const double* g0_dev, const double* acc_dev, const double* aux_dev,
                               int32_t n_blocks, double* G_dev) {
  if (!d || !g0_dev || !acc_dev || !aux_dev || !G_dev) return fail(DCAX_E_INVAL, "NULL argument");
  if (n_blocks < 1) return fail(DCAX_E_INVAL, "n_blocks must be >= 1");
  hipLaunchKernelGGL(k_dca_cluster_G, dim3(cdiv(d->p.n_freq, WG), d->geo.Nc, d->p.n_spin), dim3(WG), 0, d->stream,
                     d->dev, g0_dev, acc_dev, aux_dev, (int)n_blocks, G_dev);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_dca_self_energy(dcax_dca d, const double* g0_dev, const double* G_dev, const double* sigma_old_dev,
                                 double alpha, double* sigma_new_dev, double* max_change_out) {
  if (!d || !g0_dev || !G_dev || !sigma_old_dev || !sigma_new_dev) return fail(DCAX_E_INVAL, "NULL argument");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(DCAX_E_INVAL, "alpha must be in (0, 1]");
  return dca_launch_sigma(d, g0_dev, G_dev, sigma_old_dev, alpha, sigma_new_dev, max_change_out);
}

dcax_status dcax_set_g0(dcax_walker w, const double* g0_tau_dev, int32_t n_spin_tables, const double* g0_Kw_dev,
                        int32_t g0_Kw_stride) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (!g0_tau_dev) return fail(DCAX_E_INVAL, "g0_tau_dev is NULL");
  if (n_spin_tables != 1 && n_spin_tables != 2) return fail(DCAX_E_INVAL, "n_spin_tables must be 1 or 2");
  return set_g0_all(w, g0_tau_dev, n_spin_tables, g0_Kw_dev, g0_Kw_stride);
}

dcax_status dcax_dca_iterate(dcax_dca d, dcax_walker w, int32_t warmup_sweeps, int32_t measure_sweeps, double alpha,
                             double* sigma_dev, double* G_dev, dcax_dca_report* report) {
  if (!d || !sigma_dev) return fail(DCAX_E_INVAL, "NULL argument");
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (warmup_sweeps < 0 || measure_sweeps < 1) return fail(DCAX_E_INVAL, "warmup_sweeps >= 0, measure_sweeps >= 1");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(DCAX_E_INVAL, "alpha must be in (0, 1]");
  st = dca_fits(d, w);
  if (st != DCAX_OK) return st;
  if (d->acc_cap < w->acc_total || d->aux_cap < 3LL * w->W) {
    d->acc = (double*)d->dalloc(sizeof(double) * w->acc_total);
    d->aux = (double*)d->dalloc(sizeof(double) * 3 * w->W);
    if (!d->acc || !d->aux) return fail(DCAX_E_NOMEM, "device allocation failed");
    d->acc_cap = w->acc_total;
    d->aux_cap = 3LL * w->W;
  }
  // G0cal from the current self-energy, installed in every walker
  st = dca_launch_cg(d, sigma_dev, nullptr, d->g0);
  if (st != DCAX_OK) return st;
  st = dca_launch_tables(d, d->g0, d->tab);
  if (st != DCAX_OK) return st;
  HIPCHK(hipStreamSynchronize(d->stream));
  st = set_g0_all(w, d->tab, d->p.n_spin, d->g0, d->p.n_cg);
  if (st != DCAX_OK) return st;
  // the walkers: equilibrate under the new propagator, then measure
  if (warmup_sweeps > 0) {
    st = sweep_rng(w, warmup_sweeps);
    if (st != DCAX_OK) return st;
  }
  hipLaunchKernelGGL(k_fill_zero, dim3(std::min(cdiv(w->acc_total, WG), 1024)), dim3(WG), 0, w->stream, d->acc,
                     (long long)w->acc_total);
  hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(WG), 0, w->stream, d->aux, 3LL * w->W);
  HIPCHK(hipGetLastError());
  st = sweep_rounds(w, measure_sweeps, d->acc, d->aux);
  if (st != DCAX_OK) return st;
  HIPCHK(hipStreamSynchronize(w->stream));
  // cluster G and the new self-energy
  hipLaunchKernelGGL(k_dca_cluster_G, dim3(cdiv(d->p.n_freq, WG), d->geo.Nc, d->p.n_spin), dim3(WG), 0, d->stream,
                     d->dev, (const double*)d->g0, (const double*)d->acc, (const double*)d->aux, (int)w->W, d->G);
  HIPCHK(hipGetLastError());
  double chg = 0.0;
  st = dca_launch_sigma(d, d->g0, d->G, sigma_dev, alpha, sigma_dev, &chg);
  if (st != DCAX_OK) return st;
  if (G_dev)
    HIPCHK(hipMemcpyAsync(G_dev, d->G, sizeof(double) * 2 * d->p.n_spin * d->geo.Nc * d->p.n_freq,
                          hipMemcpyDeviceToDevice, d->stream));
  if (report) {
    std::vector<double> aux(3 * w->W);
    HIPCHK(hipMemcpyAsync(aux.data(), d->aux, sizeof(double) * aux.size(), hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
    st = sync_all(w);
    if (st != DCAX_OK) return st;
    double sg = 0.0, ko = 0.0;
    for (int i = 0; i < w->W; ++i) {
      sg += aux[3 * i];
      ko += w->h_ctl[i].k;
    }
    const long long nmeas = (long long)measure_sweeps * w->W;
    report->max_change = chg;
    report->sign = sg / (double)nmeas;
    report->mean_order = ko / w->W;
    report->measurements = nmeas;
  }
  HIPCHK(hipStreamSynchronize(d->stream));
  return DCAX_OK;
}

}  // extern "C"

// ------------------------------------------------------- two-particle G2
namespace {

constexpr int G2_Q_MAX = 4096;

template <typename T>
dcax_status enqueue_g2(dcax_walker w, int n_w4, int wm, int n_q, double* g2, double* sign_acc) {
  const int W = w->W, Nc = w->wk[0].geo.Nc;
  const int nw = (int)w->g2_nw, n4 = 2 * n_w4;
  hipStream_t s = w->stream;
  // site-sorted M = (e^V - 1) N of every walker (the single-particle measurement's first two steps)
  const View<T>* vs = w->views<T>();
  const int kb1 = std::max(std::min(w->kpad_max, w->kmax_host() + 16 * w->nc_max), 1);
  enqueue_sorted_copy<T>(w, 0);
  const long long per = (long long)nw * Nc * nw, per4 = (long long)n4 * Nc * n4;
  hipLaunchKernelGGL(k_g2_kphase<T>, dim3(cdiv((long long)Nc * Nc, WG)), dim3(WG), 0, s, vs, w->g2);
  for (int i = 0; i < W; ++i) {
    const View<T>* v = w->views<T>(i);
    hipLaunchKernelGGL(k_g2_phase<T>, dim3(cdiv(nw, 64), cdiv(kb1, 4)), dim3(256), 0, s, v, w->g2);
    for (int sp = 0; sp < 2; ++sp) {
      hipLaunchKernelGGL(k_g2_t1m<T>, dim3(cdiv(kb1, G2_RG), Nc, cdiv(nw, 16)), dim3(WG), 0, s, v, sp, w->g2);
      hipLaunchKernelGGL(k_g2_f<T>, dim3(cdiv(per, WG), Nc), dim3(WG), 0, s, v, w->g2);
      hipLaunchKernelGGL(k_g2_k1<T>, dim3(cdiv(per, WG), Nc), dim3(WG), 0, s, v, w->g2);
      hipLaunchKernelGGL(k_g2_g<T>, dim3(cdiv(per, WG), Nc), dim3(WG), 0, s, v, sp, w->g2);
    }
    hipLaunchKernelGGL(k_g2_acc<T>, dim3(cdiv(per4, WG), Nc, n_q), dim3(WG), 0, s, v, w->g2, n4, wm,
                       (const int*)w->g2_q, (const int*)w->g2_dK, (double2*)g2);
    hipLaunchKernelGGL(k_g2_sign<T>, dim3(1), dim3(1), 0, s, v, sign_acc);
  }
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

}  // namespace

extern "C" {

dcax_status dcax_measure_G2(dcax_walker w, int32_t n_w4, int32_t w_transfer, int32_t n_q, const int32_t* q_host,
                            double* g2_dev, double* sign_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (n_w4 < 1 || n_w4 > 64) return fail(DCAX_E_INVAL, "n_w4 must be in 1..64");
  if (w_transfer < 0 || w_transfer > 64) return fail(DCAX_E_INVAL, "w_transfer must be in 0..64");
  if (n_q < 1 || n_q > G2_Q_MAX || !q_host) return fail(DCAX_E_INVAL, "n_q must be in 1..4096 with q_host given");
  if (!g2_dev || !sign_dev) return fail(DCAX_E_INVAL, "NULL accumulator");
  const WalkerHost& x0 = w->wk[0];
  const int Nc = x0.geo.Nc;
  for (int i = 0; i < n_q; ++i)
    if (q_host[i] < 0 || q_host[i] >= Nc) return fail(DCAX_E_INVAL, "a transfer momentum index is out of range");
  for (const auto& x : w->wk) {
    if (std::memcmp(x.p.cluster, x0.p.cluster, sizeof(int32_t) * 4) != 0 || x.p.beta != x0.p.beta)
      return fail(DCAX_E_INVAL, "the walkers of the handle differ in cluster or beta");
    if (x.p.n_spin_tables > 0 && (!x.has_g0Kw || x.p.n_freq < n_w4 + w_transfer))
      return fail(DCAX_E_INVAL, "walkers with a caller's propagator need g0_Kw with n_freq >= n_w4 + w_transfer");
  }
  const size_t nw = 2 * (size_t)n_w4 + w_transfer, kpad = (size_t)w->kpad_max;
  if (nw > w->g2_nw || kpad > w->g2_kpad || (size_t)Nc > w->g2_nc) {
    const size_t nn = std::max(nw, w->g2_nw), kk = std::max(kpad, w->g2_kpad), cc = std::max((size_t)Nc, w->g2_nc);
    const size_t sq = cc * nn * cc * nn;
    G2Dev g{};
    g.P = (double2*)w->dalloc(sizeof(double2) * kk * nn);
    g.T1 = (double2*)w->dalloc(sizeof(double2) * cc * nn * kk);
    g.F = (double2*)w->dalloc(sizeof(double2) * sq);
    g.H = (double2*)w->dalloc(sizeof(double2) * sq);
    g.G[0] = (double2*)w->dalloc(sizeof(double2) * sq);
    g.G[1] = (double2*)w->dalloc(sizeof(double2) * sq);
    g.ph = (double2*)w->dalloc(sizeof(double2) * cc * cc);
    if (!w->g2_q) w->g2_q = (int*)w->dalloc(sizeof(int) * G2_Q_MAX);
    if (!g.P || !g.T1 || !g.F || !g.H || !g.G[0] || !g.G[1] || !g.ph || !w->g2_q)
      return fail(DCAX_E_NOMEM, "device allocation failed (two-particle scratch)");
    w->g2 = g;
    w->g2_nw = nn;
    w->g2_kpad = kk;
    w->g2_nc = cc;
  }
  w->g2.nw = (int)nw;
  w->g2.n_lo = -n_w4;
  w->g2.kpad = (int)w->g2_kpad;
  if (w->g2_dK_nc != Nc) {
    // K_a - K_b from the integer momenta q = K |det A| / (2 pi)
    const long long D = std::llabs((long long)x0.p.cluster[0] * x0.p.cluster[3] - (long long)x0.p.cluster[1] * x0.p.cluster[2]);
    std::vector<long long> qx(Nc), qy(Nc);
    for (int a = 0; a < Nc; ++a) {
      qx[a] = std::llround(x0.geo.K[2 * a] * (double)D / (2.0 * M_PI));
      qy[a] = std::llround(x0.geo.K[2 * a + 1] * (double)D / (2.0 * M_PI));
    }
    std::vector<int> dk((size_t)Nc * Nc, -1);
    for (int a = 0; a < Nc; ++a)
      for (int b = 0; b < Nc; ++b) {
        const long long dx = ((qx[a] - qx[b]) % D + D) % D, dy = ((qy[a] - qy[b]) % D + D) % D;
        for (int c = 0; c < Nc; ++c)
          if (qx[c] == dx && qy[c] == dy) dk[(size_t)a * Nc + b] = c;
        if (dk[(size_t)a * Nc + b] < 0) return fail(DCAX_E_INVAL, "momentum difference outside the cluster");
      }
    w->g2_dK = (int*)w->dalloc(sizeof(int) * dk.size());
    if (!w->g2_dK) return fail(DCAX_E_NOMEM, "device allocation failed");
    HIPCHK(hipMemcpyAsync(w->g2_dK, dk.data(), sizeof(int) * dk.size(), hipMemcpyHostToDevice, w->stream));
    w->g2_dK_nc = Nc;
  }
  HIPCHK(hipMemcpyAsync(w->g2_q, q_host, sizeof(int) * n_q, hipMemcpyHostToDevice, w->stream));
  st = w->mixed ? enqueue_g2<float>(w, n_w4, w_transfer, n_q, g2_dev, sign_dev)
                : enqueue_g2<double>(w, n_w4, w_transfer, n_q, g2_dev, sign_dev);
  if (st != DCAX_OK) return st;
  // the transfers were copied from the caller's host array: wait before returning
  HIPCHK(hipStreamSynchronize(w->stream));
  return DCAX_OK;
}

}  // extern "C"

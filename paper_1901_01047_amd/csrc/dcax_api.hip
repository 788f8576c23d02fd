// Host side of the C ABI declared in include/dcax.h.
//
// All kernels are compiled into this one translation unit.  The host never
// reads device state inside a sweep: every window's kernels take their sizes
// from the device control block, and grids are sized by a host-side upper
// bound of the order.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dcax_dev.h"
#include "dcax_window.hip"
#include "dcax_refresh.hip"
#include "dcax_measure.hip"

using namespace dcax;

namespace {

thread_local std::string g_err;

dcax_status fail(dcax_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(DCAX_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

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

__global__ void k_set_cursor(Ctl* c, long long pos, long long end) {
  c->pos = pos;
  c->end = end;
}

// A sweep is max(k, 1) proposals rounded up to a multiple of k_s, with k the
// order at the sweep's start.
__global__ void k_begin_sweep(Ctl* c, int ks) {
  if (c->status != 0) return;
  const long long k = c->k > 1 ? c->k : 1;
  c->end = c->pos + ((k + ks - 1) / ks) * ks;
}

}  // namespace

struct dcax_walker_s {
  dcax_params p{};
  dcax_allocator alloc{};
  bool have_alloc = false;
  hipStream_t stream = nullptr;
  bool mixed = false;
  Geometry geo;
  int ks = 0, cap = 0, ld = 0, max_order = 0;
  double gamma = 0.0;
  std::vector<void*> blocks;
  bool latched = false;
  int k_host = 0;  // order at the last synchronisation
  long long sweeps_done = 0;
  double last_drift = 0.0, max_drift = 0.0;
  // live kernel timing (dcax_set_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pend_fold, pend_accept, pend_window;
  double fold_s = 0.0, accept_s = 0.0, window_s = 0.0;
  long long fold_launches = 0;

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
  }

  // device buffers
  Ctl* ctl = nullptr;
  int* diff = nullptr;
  double* table = nullptr;
  int* sites_d = nullptr;
  double* K_d = nullptr;
  double* xi_d = nullptr;
  void* N[2] = {nullptr, nullptr};
  void* R[2] = {nullptr, nullptr};
  int* el_row = nullptr;
  int* remap = nullptr;
  int* moves = nullptr;
  dcax_proposal* replay_d = nullptr;
  double* ratio_d = nullptr;
  long long replay_cap = 0;
  // refresh scratch
  double* M[2] = {nullptr, nullptr};
  double* P[2] = {nullptr, nullptr};
  double* Tm[2] = {nullptr, nullptr};
  int* ipiv = nullptr;   // [2][cap]
  int* perm = nullptr;   // [2][cap]
  double* blkmax = nullptr;
  size_t blkmax_len = 0;
  double* detsign = nullptr;
  // measurement scratch
  MeasureBufs meas;

  View<double> v64{};
  View<float> v32{};

  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    void* ptr = nullptr;
    if (have_alloc) {
      ptr = alloc.alloc(bytes, alloc.ctx);
    } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
      ptr = nullptr;
    }
    if (ptr) blocks.push_back(ptr);
    return ptr;
  }
  void release() {
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
    ev_pool.clear();
    for (void* b : blocks) {
      if (have_alloc) alloc.free(b, alloc.ctx);
      else hipFree(b);
    }
    blocks.clear();
  }
};

namespace {

dcax_status measure_alloc(dcax_walker w, MeasureBufs& mb, int Nc, int n_freq, int cap);
dcax_status sweep_rng(dcax_walker w, int n_sweeps);

template <typename T>
View<T>& view(dcax_walker w);
template <>
View<double>& view<double>(dcax_walker w) { return w->v64; }
template <>
View<float>& view<float>(dcax_walker w) { return w->v32; }

dcax_status validate(const dcax_params* p) {
  if (!p) return fail(DCAX_E_INVAL, "params is NULL");
  if (p->abi_version != DCAX_ABI_VERSION) return fail(DCAX_E_INVAL, "abi_version mismatch");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(DCAX_E_INVAL, "beta must be positive");
  if (!(p->U >= 0.0) || !std::isfinite(p->U)) return fail(DCAX_E_INVAL, "U must be >= 0");
  if (!(p->K_exp > 0.0) || !std::isfinite(p->K_exp)) return fail(DCAX_E_INVAL, "K_exp must be positive");
  if (!std::isfinite(p->t) || !std::isfinite(p->tp) || !std::isfinite(p->mu)) return fail(DCAX_E_INVAL, "non-finite hopping or mu");
  if (p->n_tau < 2 || p->n_tau > (1 << 22)) return fail(DCAX_E_INVAL, "n_tau out of range");
  if (p->precision != DCAX_FP64 && p->precision != DCAX_FP32_MIXED) return fail(DCAX_E_INVAL, "unknown precision");
  if (p->submatrix_k < 1 || p->submatrix_k > KS_MAX) return fail(DCAX_E_INVAL, "submatrix_k must be in 1..64");
  if (p->refresh_every < 0) return fail(DCAX_E_INVAL, "refresh_every must be >= 0");
  if (p->max_order < 1 || p->max_order > 32768) return fail(DCAX_E_INVAL, "max_order must be in 1..32768");
  if (p->n_freq < 0 || p->n_freq > 65536) return fail(DCAX_E_INVAL, "n_freq out of range");
  Geometry g;
  if (!build_geometry(p->cluster, g)) return fail(DCAX_E_INVAL, "degenerate or too large cluster");
  return DCAX_OK;
}

template <typename T>
void fill_view(dcax_walker w) {
  View<T>& v = view<T>(w);
  v.Nc = w->geo.Nc;
  v.n_tau = w->p.n_tau;
  v.ks = w->ks;
  v.cap = w->cap;
  v.ld = w->ld;
  v.max_order = w->max_order;
  v.beta = w->p.beta;
  v.h = w->p.beta / (double)(w->p.n_tau - 1);
  v.gamma = w->gamma;
  v.K_exp = w->p.K_exp;
  for (int sp = 0; sp < 2; ++sp) {
    const double sig = sp == 0 ? 1.0 : -1.0;
    v.ev[sp][0] = std::exp(sig * w->gamma);
    v.ev[sp][1] = std::exp(-sig * w->gamma);
  }
  v.diff = w->diff;
  v.table = w->table;
  v.ctl = w->ctl;
  v.N[0] = (T*)w->N[0];
  v.N[1] = (T*)w->N[1];
  v.ratio_out = w->ratio_d;
  v.replay = w->replay_d;
}

dcax_status check_latched(dcax_walker w) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (w->latched) return fail(DCAX_E_STATE, "walker holds a latched error; call dcax_set_config");
  return DCAX_OK;
}

dcax_status sync_ctl(dcax_walker w, Ctl* h) {
  HIPCHK(hipMemcpyAsync(h, w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  w->drain_events();
  w->k_host = h->k;
  if (h->status != ST_OK) {
    w->latched = true;
    switch (h->status) {
      case ST_NUMERIC: return fail(DCAX_E_NUMERIC, "non-finite ratio or zero pivot");
      case ST_CAPACITY: return fail(DCAX_E_CAPACITY, "expansion order would exceed max_order");
      case ST_TRACE: return fail(DCAX_E_TRACE, "replay names a vertex id that is not present");
      default: return fail(DCAX_E_NUMERIC, "latched device error");
    }
  }
  return DCAX_OK;
}

template <typename T>
void enqueue_window(dcax_walker w, int kb, bool replay) {
  View<T>& v = view<T>(w);
  hipStream_t s = w->stream;
  const int ks = w->ks;
  const int kx = std::min(kb + ks, w->cap);
  T* R0 = (T*)w->R[0];
  T* R1 = (T*)w->R[1];
  hipEvent_t e_w0 = nullptr, e_a0 = nullptr, e_a1 = nullptr, e_f0 = nullptr, e_f1 = nullptr;
  if (w->timing) {
    e_w0 = w->ev();
    if (e_w0) hipEventRecord(e_w0, s);
  }
  if (replay) hipLaunchKernelGGL(k_prep_replay<T>, dim3(1), dim3(WG), 0, s, v);
  else hipLaunchKernelGGL(k_prep_rng<T>, dim3(1), dim3(WG), 0, s, v, w->p.seed);
  hipLaunchKernelGGL(k_gather<T>, dim3(cdiv(std::max(kb, 1), WG), ks), dim3(WG), 0, s, v, R0, R1);
  hipLaunchKernelGGL(k_cand_x<T>, dim3(cdiv(std::max(kb, 1), 64), 2), dim3(WG), 0, s, v, R0, R1);
  hipLaunchKernelGGL(k_gram<T>, dim3(ks, 2), dim3(WG), 0, s, v, (const T*)R0, (const T*)R1);
  if (w->timing) {
    e_a0 = w->ev();
    if (e_a0) hipEventRecord(e_a0, s);
  }
  hipLaunchKernelGGL(k_accept<T>, dim3(1), dim3(WG), 0, s, v, w->el_row, (uint64_t)w->p.seed);
  if (w->timing) {
    e_a1 = w->ev();
    if (e_a1) hipEventRecord(e_a1, s);
    w->pend_accept.push_back({e_a0, e_a1});
  }
  hipLaunchKernelGGL(k_ygemm<T>, dim3(cdiv(std::max(kb, 1), 64), 2), dim3(WG), 0, s, v);
  hipLaunchKernelGGL(k_fold_prep<T>, dim3(cdiv(kx, WG), 2), dim3(WG), 0, s, v, (const T*)R0, (const T*)R1,
                     (const int*)w->el_row);
  FoldArgs<T> f;
  for (int sp = 0; sp < 2; ++sp) {
    f.C[sp] = v.N[sp];
    f.A[sp] = v.A[sp];
    f.B[sp] = v.B[sp];
  }
  f.ldc = w->ld;
  f.lda = w->cap;
  f.ldb = w->cap;
  f.M = f.N = f.K = 0;
  f.ctl = w->ctl;
  if (w->timing) {
    e_f0 = w->ev();
    if (e_f0) hipEventRecord(e_f0, s);
  }
  hipLaunchKernelGGL(k_fold<T>, dim3(cdiv(kx, 64), cdiv(kx, 64), 2), dim3(WG), 0, s, f);
  if (w->timing) {
    e_f1 = w->ev();
    if (e_f1) hipEventRecord(e_f1, s);
    w->pend_fold.push_back({e_f0, e_f1});
  }
  hipLaunchKernelGGL(k_compact_plan<T>, dim3(1), dim3(WG), 0, s, v, w->remap, w->moves);
  hipLaunchKernelGGL(k_compact_move<T>, dim3(cdiv(kx, WG), KS_MAX, 2), dim3(WG), 0, s, v, (const int*)w->remap,
                     (const int*)w->moves);
  hipLaunchKernelGGL(k_window_end<T>, dim3(1), dim3(64), 0, s, v);
  if (w->timing) {
    hipEvent_t e_w1 = w->ev();
    if (e_w1) hipEventRecord(e_w1, s);
    w->pend_window.push_back({e_w0, e_w1});
  }
}

// FP64 refresh of N (both spins).  Returns the drift through *drift.
template <typename T>
dcax_status refresh_impl(dcax_walker w, double* drift, bool measure_drift) {
  Ctl h;
  dcax_status st = sync_ctl(w, &h);
  if (st != DCAX_OK) return st;
  const int k = h.k;
  double one[2] = {1.0, 1.0};
  HIPCHK(hipMemcpyAsync(w->detsign, one, sizeof(one), hipMemcpyHostToDevice, w->stream));
  if (k == 0) {
    if (drift) *drift = 0.0;
    HIPCHK(hipStreamSynchronize(w->stream));
    return DCAX_OK;
  }
  View<T>& v = view<T>(w);
  hipStream_t s = w->stream;
  const int ldm = w->cap;
  hipLaunchKernelGGL(k_build_ninv<T>, dim3(cdiv(k, WG), k), dim3(WG), 0, s, v, w->M[0], w->M[1], k, ldm);
  for (int p0 = 0; p0 < k; p0 += NB) {
    const int nb = std::min(NB, k - p0);
    hipLaunchKernelGGL(k_gj_panel, dim3(2), dim3(WG), 0, s, w->M[0], w->M[1], k, ldm, p0, nb, w->ipiv,
                       w->ipiv + w->cap, w->ctl, w->detsign);
    hipLaunchKernelGGL(k_gj_prep, dim3(cdiv(k, WG), 2), dim3(WG), 0, s, w->M[0], w->M[1], k, ldm, p0, nb,
                       (const int*)w->ipiv, (const int*)(w->ipiv + w->cap), w->P[0], w->P[1], w->Tm[0],
                       w->Tm[1], w->cap);
    FoldArgs<double> f;
    for (int sp = 0; sp < 2; ++sp) {
      f.C[sp] = w->M[sp];
      f.A[sp] = w->P[sp];
      f.B[sp] = w->Tm[sp];
    }
    f.ldc = ldm;
    f.lda = w->cap;
    f.ldb = w->cap;
    f.M = f.N = k;
    f.K = nb;
    f.ctl = nullptr;
    hipLaunchKernelGGL(k_fold<double>, dim3(cdiv(k, 64), cdiv(k, 64), 2), dim3(WG), 0, s, f);
  }
  // column permutation from the row interchanges
  std::vector<int> ip(2 * (size_t)w->cap);
  HIPCHK(hipMemcpyAsync(ip.data(), w->ipiv, sizeof(int) * 2 * w->cap, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int> perm(2 * (size_t)w->cap);
  for (int sp = 0; sp < 2; ++sp) {
    int* col_of = perm.data() + (size_t)sp * w->cap;
    const int* piv = ip.data() + (size_t)sp * w->cap;
    for (int j = 0; j < k; ++j) col_of[j] = j;
    for (int c = k - 1; c >= 0; --c) {
      const int q = piv[c];
      if (q < 0 || q >= k) return fail(DCAX_E_NUMERIC, "pivot index out of range");
      std::swap(col_of[c], col_of[q]);
    }
  }
  HIPCHK(hipMemcpyAsync(w->perm, perm.data(), sizeof(int) * 2 * w->cap, hipMemcpyHostToDevice, s));
  const dim3 grid(cdiv(k, WG), k, 2);
  const size_t nblk = (size_t)grid.x * grid.y * grid.z;
  if (nblk > w->blkmax_len) return fail(DCAX_E_INVAL, "refresh scratch too small");
  hipLaunchKernelGGL(k_refresh_store<T>, grid, dim3(WG), 0, s, v, (const double*)w->M[0], (const double*)w->M[1],
                     k, ldm, (const int*)w->perm, (const int*)(w->perm + w->cap), w->blkmax, measure_drift ? 1 : 0);
  std::vector<double> bm(2 * nblk);
  HIPCHK(hipMemcpyAsync(bm.data(), w->blkmax, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, s));
  st = sync_ctl(w, &h);
  if (st != DCAX_OK) return st;
  double dmax = 0.0, nmax = 0.0;
  for (size_t b = 0; b < nblk; ++b) {
    dmax = std::max(dmax, bm[2 * b]);
    nmax = std::max(nmax, bm[2 * b + 1]);
  }
  if (drift) *drift = nmax > 0.0 ? dmax / nmax : 0.0;
  return DCAX_OK;
}

dcax_status refresh_any(dcax_walker w, double* drift, bool measure) {
  return w->mixed ? refresh_impl<float>(w, drift, measure) : refresh_impl<double>(w, drift, measure);
}

template <typename T>
void wire_window_buffers(dcax_walker w, char*& base) {
  View<T>& v = view<T>(w);
  auto take = [&](size_t bytes) {
    char* p = base;
    base += (bytes + 255) & ~size_t(255);
    return (void*)p;
  };
  const size_t ks = w->ks, cap = w->cap;
  v.v_site = (int*)take(sizeof(int) * cap);
  v.v_tau = (double*)take(sizeof(double) * cap);
  v.v_s = (int*)take(sizeof(int) * cap);
  v.v_id = (long long*)take(sizeof(long long) * cap);
  v.wp = (WinProp*)take(sizeof(WinProp) * KS_MAX);
  v.el_site = (int*)take(sizeof(int) * KS_MAX);
  v.el_tau = (double*)take(sizeof(double) * KS_MAX);
  v.el_s = (int*)take(sizeof(int) * KS_MAX);
  v.el_slot = (int*)take(sizeof(int) * KS_MAX);
  v.el_cand = (int*)take(sizeof(int) * KS_MAX);
  v.cand_el = (int*)take(sizeof(int) * KS_MAX);
  v.cand_id = (long long*)take(sizeof(long long) * KS_MAX);
  v.S = (int*)take(sizeof(int) * KS_MAX);
  v.ins_el = (int*)take(sizeof(int) * KS_MAX);
  v.gcol = (T*)take(sizeof(T) * ks * cap);
  v.gCC = (double*)take(sizeof(double) * KS_MAX * KS_MAX);
  for (int sp = 0; sp < 2; ++sp) {
    v.W[sp] = (T*)take(sizeof(T) * ks * cap);
    v.X[sp] = nullptr;
    v.gram[sp] = (double*)take(sizeof(double) * KS_MAX * KS_MAX);
    v.ginv[sp] = (double*)take(sizeof(double) * KS_MAX * KS_MAX);
    v.Y[sp] = (T*)take(sizeof(T) * ks * cap);
    v.A[sp] = (T*)take(sizeof(T) * KS_MAX * cap);
    v.B[sp] = (T*)take(sizeof(T) * KS_MAX * cap);
    w->R[sp] = take(sizeof(T) * KS_MAX * cap);
  }
}

template <typename T>
size_t window_bytes(size_t ks, size_t cap) {
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  add(sizeof(int) * cap);
  add(sizeof(double) * cap);
  add(sizeof(int) * cap);
  add(sizeof(long long) * cap);
  add(sizeof(WinProp) * KS_MAX);
  for (int i = 0; i < 4; ++i) add(sizeof(int) * KS_MAX);
  add(sizeof(double) * KS_MAX);
  add(sizeof(int) * KS_MAX);
  add(sizeof(long long) * KS_MAX);
  add(sizeof(int) * KS_MAX);
  add(sizeof(int) * KS_MAX);
  add(sizeof(T) * ks * cap);
  add(sizeof(double) * KS_MAX * KS_MAX);
  for (int sp = 0; sp < 2; ++sp) {
    add(sizeof(T) * ks * cap);
    add(sizeof(double) * KS_MAX * KS_MAX);
    add(sizeof(double) * KS_MAX * KS_MAX);
    add(sizeof(T) * ks * cap);
    add(sizeof(T) * KS_MAX * cap);
    add(sizeof(T) * KS_MAX * cap);
    add(sizeof(T) * KS_MAX * cap);
  }
  return b + 4096;
}

template <typename T>
dcax_status create_buffers(dcax_walker w) {
  const size_t cap = w->cap, ld = w->ld;
  const int Nc = w->geo.Nc;
  w->ctl = (Ctl*)w->dalloc(sizeof(Ctl));
  w->diff = (int*)w->dalloc(sizeof(int) * Nc * Nc);
  w->table = (double*)w->dalloc(sizeof(double) * (size_t)Nc * w->p.n_tau);
  w->sites_d = (int*)w->dalloc(sizeof(int) * 2 * Nc);
  w->K_d = (double*)w->dalloc(sizeof(double) * 2 * Nc);
  w->xi_d = (double*)w->dalloc(sizeof(double) * Nc);
  for (int sp = 0; sp < 2; ++sp) w->N[sp] = w->dalloc(sizeof(T) * ld * cap);
  char* base = (char*)w->dalloc(window_bytes<T>(w->ks, cap));
  w->el_row = (int*)w->dalloc(sizeof(int) * KS_MAX);
  w->remap = (int*)w->dalloc(sizeof(int) * cap);
  w->moves = (int*)w->dalloc(sizeof(int) * (2 * KS_MAX + 1));
  for (int sp = 0; sp < 2; ++sp) {
    w->M[sp] = (double*)w->dalloc(sizeof(double) * cap * cap);
    w->P[sp] = (double*)w->dalloc(sizeof(double) * cap * NB);
    w->Tm[sp] = (double*)w->dalloc(sizeof(double) * cap * NB);
  }
  w->ipiv = (int*)w->dalloc(sizeof(int) * 2 * cap);
  w->perm = (int*)w->dalloc(sizeof(int) * 2 * cap);
  w->blkmax_len = (size_t)cdiv(cap, WG) * cap * 2;
  w->blkmax = (double*)w->dalloc(sizeof(double) * 2 * w->blkmax_len);
  w->detsign = (double*)w->dalloc(sizeof(double) * 2);
  if (!w->ctl || !w->diff || !w->table || !w->sites_d || !w->K_d || !w->xi_d || !w->N[0] || !w->N[1] || !base ||
      !w->el_row || !w->remap || !w->moves || !w->M[0] || !w->M[1] || !w->P[0] || !w->P[1] || !w->Tm[0] ||
      !w->Tm[1] || !w->ipiv || !w->perm || !w->blkmax || !w->detsign)
    return fail(DCAX_E_NOMEM, "device allocation failed");
  fill_view<T>(w);
  wire_window_buffers<T>(w, base);
  dcax_status st = measure_alloc(w, w->meas, Nc, w->p.n_freq, (int)cap);
  if (st != DCAX_OK) return st;
  return DCAX_OK;
}

dcax_status reset_ctl(dcax_walker w, int k, long long next_id, double sign) {
  Ctl h;
  std::memset(&h, 0, sizeof(h));
  h.k = k;
  h.next_id = next_id;
  h.sign = sign;
  h.carry_id = -1;
  HIPCHK(hipMemcpyAsync(w->ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  w->k_host = k;
  return DCAX_OK;
}

dcax_status measure_alloc(dcax_walker w, MeasureBufs& mb, int Nc, int n_freq, int cap) {
  const size_t es = w->mixed ? sizeof(float) : sizeof(double);
  mb.kpad_cap = cap + 16 * Nc;
  mb.n_freq = n_freq;
  const size_t kp = mb.kpad_cap, nf = std::max(n_freq, 1);
  mb.order = (int*)w->dalloc(sizeof(int) * kp);
  mb.off = (int*)w->dalloc(sizeof(int) * (Nc + 1));
  mb.E = w->dalloc(es * 2 * kp * nf);
  for (int sp = 0; sp < 2; ++sp) {
    mb.Ms[sp] = w->dalloc(es * kp * kp);
    mb.Mab[sp] = (double*)w->dalloc(sizeof(double) * 2 * (size_t)Nc * Nc * nf);
  }
  if (!mb.order || !mb.off || !mb.E || !mb.Ms[0] || !mb.Ms[1] || !mb.Mab[0] || !mb.Mab[1])
    return fail(DCAX_E_NOMEM, "measurement buffer allocation failed");
  return DCAX_OK;
}

template <typename T>
void enqueue_measure(dcax_walker w, double* acc, double* aux) {
  View<T>& v = view<T>(w);
  hipStream_t s = w->stream;
  MeasureBufs& mb = w->meas;
  const int Nc = w->geo.Nc, nf = w->p.n_freq;
  const int kb = std::min(mb.kpad_cap, w->k_host + 16 * Nc);
  hipLaunchKernelGGL(k_meas_diag<T>, dim3(2), dim3(WG), 0, s, v, aux);
  if (nf == 0) return;
  hipLaunchKernelGGL(k_meas_sort<T>, dim3(1), dim3(WG), sizeof(int) * (Nc + 1), s, v, mb.order, mb.off, mb.kpad_cap);
  hipLaunchKernelGGL(k_meas_copy<T>, dim3(cdiv(kb, WG), kb), dim3(WG), 0, s, v, (const int*)mb.order,
                     (const int*)mb.off, (T*)mb.Ms[0], (T*)mb.Ms[1], mb.kpad_cap);
  hipLaunchKernelGGL(k_meas_phase<T>, dim3(cdiv(nf, WG), kb), dim3(WG), 0, s, v, (const int*)mb.order,
                     (const int*)mb.off, (T*)mb.E, nf);
  hipLaunchKernelGGL(k_meas_block<T>, dim3(Nc * Nc, cdiv(nf, 16), 2), dim3(64), 0, s, v, (const int*)mb.order,
                     (const int*)mb.off, (const T*)mb.Ms[0], (const T*)mb.Ms[1], mb.kpad_cap, (const T*)mb.E, nf,
                     mb.Mab[0], mb.Mab[1]);
  hipLaunchKernelGGL(k_meas_K<T>, dim3(cdiv(nf, WG), Nc, 2), dim3(WG), 0, s, v, (const int*)w->sites_d,
                     (const double*)w->K_d, (const double*)mb.Mab[0], (const double*)mb.Mab[1], nf, acc);
}

dcax_status sweep_rng(dcax_walker w, int n_sweeps) {
  Ctl h;
  dcax_status st = sync_ctl(w, &h);
  if (st != DCAX_OK) return st;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    hipLaunchKernelGGL(k_begin_sweep, dim3(1), dim3(1), 0, w->stream, w->ctl, w->ks);
    const int nwin = cdiv(std::max(h.k, 1), w->ks);
    int kb = h.k;
    for (int i = 0; i < nwin; ++i) {
      kb = std::min(w->max_order, kb + w->ks);
      if (w->mixed) enqueue_window<float>(w, kb, false);
      else enqueue_window<double>(w, kb, false);
    }
    HIPCHK(hipGetLastError());
    st = sync_ctl(w, &h);
    if (st != DCAX_OK) return st;
    // windows closed early by a carried removal leave proposals of the sweep
    while (h.pos < h.end) {
      const int kb2 = std::min(w->max_order, h.k + w->ks);
      if (w->mixed) enqueue_window<float>(w, kb2, false);
      else enqueue_window<double>(w, kb2, false);
      st = sync_ctl(w, &h);
      if (st != DCAX_OK) return st;
    }
    ++w->sweeps_done;
    if (w->p.refresh_every > 0 && w->sweeps_done % w->p.refresh_every == 0) {
      double d = 0.0;
      st = refresh_any(w, &d, true);
      if (st != DCAX_OK) return st;
      w->last_drift = d;
      w->max_drift = std::max(w->max_drift, d);
      st = sync_ctl(w, &h);
      if (st != DCAX_OK) return st;
    }
  }
  return DCAX_OK;
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
  dcax_status st = validate(p);
  if (st != DCAX_OK) return st;
  if (n_walkers != 1) return fail(DCAX_E_INVAL, "n_walkers must be 1");
  if (a && (!a->alloc || !a->free)) return fail(DCAX_E_INVAL, "allocator needs alloc and free");
  dcax_walker w = new dcax_walker_s();
  w->p = *p;
  if (a) {
    w->alloc = *a;
    w->have_alloc = true;
  }
  w->stream = (hipStream_t)stream;
  w->mixed = p->precision == DCAX_FP32_MIXED;
  build_geometry(p->cluster, w->geo);
  w->ks = p->submatrix_k;
  w->max_order = p->max_order;
  w->cap = ((p->max_order + w->ks + 63) / 64) * 64;
  w->ld = w->cap;
  w->gamma = std::acosh(1.0 + p->U * p->beta * (double)w->geo.Nc / (2.0 * p->K_exp));
  st = w->mixed ? create_buffers<float>(w) : create_buffers<double>(w);
  if (st != DCAX_OK) {
    w->release();
    delete w;
    return st;
  }
  // cluster tables and the G0(r, tau) table
  const int Nc = w->geo.Nc;
  std::vector<double> xi(Nc);
  for (int q = 0; q < Nc; ++q) {
    const double cx = std::cos(w->geo.K[2 * q]), cy = std::cos(w->geo.K[2 * q + 1]);
    xi[q] = -2.0 * p->t * (cx + cy) - 4.0 * p->tp * cx * cy - p->mu;
  }
  auto cleanup = [&](dcax_status s) {
    w->release();
    delete w;
    return s;
  };
#define HIPCHK_C(x)                                                                                \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) return cleanup(fail(DCAX_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_))); \
  } while (0)
  HIPCHK_C(hipMemcpyAsync(w->diff, w->geo.diff.data(), sizeof(int) * Nc * Nc, hipMemcpyHostToDevice, w->stream));
  HIPCHK_C(hipMemcpyAsync(w->sites_d, w->geo.sites.data(), sizeof(int) * 2 * Nc, hipMemcpyHostToDevice, w->stream));
  HIPCHK_C(hipMemcpyAsync(w->K_d, w->geo.K.data(), sizeof(double) * 2 * Nc, hipMemcpyHostToDevice, w->stream));
  HIPCHK_C(hipMemcpyAsync(w->xi_d, xi.data(), sizeof(double) * Nc, hipMemcpyHostToDevice, w->stream));
  hipLaunchKernelGGL(k_g0_table, dim3(cdiv(p->n_tau, WG), Nc), dim3(WG), 0, w->stream, w->table, Nc, p->n_tau,
                     p->beta, (const int*)w->sites_d, (const double*)w->K_d, (const double*)w->xi_d);
  HIPCHK_C(hipGetLastError());
  st = reset_ctl(w, 0, 0, 1.0);
  if (st != DCAX_OK) return cleanup(st);
#undef HIPCHK_C
  *out = w;
  return DCAX_OK;
}

dcax_status dcax_walker_destroy(dcax_walker w) {
  if (!w) return DCAX_OK;
  if (w->stream || true) hipStreamSynchronize(w->stream);
  w->release();
  delete w;
  return DCAX_OK;
}

dcax_status dcax_set_config(dcax_walker w, const dcax_vertex* v, int32_t k) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  if (k < 0 || k > w->max_order || (k > 0 && !v)) return fail(DCAX_E_INVAL, "bad configuration size");
  std::vector<int> site(k), s(k);
  std::vector<double> tau(k);
  std::vector<long long> id(k);
  long long next_id = 0;
  for (int i = 0; i < k; ++i) {
    if (v[i].site < 0 || v[i].site >= w->geo.Nc) return fail(DCAX_E_INVAL, "vertex site out of range");
    if (v[i].aux_spin != 1 && v[i].aux_spin != -1) return fail(DCAX_E_INVAL, "aux_spin must be +1 or -1");
    if (!(v[i].tau >= 0.0 && v[i].tau < w->p.beta)) return fail(DCAX_E_INVAL, "tau must be in [0, beta)");
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
  int* vs = w->mixed ? w->v32.v_site : w->v64.v_site;
  double* vt = w->mixed ? w->v32.v_tau : w->v64.v_tau;
  int* vsp = w->mixed ? w->v32.v_s : w->v64.v_s;
  long long* vid = w->mixed ? w->v32.v_id : w->v64.v_id;
  if (k > 0) {
    HIPCHK(hipMemcpyAsync(vs, site.data(), sizeof(int) * k, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync(vt, tau.data(), sizeof(double) * k, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync(vsp, s.data(), sizeof(int) * k, hipMemcpyHostToDevice, w->stream));
    HIPCHK(hipMemcpyAsync(vid, id.data(), sizeof(long long) * k, hipMemcpyHostToDevice, w->stream));
  }
  w->latched = false;
  dcax_status st = reset_ctl(w, k, next_id, 1.0);
  if (st != DCAX_OK) return st;
  st = refresh_any(w, nullptr, false);
  if (st != DCAX_OK) return st;
  double ds[2];
  HIPCHK(hipMemcpyAsync(ds, w->detsign, sizeof(ds), hipMemcpyDeviceToHost, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  const double sign = ds[0] * ds[1];
  HIPCHK(hipMemcpyAsync(&w->ctl->sign, &sign, sizeof(double), hipMemcpyHostToDevice, w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  return DCAX_OK;
}

dcax_status dcax_sweep(dcax_walker w, int32_t n_sweeps, const dcax_proposal* replay, int64_t n_replay,
                       double* ratio_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (replay) {
    if (n_replay < 0) return fail(DCAX_E_INVAL, "n_replay < 0");
    if (n_replay == 0) return DCAX_OK;
    for (int64_t i = 0; i < n_replay; ++i) {
      const dcax_proposal& r = replay[i];
      if (r.kind != 0 && r.kind != 1) return fail(DCAX_E_INVAL, "replay kind must be 0 or 1");
      if (r.accepted != 0 && r.accepted != 1) return fail(DCAX_E_INVAL, "replay accepted must be 0 or 1");
      if (r.kind == 0) {
        if (r.site < 0 || r.site >= w->geo.Nc) return fail(DCAX_E_INVAL, "replay site out of range");
        if (r.aux_spin != 1 && r.aux_spin != -1) return fail(DCAX_E_INVAL, "replay aux_spin must be +1 or -1");
        if (!(r.tau >= 0.0 && r.tau < w->p.beta)) return fail(DCAX_E_INVAL, "replay tau outside [0, beta)");
        if (r.accepted && r.id < 0) return fail(DCAX_E_INVAL, "accepted insertion needs an id >= 0");
      } else if (r.id < 0 && r.accepted) {
        return fail(DCAX_E_INVAL, "a removal without target cannot be accepted");
      }
    }
    if (n_replay > w->replay_cap) {
      long long cap = std::max<long long>(n_replay, 4096);
      w->replay_d = (dcax_proposal*)w->dalloc(sizeof(dcax_proposal) * cap);
      w->ratio_d = (double*)w->dalloc(sizeof(double) * cap);
      if (!w->replay_d || !w->ratio_d) return fail(DCAX_E_NOMEM, "replay buffer allocation failed");
      w->replay_cap = cap;
      w->v64.replay = w->v32.replay = w->replay_d;
      w->v64.ratio_out = w->v32.ratio_out = w->ratio_d;
    }
    HIPCHK(hipMemcpyAsync(w->replay_d, replay, sizeof(dcax_proposal) * n_replay, hipMemcpyHostToDevice, w->stream));
    hipLaunchKernelGGL(k_set_cursor, dim3(1), dim3(1), 0, w->stream, w->ctl, 0LL, (long long)n_replay);
    const long long nwin = (n_replay + w->ks - 1) / w->ks;
    int kb = w->k_host;
    for (long long i = 0; i < nwin; ++i) {
      kb = std::min(w->max_order, kb + w->ks);
      if (w->mixed) enqueue_window<float>(w, kb, true);
      else enqueue_window<double>(w, kb, true);
    }
    HIPCHK(hipGetLastError());
    if (ratio_out)
      HIPCHK(hipMemcpyAsync(ratio_out, w->ratio_d, sizeof(double) * n_replay, hipMemcpyDeviceToHost, w->stream));
    Ctl h;
    return sync_ctl(w, &h);
  }
  if (n_sweeps < 0) return fail(DCAX_E_INVAL, "n_sweeps < 0");
  return sweep_rng(w, n_sweeps);
}

dcax_status dcax_measure_G(dcax_walker w, double* acc_dev, double* aux_dev) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  if (!aux_dev || (!acc_dev && w->p.n_freq > 0)) return fail(DCAX_E_INVAL, "NULL accumulator");
  if (w->mixed) enqueue_measure<float>(w, acc_dev, aux_dev);
  else enqueue_measure<double>(w, acc_dev, aux_dev);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_finalize_G(dcax_walker w, const double* acc_dev, const double* aux_dev, double* Giw_dev,
                            int32_t n_tau_out, double* Gtau_dev) {
  if (!w || !acc_dev || !aux_dev || !Giw_dev) return fail(DCAX_E_INVAL, "NULL argument");
  if (n_tau_out < 0 || (n_tau_out == 1) || (n_tau_out > 0 && !Gtau_dev)) return fail(DCAX_E_INVAL, "bad n_tau_out");
  const int Nc = w->geo.Nc, nf = w->p.n_freq;
  const int nx = std::max(nf, n_tau_out);
  if (nx == 0) return DCAX_OK;
  hipLaunchKernelGGL(k_finalize, dim3(cdiv(nx, WG), Nc, 2), dim3(WG), 0, w->stream, Nc, nf, w->p.beta,
                     (const double*)w->xi_d, acc_dev, aux_dev, Giw_dev, n_tau_out, n_tau_out > 0 ? Gtau_dev : nullptr);
  HIPCHK(hipGetLastError());
  return DCAX_OK;
}

dcax_status dcax_refresh(dcax_walker w, double* drift_out) {
  dcax_status st = check_latched(w);
  if (st != DCAX_OK) return st;
  return refresh_any(w, drift_out, true);
}

dcax_status dcax_get_order(dcax_walker w, int32_t* k) {
  if (!w || !k) return fail(DCAX_E_INVAL, "NULL argument");
  Ctl h;
  dcax_status st = sync_ctl(w, &h);
  *k = h.k;
  return st;
}

dcax_status dcax_get_config(dcax_walker w, dcax_vertex* out, int32_t cap, int32_t* k) {
  if (!w || !k) return fail(DCAX_E_INVAL, "NULL argument");
  Ctl h;
  dcax_status st = sync_ctl(w, &h);
  if (st != DCAX_OK && st != DCAX_E_NUMERIC && st != DCAX_E_CAPACITY && st != DCAX_E_TRACE) return st;
  *k = h.k;
  if (!out) return DCAX_OK;
  if (cap < h.k) return fail(DCAX_E_INVAL, "output too small");
  const int n = h.k;
  std::vector<int> site(n), s(n);
  std::vector<double> tau(n);
  std::vector<long long> id(n);
  const bool mx = w->mixed;
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(site.data(), mx ? w->v32.v_site : w->v64.v_site, sizeof(int) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(tau.data(), mx ? w->v32.v_tau : w->v64.v_tau, sizeof(double) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(s.data(), mx ? w->v32.v_s : w->v64.v_s, sizeof(int) * n, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipMemcpyAsync(id.data(), mx ? w->v32.v_id : w->v64.v_id, sizeof(long long) * n, hipMemcpyDeviceToHost, w->stream));
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

dcax_status dcax_copy_N(dcax_walker w, int32_t spin, double* host, int64_t ld, int64_t* ids_host) {
  if (!w || !host || (spin != 0 && spin != 1)) return fail(DCAX_E_INVAL, "bad argument");
  Ctl h;
  dcax_status st = sync_ctl(w, &h);
  if (st != DCAX_OK && st != DCAX_E_NUMERIC && st != DCAX_E_CAPACITY && st != DCAX_E_TRACE) return st;
  const int k = h.k;
  if (ld < k) return fail(DCAX_E_INVAL, "ld < k");
  if (k == 0) return st;
  std::vector<long long> id(k);
  const bool mx = w->mixed;
  HIPCHK(hipMemcpyAsync(id.data(), mx ? w->v32.v_id : w->v64.v_id, sizeof(long long) * k, hipMemcpyDeviceToHost, w->stream));
  std::vector<double> Nh((size_t)k * k);
  if (mx) {
    std::vector<float> Nf((size_t)w->ld * k);
    HIPCHK(hipMemcpyAsync(Nf.data(), w->N[spin], sizeof(float) * (size_t)w->ld * k, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) Nh[i + (size_t)j * k] = Nf[i + (size_t)j * w->ld];
  } else {
    std::vector<double> Nd((size_t)w->ld * k);
    HIPCHK(hipMemcpyAsync(Nd.data(), w->N[spin], sizeof(double) * (size_t)w->ld * k, hipMemcpyDeviceToHost, w->stream));
    HIPCHK(hipStreamSynchronize(w->stream));
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) Nh[i + (size_t)j * k] = Nd[i + (size_t)j * w->ld];
  }
  std::vector<int> o(k);
  for (int i = 0; i < k; ++i) o[i] = i;
  std::sort(o.begin(), o.end(), [&](int a, int b) { return id[a] < id[b]; });
  // host is row-major [i][j] with row stride ld, canonical order
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) host[(size_t)a * ld + b] = Nh[o[a] + (size_t)o[b] * k];
  if (ids_host)
    for (int a = 0; a < k; ++a) ids_host[a] = id[o[a]];
  return st;
}

dcax_status dcax_get_stats(dcax_walker w, dcax_stats* out) {
  if (!w || !out) return fail(DCAX_E_INVAL, "NULL argument");
  Ctl h;
  dcax_status st = sync_ctl(w, &h);
  out->proposals = h.n_prop;
  out->accepted_insertions = h.n_acc_ins;
  out->accepted_removals = h.n_acc_rem;
  out->windows = h.n_windows;
  out->flips_folded = h.sum_m;
  out->decision_mismatches = h.n_mismatch;
  out->sweeps = w->sweeps_done;
  out->sign = h.sign;
  out->fold_flops = h.fold_flops;
  out->fold_bytes = h.fold_bytes;
  out->fold_seconds = w->fold_s;
  out->fold_launches = w->fold_launches;
  out->accept_seconds = w->accept_s;
  out->window_seconds = w->window_s;
  out->aborted_windows = h.n_abort;
  out->last_drift = w->last_drift;
  out->max_drift = w->max_drift;
  return st;
}

dcax_status dcax_set_timing(dcax_walker w, int32_t on) {
  if (!w) return fail(DCAX_E_INVAL, "walker is NULL");
  Ctl h;
  dcax_status st = sync_ctl(w, &h);  // drains pending events
  w->timing = on != 0;
  return st;
}

dcax_status dcax_copy_g0_table(dcax_walker w, double* host) {
  if (!w || !host) return fail(DCAX_E_INVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(host, w->table, sizeof(double) * (size_t)w->geo.Nc * w->p.n_tau, hipMemcpyDeviceToHost,
                        w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  return DCAX_OK;
}

}  // extern "C"

// From-scratch rebuild of the walker matrices in FP64.  The kernels rebuild
// each walker of the views array they are given (the whole batch, or the
// walkers the drift control selected) at the order k_ref its control block
// holds, set to its order k by the sequence's first kernel.
//
// N_sigma^{-1} = e^{V_sigma} - g (e^{V_sigma} - 1) is assembled from k^2
// propagator gathers (Sec. 2.3's definition of N through Z_k) and inverted by
// blocked Gauss-Jordan elimination with partial pivoting:
//   for each panel of NB columns, the panel columns are eliminated one by one
//   (pivot search over the not yet pivoted rows, row swap, in-place GJ step)
//   with one panel row per thread in registers: by one workgroup for orders
//   up to PANEL_ROWS, otherwise by one launch per column over workgroups;
//   the other columns receive the panel's row swaps and then the rank-NB
//   update  A_{.x} <- P_{.J} A_{Jx} + (A_{.x} with rows J zeroed),
//   where P holds the eliminated panel columns, run on the MFMA fold tile.
// The column permutation implied by the row swaps is undone when the result
// is copied into N.  All walkers of a batch step through the panels
// together; a walker whose order is below the current panel skips it.
#include "dcax_dev.h"

namespace dcax {

// Panel widths.  The column-step form takes 64 columns when it rebuilds
// many walkers (each rank-64 update streams the matrix once per 64 columns
// instead of per 32) and 32 for a few (its column launches, which dominate
// then, read and write the whole panel each); the one-workgroup form takes
// 32 (one panel row per thread in registers at 1024 threads).  NB sizes the
// panel buffers and the pivot records for either width.
constexpr int NB = 64, NB_ONE = 32;
// column-step pivot records: two rows at the pivot position, then per parity
// one slot of 2 + NB doubles per workgroup of WG rows
constexpr int GJC_OC = 0, GJC_SLOT = 2 * NB;
__host__ __device__ inline size_t gjc_slot(int par, int b, int cap) {
  return GJC_SLOT + ((size_t)par * ((cap + WG - 1) / WG) + b) * (2 + NB);
}
inline size_t gjc_len(int cap) { return gjc_slot(2, 0, cap); }

template <typename T>
__global__ void __launch_bounds__(WG) k_build_ninv(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const int k = w.ctl->k_ref;
  const int j = blockIdx.y;
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= k || j >= k) return;
  const int ri = w.v_site[i], rj = w.v_site[j];
  const double ti = w.v_tau[i], tj = w.v_tau[j];
  const double g = gfun(w, 0, ri, ti, rj, tj);
  const double g1 = w.spin_tables == 2 ? gfun(w, 1, ri, ti, rj, tj) : g;
  const int sj = s01(w.v_s[j]);
  const double e0 = w.ev[0][sj], e1 = w.ev[1][sj];
  const size_t o = i + (size_t)j * w.cap;
  w.M[0][o] = (i == j ? e0 : 0.0) - g * (e0 - 1.0);
  w.M[1][o] = (i == j ? e1 : 0.0) - g1 * (e1 - 1.0);
}

// Eliminates panel columns [p0, p0 + nb) in one workgroup for orders up to
// PANEL_ROWS (blockIdx.x = spin, blockIdx.z = walker; at least k threads):
// one row of the panel per thread, in registers.  Per column: the pivot
// search (wavefronts, then their candidates in LDS; ties in |pivot| go to
// the smaller row index), the pivot row divided by the pivot and the old row
// at the pivot position shared through LDS, and the Gauss-Jordan step of
// every row.
constexpr int PANEL_ROWS = 1024;

__device__ inline void argmax_wave(double& v, int& i) {
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(v, o, 64);
    const int i2 = __shfl_xor(i, o, 64);
    if (v2 > v || (v2 == v && i2 < i)) {
      v = v2;
      i = i2;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(PANEL_ROWS) k_gj_panel(const View<T>* __restrict__ vs, int p0) {
  const View<T>& w = vs[blockIdx.z];
  const int k = w.ctl->k_ref;
  if (p0 >= k) return;
  const int nb = (k - p0 < NB_ONE) ? k - p0 : NB_ONE;
  const int sp = blockIdx.x;
  const auto Mg = gp(w.M[sp]);
  const size_t ld = w.cap;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = (int)(blockDim.x >> 6);
  const bool live = t < k;
  const size_t ro = live ? (size_t)t : 0;
  __shared__ double rs_s[NB_ONE], oc_s[NB_ONE], vmax_s[PANEL_ROWS / 64];
  __shared__ int imax_s[PANEL_ROWS / 64];
  __shared__ double app_s;
  double a[NB_ONE];
#pragma unroll
  for (int x = 0; x < NB_ONE; ++x) a[x] = Mg[ro + (size_t)(p0 + (x < nb ? x : 0)) * ld];
  double dsign = 1.0;
  for (int cidx = 0; cidx < nb; ++cidx) {
    const int c = p0 + cidx;
    double best = -1.0;
    int bi = k;
    if (live && t >= c) {
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) best = (x == cidx) ? fabs(a[x]) : best;
      bi = t;
    }
    argmax_wave(best, bi);
    if (lane == 0) {
      vmax_s[wv] = best;
      imax_s[wv] = bi;
    }
    __syncthreads();
    double pv = vmax_s[0];
    int piv = imax_s[0];
    for (int x = 1; x < nwv; ++x)
      if (vmax_s[x] > pv || (vmax_s[x] == pv && imax_s[x] < piv)) {
        pv = vmax_s[x];
        piv = imax_s[x];
      }
    const int pr = (piv >= c && piv < k) ? piv : c;
    if (t == pr) {
      double app = 0.0;
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) app = (x == cidx) ? a[x] : app;
      app_s = app;
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) rs_s[x] = (x == cidx) ? 1.0 / app : a[x] / app;
    }
    if (t == c)
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) oc_s[x] = a[x];
    __syncthreads();
    const double a_pp = app_s;
    if (t == 0) {
      w.ipiv[sp][c] = pr;
      if (!(pv > 0.0) || !isfinite(pv)) latch(w.ctl, ST_NUMERIC);
    }
    // sign of det: product of the pivots, one factor -1 per row interchange
    dsign *= ((a_pp < 0.0) ? -1.0 : 1.0) * ((pr != c) ? -1.0 : 1.0);
    if (t == c) {
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) a[x] = rs_s[x];
    } else {
      if (t == pr)
#pragma unroll
        for (int x = 0; x < NB_ONE; ++x) a[x] = oc_s[x];
      double f = 0.0;
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) f = (x == cidx) ? a[x] : f;
#pragma unroll
      for (int x = 0; x < NB_ONE; ++x) a[x] = (x == cidx) ? -f * rs_s[x] : a[x] - f * rs_s[x];
    }
    __syncthreads();      // rs_s, oc_s and the candidates are rewritten
  }
  if (live)
#pragma unroll
    for (int x = 0; x < NB_ONE; ++x)
      if (x < nb) Mg[t + (size_t)(p0 + x) * ld] = a[x];
  if (t == 0) w.detsign[sp] *= dsign;
}

// Column-step panel elimination for orders above PANEL_ROWS.  The panel rows
// are spread over workgroups, one row of the panel per thread (in registers).
// Launch cidx (0 .. nb):
// * cidx > 0: every workgroup reduces the pivot candidates that the previous
//   launch published for column cidx - 1 (the same winner everywhere: the
//   largest |value|, ties to the smaller row), takes the winner's row from
//   its slot and the old row at the pivot position, and applies that
//   column's Gauss-Jordan step to its rows, which it stores; workgroup 0
//   records the pivot and the determinant sign;
// * cidx < nb: each workgroup publishes its best candidate for column cidx
//   among rows >= p0 + cidx with that row's values, and the owner of row
//   p0 + cidx publishes it.
// The next launch reads what this one wrote; two sets of slots alternate
// between launches, so no launch writes what the one before it reads, and
// kernel boundaries order everything (no fences, counters or waits).  The
// arithmetic and tie rule are those of the one-workgroup form (k_gj_panel).
// Record layout (gjc, doubles per spin): [GJC_OC + p NB ..) the row at the
// pivot position for parity p = column & 1; then per parity and workgroup b
// a slot of 2 + NB doubles at gjc_slot(p, b, cap): |value|, row, row values.
template <typename T, int PW>
__global__ void __launch_bounds__(WG) k_gj_col(const View<T>* __restrict__ vs, int p0, int cidx) {
  const View<T>& w = vs[blockIdx.z];
  const int k = w.ctl->k_ref;
  if (p0 >= k) return;
  const int nb = (k - p0 < PW) ? k - p0 : PW;
  const int nwg = (k + WG - 1) / WG;
  if (cidx > nb || (int)blockIdx.x >= nwg) return;
  const int sp = blockIdx.y;
  const auto Mg = gp(w.M[sp]);
  const size_t ld = w.cap;
  double* rec = w.gjc[sp];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int r = blockIdx.x * WG + t;
  const bool live = r < k;
  const size_t ro = live ? (size_t)r : 0;
  __shared__ double vmax_s[WG / 64], rs_s[PW], oc_s[PW];
  __shared__ int imax_s[WG / 64];
  __shared__ double app_s;
  double a[PW];
#pragma unroll
  for (int x = 0; x < PW; ++x) a[x] = Mg[ro + (size_t)(p0 + (x < nb ? x : 0)) * ld];
  if (cidx > 0) {
    const int cm = cidx - 1, cp = p0 + cm, par = cm & 1;
    double best = -1.0;
    int bi = k;
    for (int b = t; b < nwg; b += WG) {
      const double* sl = rec + gjc_slot(par, b, w.cap);
      const double v = sl[0];
      const int i = (int)sl[1];
      if (v > best || (v == best && i < bi)) {
        best = v;
        bi = i;
      }
    }
    argmax_wave(best, bi);
    if (lane == 0) {
      vmax_s[wv] = best;
      imax_s[wv] = bi;
    }
    __syncthreads();
    double pv = vmax_s[0];
    int piv = imax_s[0];
    for (int x = 1; x < WG / 64; ++x)
      if (vmax_s[x] > pv || (vmax_s[x] == pv && imax_s[x] < piv)) {
        pv = vmax_s[x];
        piv = imax_s[x];
      }
    const bool valid = piv >= cp && piv < k;
    const int pr = valid ? piv : cp;
    // the pivot row: the winner's slot (or, without a valid pivot, the row at
    // the pivot position itself)
    const double* prow = valid ? rec + gjc_slot(par, piv / WG, w.cap) + 2 : rec + GJC_OC + par * NB;
    if (t == 0) app_s = prow[cm];
    __syncthreads();
    const double a_pp = app_s;
    if (t < PW) {
      rs_s[t] = (t == cm) ? 1.0 / a_pp : prow[t] / a_pp;
      oc_s[t] = rec[GJC_OC + par * NB + t];
    }
    if (blockIdx.x == 0 && t == 0) {
      w.ipiv[sp][cp] = pr;
      if (!(pv > 0.0) || !isfinite(pv)) latch(w.ctl, ST_NUMERIC);
      w.detsign[sp] *= ((a_pp < 0.0) ? -1.0 : 1.0) * ((pr != cp) ? -1.0 : 1.0);
    }
    __syncthreads();
    if (r == cp) {
#pragma unroll
      for (int x = 0; x < PW; ++x) a[x] = rs_s[x];
    } else {
      if (r == pr)
#pragma unroll
        for (int x = 0; x < PW; ++x) a[x] = oc_s[x];
      double f = 0.0;
#pragma unroll
      for (int x = 0; x < PW; ++x) f = (x == cm) ? a[x] : f;
#pragma unroll
      for (int x = 0; x < PW; ++x) a[x] = (x == cm) ? -f * rs_s[x] : a[x] - f * rs_s[x];
    }
    if (live)
#pragma unroll
      for (int x = 0; x < PW; ++x)
        if (x < nb) Mg[r + (size_t)(p0 + x) * ld] = a[x];
    __syncthreads();      // the candidates below reuse vmax_s / imax_s
  }
  if (cidx == nb) return;
  const int c = p0 + cidx, par = cidx & 1;
  double best = -1.0;
  int bi = k;
  if (live && r >= c) {
#pragma unroll
    for (int x = 0; x < PW; ++x) best = (x == cidx) ? fabs(a[x]) : best;
    bi = r;
  }
  argmax_wave(best, bi);
  if (lane == 0) {
    vmax_s[wv] = best;
    imax_s[wv] = bi;
  }
  __syncthreads();
  double wbest = vmax_s[0];
  int wbi = imax_s[0];
  for (int x = 1; x < WG / 64; ++x)
    if (vmax_s[x] > wbest || (vmax_s[x] == wbest && imax_s[x] < wbi)) {
      wbest = vmax_s[x];
      wbi = imax_s[x];
    }
  double* sl = rec + gjc_slot(par, blockIdx.x, w.cap);
  if (t == 0) {
    sl[0] = wbest;
    sl[1] = (double)wbi;
  }
  if (r == wbi)
#pragma unroll
    for (int x = 0; x < PW; ++x) sl[2 + x] = a[x];
  if (r == c)
#pragma unroll
    for (int x = 0; x < PW; ++x) rec[GJC_OC + par * NB + x] = a[x];
}

// Applies the panel's row swaps to the other columns, moves their panel rows
// into Tm (row-major, [nb][cap]) and zeroes them; copies the panel columns
// into P (column-major); pw is the panel width.  One thread per column
// (blockIdx.y = spin).
template <typename T>
__global__ void __launch_bounds__(WG) k_gj_prep(const View<T>* __restrict__ vs, int p0, int pw) {
  const View<T>& w = vs[blockIdx.z];
  const int k = w.ctl->k_ref;
  if (p0 >= k) return;
  const int nb = (k - p0 < pw) ? k - p0 : pw;
  const int sp = blockIdx.y;
  const auto M = gp(w.M[sp]);
  const auto ipiv = gp(w.ipiv[sp]);
  const auto P = gp(w.P[sp]);
  const auto Tm = gp(w.Tm[sp]);
  const size_t ldm = w.cap, ldt = w.cap;
  const int j = blockIdx.x * WG + threadIdx.x;
  if (j >= k) return;
  const size_t col = (size_t)j * ldm;
  const bool in_panel = (j >= p0 && j < p0 + nb);
  if (!in_panel) {
    for (int c = p0; c < p0 + nb; ++c) {
      const int piv = ipiv[c];
      if (piv != c && piv < k) {
        const double x = M[c + col];
        M[c + col] = M[piv + col];
        M[piv + col] = x;
      }
    }
  }
  for (int r = 0; r < nb; ++r) {
    if (in_panel) {
      Tm[(size_t)r * ldt + j] = 0.0;
    } else {
      Tm[(size_t)r * ldt + j] = M[p0 + r + col];
      M[p0 + r + col] = 0.0;
    }
  }
  for (int x = 0; x < nb; ++x) P[j + (size_t)x * ldt] = M[j + (size_t)(p0 + x) * ldm];
}

// Trailing update M += P Tm of the panel of pw columns from p0
// (blockIdx.z = 2 walker + spin).
template <typename T>
__global__ void __launch_bounds__(WG) k_gj_update(const View<T>* __restrict__ vs, int p0, int pw) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int sp = blockIdx.z & 1;
  const int k = w.ctl->k_ref;
  if (p0 >= k) return;
  const int nb = (k - p0 < pw) ? k - p0 : pw;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (i0 >= k || j0 >= k) return;
  fold_tile<double>(w.M[sp], w.cap, w.P[sp], w.cap, w.Tm[sp], w.cap, k, k, nb, i0, j0);
}

// Column permutation implied by the row interchanges: inv(A) = inv(P A) P,
// i.e. the column swaps (c, ipiv[c]) applied for c = k-1 down to 0.  One
// thread per walker and spin replays them in LDS (blockIdx.x = spin).
constexpr int PERM_MAX = 32768 + 128;
template <typename T>
__global__ void __launch_bounds__(64) k_gj_perm(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const int k = w.ctl->k_ref;
  const int sp = blockIdx.x;
  __shared__ unsigned short col_s[PERM_MAX];
  for (int j = threadIdx.x; j < k; j += 64) col_s[j] = (unsigned short)j;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int* ipiv = w.ipiv[sp];
    for (int c = k - 1; c >= 0; --c) {
      int q = ipiv[c];
      if (q < 0 || q >= k) {
        latch(w.ctl, ST_NUMERIC);
        q = c;
      }
      const unsigned short x = col_s[c];
      col_s[c] = col_s[q];
      col_s[q] = x;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += 64) w.perm[sp][j] = col_s[j];
}

// N[:, j] = M[:, perm[j]] (rounded to T), and per-block maxima of
// |N_old - N_new| and |N_new| for the drift (blockIdx.z = 2 walker + spin).
template <typename T>
__global__ void __launch_bounds__(WG) k_refresh_store(const View<T>* __restrict__ vs, int measure) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int sp = blockIdx.z & 1;
  const int k = w.ctl->k_ref;
  const int nbx = (k + WG - 1) / WG;
  if ((int)blockIdx.x >= nbx || (int)blockIdx.y >= k) return;
  const double* M = w.M[sp];
  const int* perm = w.perm[sp];
  T* N = w.N[sp];
  const int j = blockIdx.y;
  const int i = blockIdx.x * WG + threadIdx.x;
  double dmax = 0.0, nmax = 0.0;
  if (i < k) {
    const double v = M[i + (size_t)perm[j] * w.cap];
    const size_t o = i + (size_t)j * w.ld;
    if (measure) {
      dmax = fabs((double)N[o] - v);
      nmax = fabs(v);
    }
    N[o] = (T)v;
  }
  __shared__ double a_s[WG], b_s[WG];
  a_s[threadIdx.x] = dmax;
  b_s[threadIdx.x] = nmax;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      a_s[threadIdx.x] = max_nan(a_s[threadIdx.x], a_s[threadIdx.x + o]);
      b_s[threadIdx.x] = max_nan(b_s[threadIdx.x], b_s[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const size_t b = ((size_t)sp * k + j) * nbx + blockIdx.x;
    w.blkmax[2 * b] = a_s[0];
    w.blkmax[2 * b + 1] = b_s[0];
  }
}

// drift = max |N_old - N_new| / max |N_new| over both spins, into ctl->drift
// (NaN if either maximum met a NaN).
template <typename T>
__global__ void __launch_bounds__(WG) k_drift(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const int k = w.ctl->k_ref;
  const size_t n = (size_t)2 * k * ((k + WG - 1) / WG);
  double a = 0.0, b = 0.0;
  for (size_t x = threadIdx.x; x < n; x += WG) {
    a = max_nan(a, w.blkmax[2 * x]);
    b = max_nan(b, w.blkmax[2 * x + 1]);
  }
  __shared__ double a_s[WG], b_s[WG];
  a_s[threadIdx.x] = a;
  b_s[threadIdx.x] = b;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      a_s[threadIdx.x] = max_nan(a_s[threadIdx.x], a_s[threadIdx.x + o]);
      b_s[threadIdx.x] = max_nan(b_s[threadIdx.x], b_s[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // a non-finite N before the refresh (the chain's decisions since the
    // last refresh are void) is latched rather than silently replaced
    const double d = (b_s[0] > 0.0) ? a_s[0] / b_s[0] : (a_s[0] != a_s[0] ? a_s[0] : 0.0);
    w.ctl->drift = d;
    if (!isfinite(d)) latch(w.ctl, ST_NUMERIC);
  }
}

// Probe of N against its definition, without rebuilding it: for PROBE_PAIRS
// index pairs (p, q) per spin, drawn by a hash of (salt, walker, pair), the
// normalised residual
//   |sum_i A_pi N_iq - delta_pq| / sum_i |A_pi N_iq|,  A = N^{-1} = e^V - g (e^V - 1)
// assembled from the propagator (O(k) work per pair).  N carries the
// rounding of its updates; the residual measures what it has drifted from
// the inverse of A.  out[2 walker + spin] = the largest over the pairs.
// Grid (1, 2, W), WG threads: wavefront v takes pairs v, v + 4, ...
constexpr int PROBE_PAIRS = 64;

__device__ inline unsigned long long probe_mix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

// gate_tol > 0: only walkers whose sweep has just ended with its measurement
// pending are probed (the others report 0), each with pairs drawn afresh per
// sweep, and a residual above gate_tol (or NaN) sets the walker's hold flag,
// which keeps its measurement and next sweep back until N is rebuilt.
template <typename T>
__global__ void __launch_bounds__(WG) k_probe(const View<T>* __restrict__ vs, unsigned long long salt,
                                              double* __restrict__ out, double gate_tol) {
  const View<T>& w = vs[blockIdx.z];
  const int sp = blockIdx.y;
  Ctl* ctl = w.ctl;
  const bool gated = gate_tol > 0.0;
  if (gated) salt ^= probe_mix((unsigned long long)ctl->n_sweeps + 0x51ED270B7ULL);
  const int k = (gated && (ctl->hold || meas_skip(ctl, 1))) ? 0 : ctl->k;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const auto N = gp(w.N[sp]);
  double worst = 0.0;
  if (k > 0) {
    for (int j = wv; j < PROBE_PAIRS; j += WG / 64) {
      const unsigned long long h = probe_mix(salt ^ probe_mix(((unsigned long long)w.wid << 20) + (unsigned)j));
      // every fourth pair is a diagonal one
      const int p = (int)((h & 0xffffffffULL) % (unsigned long long)k);
      const int q = (j & 3) == 0 ? p : (int)((h >> 32) % (unsigned long long)k);
      const int rp = w.v_site[p];
      const double tp = w.v_tau[p];
      double sum = 0.0, mag = 0.0;
      for (int i = lane; i < k; i += 64) {
        const double e = w.ev[sp][s01(w.v_s[i])];
        const double a = (i == p ? e : 0.0) - gfun(w, sp, rp, tp, w.v_site[i], w.v_tau[i]) * (e - 1.0);
        const double t = a * (double)N[i + (size_t)q * w.ld];
        sum += t;
        mag += fabs(t);
      }
      for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 64);
        mag += __shfl_xor(mag, o, 64);
      }
      const double r = fabs(sum - (p == q ? 1.0 : 0.0));
      const double res = mag > 0.0 ? r / mag : r;
      worst = (res > worst || res != res) ? res : worst;
    }
  }
  __shared__ double w_s[WG / 64];
  if (lane == 0) w_s[wv] = worst;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int v = 0; v < WG / 64; ++v) m = (w_s[v] > m || w_s[v] != w_s[v]) ? w_s[v] : m;
    out[2 * blockIdx.z + sp] = m;
    if (gated && !(m <= gate_tol)) atomicOr(&ctl->hold, 1);
  }
}

#define DCAX_INSTANTIATE_REFRESH(T)                                   \
  template __global__ void k_probe<T>(const View<T>*, unsigned long long, double*, double); \
  template __global__ void k_build_ninv<T>(const View<T>*);           \
  template __global__ void k_gj_panel<T>(const View<T>*, int);        \
  template __global__ void k_gj_col<T, NB>(const View<T>*, int, int);  \
  template __global__ void k_gj_col<T, NB_ONE>(const View<T>*, int, int); \
  template __global__ void k_gj_prep<T>(const View<T>*, int, int);    \
  template __global__ void k_gj_update<T>(const View<T>*, int, int);  \
  template __global__ void k_refresh_store<T>(const View<T>*, int);   \
  template __global__ void k_gj_perm<T>(const View<T>*);              \
  template __global__ void k_drift<T>(const View<T>*);

DCAX_INSTANTIATE_REFRESH(double)
DCAX_INSTANTIATE_REFRESH(float)

}  // namespace dcax

// From-scratch rebuild of the walker matrices in FP64.
//
// N_sigma^{-1} = e^{V_sigma} - g (e^{V_sigma} - 1) is assembled from k^2
// propagator gathers (Sec. 2.3's definition of N through Z_k) and inverted by
// blocked Gauss-Jordan elimination with partial pivoting:
//   for each panel of NB columns, one workgroup eliminates the panel columns
//   (pivot search over the not yet pivoted rows, row swap, in-place GJ step);
//   the other columns receive the panel's row swaps and then the rank-NB
//   update  A_{.x} <- P_{.J} A_{Jx} + (A_{.x} with rows J zeroed),
//   where P holds the eliminated panel columns, run on the MFMA fold kernel.
// The column permutation implied by the row swaps is undone when the result
// is copied into N.
#include "dcax_dev.h"

namespace dcax {

constexpr int NB = 32;

template <typename T>
__global__ void __launch_bounds__(WG) k_build_ninv(View<T> w, double* M0, double* M1, int k, int ldm) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= k || j >= k) return;
  const double g = gfun(w, w.v_site[i], w.v_tau[i], w.v_site[j], w.v_tau[j]);
  const int sj = s01(w.v_s[j]);
  const double e0 = w.ev[0][sj], e1 = w.ev[1][sj];
  M0[i + (size_t)j * ldm] = (i == j ? e0 : 0.0) - g * (e0 - 1.0);
  M1[i + (size_t)j * ldm] = (i == j ? e1 : 0.0) - g * (e1 - 1.0);
}

// Eliminates panel columns [p0, p0 + nb) of both matrices (blockIdx.x = spin).
__global__ void __launch_bounds__(WG) k_gj_panel(double* M0, double* M1, int k, int ldm, int p0, int nb,
                                                 int* ipiv0, int* ipiv1, Ctl* ctl, double* detsign) {
  const int sp = blockIdx.x;
  double* M = sp ? M1 : M0;
  int* ipiv = sp ? ipiv1 : ipiv0;
  const int t = threadIdx.x;
  __shared__ double vmax_s[WG];
  __shared__ int imax_s[WG];
  __shared__ double row_s[NB];
  for (int cidx = 0; cidx < nb; ++cidx) {
    const int c = p0 + cidx;
    double best = -1.0;
    int bi = k;
    for (int r = c + t; r < k; r += WG) {
      const double v = fabs(M[r + (size_t)c * ldm]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
    vmax_s[t] = best;
    imax_s[t] = bi;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
      if (t < o) {
        const double v2 = vmax_s[t + o];
        const int i2 = imax_s[t + o];
        if (v2 > vmax_s[t] || (v2 == vmax_s[t] && i2 < imax_s[t])) {
          vmax_s[t] = v2;
          imax_s[t] = i2;
        }
      }
      __syncthreads();
    }
    const int piv = imax_s[0];
    const double pv = vmax_s[0];
    if (t == 0) {
      ipiv[c] = piv;
      if (!(pv > 0.0) || !isfinite(pv)) latch(ctl, ST_NUMERIC);
    }
    // swap rows c and piv inside the panel, then scale row c
    if (t < nb && piv != c) {
      const size_t col = (size_t)(p0 + t) * ldm;
      const double x = M[c + col];
      M[c + col] = M[piv + col];
      M[piv + col] = x;
    }
    __syncthreads();
    const double a_cc = M[c + (size_t)c * ldm];
    // sign of det: product of the pivots, one factor -1 per row interchange
    if (t == 0) detsign[sp] *= ((a_cc < 0.0) ? -1.0 : 1.0) * ((piv != c) ? -1.0 : 1.0);
    __syncthreads();
    if (t < nb) {
      const size_t col = (size_t)(p0 + t) * ldm;
      const double v = (p0 + t == c) ? 1.0 / a_cc : M[c + col] / a_cc;
      M[c + col] = v;
      row_s[t] = v;
    }
    __syncthreads();
    for (int r = t; r < k; r += WG) {
      if (r == c) continue;
      const double f = M[r + (size_t)c * ldm];
      for (int x = 0; x < nb; ++x) {
        const size_t o = r + (size_t)(p0 + x) * ldm;
        if (p0 + x == c) M[o] = -f * row_s[x];
        else M[o] -= f * row_s[x];
      }
    }
    __syncthreads();
  }
}

// Applies the panel's row swaps to the other columns, moves their panel rows
// into Tm (row-major, [nb][ldt]) and zeroes them; copies the panel columns
// into P (column-major).  One thread per column.
__global__ void __launch_bounds__(WG) k_gj_prep(double* M0, double* M1, int k, int ldm, int p0, int nb,
                                                const int* ipiv0, const int* ipiv1, double* P0, double* P1,
                                                double* T0, double* T1, int ldt) {
  const int sp = blockIdx.y;
  double* M = sp ? M1 : M0;
  const int* ipiv = sp ? ipiv1 : ipiv0;
  double* P = sp ? P1 : P0;
  double* Tm = sp ? T1 : T0;
  const int j = blockIdx.x * WG + threadIdx.x;
  if (j >= k) return;
  const size_t col = (size_t)j * ldm;
  const bool in_panel = (j >= p0 && j < p0 + nb);
  if (!in_panel) {
    for (int c = p0; c < p0 + nb; ++c) {
      const int piv = ipiv[c];
      if (piv != c) {
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
  // panel column copy: thread j copies row j of the panel
  for (int x = 0; x < nb; ++x) P[j + (size_t)x * ldt] = M[j + (size_t)(p0 + x) * ldm];
}

// N[:, j] = M[:, perm[j]] (rounded to T), and per-block maxima of
// |N_old - N_new| and |N_new| for the drift.
template <typename T>
__global__ void __launch_bounds__(WG) k_refresh_store(View<T> w, const double* M0, const double* M1, int k, int ldm,
                                                      const int* perm0, const int* perm1, double* blkmax, int measure) {
  const int sp = blockIdx.z;
  const double* M = sp ? M1 : M0;
  const int* perm = sp ? perm1 : perm0;
  T* N = w.N[sp];
  const int j = blockIdx.y;
  const int i = blockIdx.x * WG + threadIdx.x;
  double dmax = 0.0, nmax = 0.0;
  if (i < k && j < k) {
    const double v = M[i + (size_t)perm[j] * ldm];
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
      a_s[threadIdx.x] = fmax(a_s[threadIdx.x], a_s[threadIdx.x + o]);
      b_s[threadIdx.x] = fmax(b_s[threadIdx.x], b_s[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const size_t b = ((size_t)sp * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    blkmax[2 * b] = a_s[0];
    blkmax[2 * b + 1] = b_s[0];
  }
}

template __global__ void k_build_ninv<double>(View<double>, double*, double*, int, int);
template __global__ void k_build_ninv<float>(View<float>, double*, double*, int, int);
template __global__ void k_refresh_store<double>(View<double>, const double*, const double*, int, int, const int*,
                                                 const int*, double*, int);
template __global__ void k_refresh_store<float>(View<float>, const double*, const double*, int, int, const int*,
                                                const int*, double*, int);

}  // namespace dcax

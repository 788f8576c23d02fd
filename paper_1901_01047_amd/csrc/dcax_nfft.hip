// Delayed-NFFT measurement of M (Sec. 2.3, non-equidistant FFT measurements).
//
// The quantity is the one the direct measurement accumulates,
//   M(K, i w_n) = (1/Nc) sum_ij e^{i w_n (tau_i - tau_j)} e^{-i K (r_i - r_j)} M_ij,
// which depends on a pair only through tau_i - tau_j and the displacement
// d = r_i - r_j.  Per measurement every pair is spread onto an equispaced
// grid of L = 4 n_freq points on [0, beta) (row d, per spin), with the
// Gaussian kernel exp(-x^2 / (4 t)) of Greengard & Lee (SIAM Review 46, 2004;
// oversampling ratio 2, half-width M_sp points, t = M_sp beta^2 /
// (48 pi n_freq^2)).  A pair with tau_i < tau_j is the antiperiodic image at
// tau_i - tau_j + beta with the opposite sign, and grid points beyond [0, L)
// wrap with a factor -1.  The grids are accumulated with the configuration's
// sign over the run; once at the end each row is transformed,
//   F_d(w_n) = h sum_l G_d[l] e^{i w_n l h} / g(w_n),  g(w) = sqrt(4 pi t) e^{-t w^2},
// and M(K, i w_n) = (1/Nc) sum_d e^{-i K r_d} F_d(w_n) is added to the direct
// measurement's accumulator layout.  The error is of order
// exp(-(2/3) pi M_sp) per unit of sum |M_ij| (aliasing of the highest
// frequency by the grid).
//
// Gridding runs per (walker, spin, d, group of sites a) in one workgroup:
// the pairs of d come from the site-sorted copy of M that the direct
// measurement's sort and copy kernels produce (blocks (a, b) with
// r_a - r_b = d), the workgroup accumulates its part of the row in LDS and
// then adds it to the caller's grid (plainly when one workgroup covers the
// row, with atomic adds when several share it).  The kernel weights use the product form of the
// Gaussian (Greengard & Lee, Sec. 3): for x = s - l0 h,
//   exp(-(x - q h)^2 / 4t) = exp(-x^2 / 4t) (exp(x h / 2t))^q exp(-q^2 h^2 / 4t).
#include "dcax_dev.h"

namespace dcax {

constexpr int NFFT_L_MAX = 8192;      // grid points per row held in LDS (n_freq <= 2048)
constexpr int NFFT_MSP_MAX = 16;

template <typename T>
__global__ void __launch_bounds__(WG) k_nfft_grid(const View<T>* __restrict__ vs, int m_sp, int groups,
                                                  double* grid_all, int gated) {
  const View<T>& w = vs[blockIdx.z];
  if (meas_skip(w.ctl, gated)) return;
  const int Nc = w.Nc;
  const int d = blockIdx.x % Nc, grp = blockIdx.x / Nc;
  // sites a of this workgroup: [a0, a1)
  const int per = (Nc + groups - 1) / groups;
  const int a0 = grp * per, a1 = min(Nc, a0 + per);
  if ((int)blockIdx.x >= Nc * groups || a0 >= a1) return;
  const int sp = blockIdx.y;
  const int L = 4 * w.n_freq;
  const double beta = w.beta;
  const double h = beta / L;
  const double t4 = 4.0 * (m_sp * beta * beta / (48.0 * M_PI * (double)w.n_freq * (double)w.n_freq));
  const auto order = gp(w.m_order);
  const auto off = gp(w.m_off);
  const auto Ms = gp(w.m_Ms[sp]);
  const auto tau = gp(w.v_tau);
  const int ldm = w.kpad_cap;
  extern __shared__ double g_s[];     // [L], sized at launch
  __shared__ double q2_s[2 * NFFT_MSP_MAX];
  __shared__ int partner_s[MEAS_NC_MAX];
  for (int l = threadIdx.x; l < L; l += WG) g_s[l] = 0.0;
  for (int q = threadIdx.x; q < 2 * m_sp; q += WG) {
    const double qq = (double)(q - m_sp + 1);
    q2_s[q] = exp(-qq * qq * h * h / t4);
  }
  // b with r_a - r_b = d, for every site a
  for (int x = threadIdx.x; x < Nc * Nc; x += WG)
    if (w.diff[x] == d) partner_s[x / Nc] = x % Nc;
  __syncthreads();
  const double sign = w.ctl->sign;
  for (int a = a0; a < a1; ++a) {
    const int b = partner_s[a];
    const int i0 = off[a], na = off[a + 1] - i0;
    const int j0 = off[b], nbb = off[b + 1] - j0;
    const int np = na * nbb;
    for (int p = threadIdx.x; p < np; p += WG) {
      const int ip = i0 + p % na, jp = j0 + p / na;
      const int i = order[ip], j = order[jp];
      if (i < 0 || j < 0) continue;
      double f = (double)Ms[ip + (size_t)jp * ldm];
      double s = tau[i] - tau[j];
      if (s < 0.0) {
        s += beta;
        f = -f;
      }
      const int l0 = (int)floor(s / h);
      const double x = s - l0 * h;
      const double e0 = exp(-x * x / t4);
      const double e1 = exp(2.0 * x * h / t4);
      // (e1)^q from q = -(m_sp - 1) upwards
      double ep = exp(-2.0 * x * h * (double)(m_sp - 1) / t4);
      for (int q = 0; q < 2 * m_sp; ++q) {
        int l = l0 + q - m_sp + 1;
        double sg = 1.0;
        if (l < 0) {
          l += L;
          sg = -1.0;
        } else if (l >= L) {
          l -= L;
          sg = -1.0;
        }
        atomicAdd(&g_s[l], sg * f * e0 * ep * q2_s[q]);
        ep *= e1;
      }
    }
  }
  __syncthreads();
  double* row = grid_all + 2 * w.acc_off + ((size_t)sp * Nc + d) * L;
  if (per >= Nc)
    for (int l = threadIdx.x; l < L; l += WG) row[l] += sign * g_s[l];
  else
    for (int l = threadIdx.x; l < L; l += WG) atomicAdd(&row[l], sign * g_s[l]);
}

// F_d(w_n) for every row of a walker's grid, into m_Mab[sp] as [d][n][2]
// (blockIdx.x: frequencies, y: displacement, z = 2 walker + spin).  The phase
// w_n l h = pi (2n+1) l / L is reduced exactly, (2n+1) l mod 2L, before sinpi/cospi.
template <typename T>
__global__ void __launch_bounds__(WG) k_nfft_rows(const View<T>* __restrict__ vs, int m_sp, const double* grid_all) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int sp = blockIdx.z & 1;
  const int Nc = w.Nc, nf = w.n_freq;
  const int n = blockIdx.x * WG + threadIdx.x;
  const int d = blockIdx.y;
  if (d >= Nc || n >= nf) return;
  const int L = 4 * nf;
  const double beta = w.beta;
  const double h = beta / L;
  const double t = m_sp * beta * beta / (48.0 * M_PI * (double)nf * (double)nf);
  const double* row = grid_all + 2 * w.acc_off + ((size_t)sp * Nc + d) * L;
  const long long k2 = 2 * n + 1, twoL = 2 * (long long)L;
  double re = 0.0, im = 0.0;
  long long m = 0;
  for (int l = 0; l < L; ++l) {
    double sn, cs;
    sincospi((double)m / (double)L, &sn, &cs);
    const double gv = row[l];
    re += gv * cs;
    im += gv * sn;
    m += k2;
    if (m >= twoL) m -= twoL;
  }
  const double wn = (2.0 * n + 1.0) * M_PI / beta;
  const double scale = h / (sqrt(4.0 * M_PI * t) * exp(-t * wn * wn));
  double* F = w.m_Mab[sp];
  F[2 * ((size_t)d * nf + n)] = re * scale;
  F[2 * ((size_t)d * nf + n) + 1] = im * scale;
}

// acc[sp][q][n] += (1/Nc) sum_d e^{-i K_q r_d} F_d(w_n) (blockIdx.x:
// frequencies, y: momenta, z = 2 walker + spin).
template <typename T>
__global__ void __launch_bounds__(WG) k_nfft_K(const View<T>* __restrict__ vs, double* acc_all) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int sp = blockIdx.z & 1;
  const int Nc = w.Nc, nf = w.n_freq;
  const int n = blockIdx.x * WG + threadIdx.x;
  const int q = blockIdx.y;
  if (q >= Nc) return;
  __shared__ double pr_s[MEAS_NC_MAX], pi_s[MEAS_NC_MAX];
  for (int dd = threadIdx.x; dd < Nc; dd += WG) {
    double s, c;
    sincos(-(w.Kp[2 * q] * (double)w.sites[2 * dd] + w.Kp[2 * q + 1] * (double)w.sites[2 * dd + 1]), &s, &c);
    pr_s[dd] = c;
    pi_s[dd] = s;
  }
  __syncthreads();
  if (n >= nf) return;
  const double* F = w.m_Mab[sp];
  double re = 0.0, im = 0.0;
  for (int dd = 0; dd < Nc; ++dd) {
    const double fr = F[2 * ((size_t)dd * nf + n)], fi = F[2 * ((size_t)dd * nf + n) + 1];
    re += pr_s[dd] * fr - pi_s[dd] * fi;
    im += pr_s[dd] * fi + pi_s[dd] * fr;
  }
  double* acc = acc_all + w.acc_off;
  const size_t o = 2 * (((size_t)sp * Nc + q) * nf + n);
  acc[o] += re / (double)Nc;
  acc[o + 1] += im / (double)Nc;
}

#define DCAX_INSTANTIATE_NFFT(T)                                                     \
  template __global__ void k_nfft_grid<T>(const View<T>*, int, int, double*, int);   \
  template __global__ void k_nfft_rows<T>(const View<T>*, int, const double*);       \
  template __global__ void k_nfft_K<T>(const View<T>*, double*);

DCAX_INSTANTIATE_NFFT(double)
DCAX_INSTANTIATE_NFFT(float)

}  // namespace dcax

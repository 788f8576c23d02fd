// Kernels of the DCA self-consistency loop around the walkers (Sec. 2.1):
// coarse-graining over the patches, cluster exclusion, the transform of the
// cluster-excluded G0 to the walkers' G0(r, tau) tables, the cluster G from
// the walkers' accumulators, and Dyson's equation with self-energy mixing.
// All in FP64; complex numbers are (re, im) pairs in interleaved arrays.
#include "dcax_dev.h"

namespace dcax {

// Device-side constants of a DCA handle, passed by value.
struct DcaDev {
  int Nc, P, nf, ncg, n_tau, n_spin;
  double beta, mu, h, inv_l2;
  const double* eps;      // [Nc][P] eps(K + k~_p) over the patch quadrature
  const double* wt;       // [P] quadrature weights (sum L^2)
  const double* epsbar;   // [Nc] patch means of eps
  const double* epsvar;   // [Nc] patch variances of eps
  const double* Kr;       // [Nc r][Nc K] K . r_d
};

__device__ inline double dca_shift(const DcaDev& d, int s) { return s == 0 ? d.h : -d.h; }

// Sigma(K, i w_n) of spin block s at any n < ncg: measured values below nf;
// above, the last measured real part and an imaginary part falling as 1/w_n.
__device__ inline void dca_sigma(const DcaDev& d, const double* sigma, int s, int K, int n, double& sr, double& si) {
  const size_t row = ((size_t)s * d.Nc + K) * d.nf;
  if (n < d.nf) {
    sr = sigma[2 * (row + n)];
    si = sigma[2 * (row + n) + 1];
  } else {
    const int l = d.nf - 1;
    sr = sigma[2 * (row + l)];
    si = sigma[2 * (row + l) + 1] * (double)(2 * l + 1) / (double)(2 * n + 1);
  }
}

// Coarse-graining and cluster exclusion: one thread per (n, K, spin block),
//   Gbar = (1/L^2) sum_p wt_p / (i w_n + mu + sigma h - eps_{K,p} - Sigma),
//   G0cal = 1 / (1/Gbar + Sigma).
// Grid (ceil(ncg / WG), Nc, n_spin).
__global__ void __launch_bounds__(WG) k_dca_coarse_grain(DcaDev d, const double* __restrict__ sigma,
                                                         double* __restrict__ gbar, double* __restrict__ g0) {
  const int n = blockIdx.x * WG + threadIdx.x;
  const int K = blockIdx.y, s = blockIdx.z;
  if (n >= d.ncg) return;
  double sr, si;
  dca_sigma(d, sigma, s, K, n, sr, si);
  const double w = (double)(2 * n + 1) * M_PI / d.beta;
  const double zr = d.mu + dca_shift(d, s) - sr, zi = w - si;
  const double* e = d.eps + (size_t)K * d.P;
  double ar = 0.0, ai = 0.0;
  for (int p = 0; p < d.P; ++p) {
    const double a = zr - e[p];
    const double q = d.wt[p] / (a * a + zi * zi);
    ar += a * q;
    ai -= zi * q;
  }
  ar *= d.inv_l2;
  ai *= d.inv_l2;
  const size_t o = 2 * (((size_t)s * d.Nc + K) * d.ncg + n);
  if (gbar) {
    gbar[o] = ar;
    gbar[o + 1] = ai;
  }
  // 1/Gbar + Sigma, then its reciprocal
  const double m2 = ar * ar + ai * ai;
  const double br = ar / m2 + sr, bi = -ai / m2 + si;
  const double b2 = br * br + bi * bi;
  g0[o] = br / b2;
  g0[o + 1] = -bi / b2;
}

// G0cal(K, tau_l) on the table grid, tau_l = l beta / (n_tau - 1): the sum
// over n < ncg of (2/beta) Re[e^{-i w_n tau} R(i w_n)] with
// R = G0cal - 1/(i w) - c2/(i w)^2 - c3/(i w)^3, plus the closed forms of the
// three tail terms: the exact moments c2 = epsbar_K - mu - sigma h and
// c3 = c2^2 + var_K (expanding the patch average in 1/(i w); the self-energy
// cancels in the exclusion to that order).  The phase w_n tau_l = pi (2n+1) l /
// (n_tau - 1) is reduced modulo 2 pi in integers.  One thread per (l, K,
// spin block); grid (ceil(n_tau / WG), Nc, n_spin).
__global__ void __launch_bounds__(WG) k_dca_K_tau(DcaDev d, const double* __restrict__ g0, double* __restrict__ out) {
  const int l = blockIdx.x * WG + threadIdx.x;
  const int K = blockIdx.y, s = blockIdx.z;
  if (l >= d.n_tau) return;
  const double* g = g0 + 2 * ((size_t)s * d.Nc + K) * d.ncg;
  const double c2 = d.epsbar[K] - d.mu - dca_shift(d, s);
  const double c3 = c2 * c2 + d.epsvar[K];
  const long long per = 2LL * (d.n_tau - 1);
  const double inv = 1.0 / (double)(d.n_tau - 1);
  double acc = 0.0;
  long long red = l % per;              // (2n + 1) l mod 2 (n_tau - 1), n = 0
  const long long step = (2LL * l) % per;
  for (int n = 0; n < d.ncg; ++n) {
    const double w = (double)(2 * n + 1) * M_PI / d.beta;
    const double w2 = w * w;
    const double rr = g[2 * n] + c2 / w2;
    const double ri = g[2 * n + 1] + 1.0 / w - c3 / (w2 * w);
    double sn, cs;
    sincospi((double)red * inv, &sn, &cs);
    acc += rr * cs + ri * sn;
    red += step;
    if (red >= per) red -= per;
  }
  const double tau = (double)l * d.beta * inv;
  out[((size_t)s * d.Nc + K) * d.n_tau + l] =
      (2.0 / d.beta) * acc - 0.5 + c2 * (2.0 * tau - d.beta) * 0.25 + c3 * tau * (d.beta - tau) * 0.25;
}

// The walkers' table G0cal(r_d, tau_l) = (1/Nc) sum_K cos(K . r_d) G0cal(K, tau_l)
// (the real part of the Fourier sum).  Grid (ceil(n_tau / WG), Nc r, n_spin).
__global__ void __launch_bounds__(WG) k_dca_table(DcaDev d, const double* __restrict__ gk, double* __restrict__ tab) {
  const int l = blockIdx.x * WG + threadIdx.x;
  const int r = blockIdx.y, s = blockIdx.z;
  if (l >= d.n_tau) return;
  double acc = 0.0;
  for (int K = 0; K < d.Nc; ++K) acc += cos(d.Kr[(size_t)r * d.Nc + K]) * gk[((size_t)s * d.Nc + K) * d.n_tau + l];
  tab[((size_t)s * d.Nc + r) * d.n_tau + l] = acc / (double)d.Nc;
}

// The cluster G from accumulators of n_blocks walkers (each block
// [2 spins][Nc][nf] complex, then aux [n_blocks][3] = sign, ...):
//   <M_sigma> = sum_b acc_b / sum_b sign_b,
//   G_sigma = G0cal - G0cal <M_sigma> G0cal / beta,
// averaged over the two spins when the handle carries one spin block.
// One thread per (n, K, spin block); grid (ceil(nf / WG), Nc, n_spin).
__global__ void __launch_bounds__(WG) k_dca_cluster_G(DcaDev d, const double* __restrict__ g0,
                                                      const double* __restrict__ acc, const double* __restrict__ aux,
                                                      int n_blocks, double* __restrict__ G) {
  const int n = blockIdx.x * WG + threadIdx.x;
  const int K = blockIdx.y, s = blockIdx.z;
  if (n >= d.nf) return;
  double sg = 0.0;
  for (int b = 0; b < n_blocks; ++b) sg += aux[3 * b];
  const size_t blk = 4 * (size_t)d.Nc * d.nf;
  const size_t og = 2 * (((size_t)s * d.Nc + K) * d.ncg + n);
  const double gr = g0[og], gi = g0[og + 1];
  const double g2r = gr * gr - gi * gi, g2i = 2.0 * gr * gi;
  double outr = 0.0, outi = 0.0;
  const int s0 = d.n_spin == 2 ? s : 0, s1 = d.n_spin == 2 ? s : 1;
  for (int sp = s0; sp <= s1; ++sp) {
    double mr = 0.0, mi = 0.0;
    const size_t o = 2 * (((size_t)sp * d.Nc + K) * d.nf + n);
    for (int b = 0; b < n_blocks; ++b) {
      mr += acc[b * blk + o];
      mi += acc[b * blk + o + 1];
    }
    mr /= sg;
    mi /= sg;
    outr += gr - (g2r * mr - g2i * mi) / d.beta;
    outi += gi - (g2r * mi + g2i * mr) / d.beta;
  }
  const double f = 1.0 / (double)(s1 - s0 + 1);
  const size_t oo = 2 * (((size_t)s * d.Nc + K) * d.nf + n);
  G[oo] = outr * f;
  G[oo + 1] = outi * f;
}

// Dyson's equation and mixing on the measured frequencies:
//   Sigma_new = alpha (1/G0cal - 1/G) + (1 - alpha) Sigma_old
// (sigma_new may alias sigma_old), and max |Sigma_new - Sigma_old| into
// *maxchg as the bit pattern of a non-negative double (ordered like the
// value).  Grid (ceil(nf / WG), Nc, n_spin).
__global__ void __launch_bounds__(WG) k_dca_sigma(DcaDev d, const double* __restrict__ g0, const double* G,
                                                  const double* sigma_old, double alpha, double* sigma_new,
                                                  unsigned long long* maxchg) {
  const int n = blockIdx.x * WG + threadIdx.x;
  const int K = blockIdx.y, s = blockIdx.z;
  double chg = 0.0;
  if (n < d.nf) {
    const size_t og = 2 * (((size_t)s * d.Nc + K) * d.ncg + n);
    const size_t o = 2 * (((size_t)s * d.Nc + K) * d.nf + n);
    const double ar = g0[og], ai = g0[og + 1];
    const double a2 = ar * ar + ai * ai;
    const double br = G[o], bi = G[o + 1];
    const double b2 = br * br + bi * bi;
    const double qr = ar / a2 - br / b2, qi = -ai / a2 + bi / b2;
    const double orr = sigma_old[o], oi = sigma_old[o + 1];
    const double nr = alpha * qr + (1.0 - alpha) * orr, ni = alpha * qi + (1.0 - alpha) * oi;
    sigma_new[o] = nr;
    sigma_new[o + 1] = ni;
    chg = sqrt((nr - orr) * (nr - orr) + (ni - oi) * (ni - oi));
  }
  __shared__ double red_s[WG];
  red_s[threadIdx.x] = chg;
  __syncthreads();
  for (int h = WG / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red_s[threadIdx.x] = fmax(red_s[threadIdx.x], red_s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && maxchg) atomicMax(maxchg, (unsigned long long)__double_as_longlong(red_s[0]));
}

}  // namespace dcax

// Two-particle Green's function of the cluster, particle-particle up-down
// channel (Sec. 2.5's G_2 of the Bethe-Salpeter equation; App. B four-point
// type PARTICLE_PARTICLE_UP_DOWN).  For one configuration the spins are
// independent quadratic problems, so
//   G2(k1, k2; q) = G_up(k1, k2) G_down(q - k1, q - k2),
// with the configuration's (not translation-averaged) Green's function
//   G(k1, k2) = G0(k1) delta - G0(k1) M(k1, k2) G0(k2) / beta,
//   M(k1, k2) = (1/Nc) sum_ij e^{i (w1 tau_i - K1 r_i)} M_ij e^{-i (w2 tau_j - K2 r_j)},
// M = (e^V - 1) N in the site-sorted, padded order of the single-particle
// measurement.  The contraction runs site-blocked like that measurement:
//   T1[i'][b][w2] = sum_{j' in b} M_{i'j'} e^{-i w2 tau_j}            (k^2 n_w)
//   F[a][w1][b][w2] = sum_{i' in a} e^{i w1 tau_i} T1[i'][b][w2]      (k Nc n_w^2)
//   M(k1, k2) = (1/Nc) sum_ab e^{-i K1 r_a} F[a][w1][b][w2] e^{i K2 r_b}
// (4 Nc^2 ... instead of the k^2 Nc^2 n_w^2 of the direct double sum).
// Frequencies w_c = (2 (n_lo + c) + 1) pi / beta, c = 0 .. nw - 1; complex
// numbers interleaved (re, im), FP64 throughout.
#include "dcax_dev.h"

namespace dcax {

struct G2Dev {
  int nw, n_lo, kpad;      // one-particle frequencies, their first index, rows of the scratch (>= every walker's kpad)
  double2* P;              // [kpad][nw]    e^{-i w_c tau_j} (0 on padding)
  double2* T1;             // [Nc][nw][kpad]
  double2* F;              // [Nc a][nw][Nc b][nw]
  double2* H;              // [Nc K1][nw][Nc b][nw]
  double2* G[2];           // [Nc K1][nw][Nc K2][nw] per spin
  double2* ph;             // [Nc K][Nc a] e^{-i K r_a}
};

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b) {     // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Phases of the sorted vertices; grid (ceil(nw / 64), ceil(kpad / 4)), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256) k_g2_phase(const View<T>* __restrict__ vs, G2Dev g) {
  const View<T>& w = vs[0];
  const int kp = gp(w.m_off)[w.Nc];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int jp = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= g.nw || jp >= kp) return;
  const int j = gp(w.m_order)[jp];
  double2 v = make_double2(0.0, 0.0);
  if (j >= 0) {
    const double wn = (2.0 * (g.n_lo + c) + 1.0) * M_PI / w.beta;
    double s, co;
    sincos(wn * w.v_tau[j], &s, &co);
    v = make_double2(co, -s);
  }
  g.P[(size_t)jp * g.nw + c] = v;
}

// Momentum phases e^{-i K r_a} of the cluster; one thread per (K, a).
template <typename T>
__global__ void __launch_bounds__(WG) k_g2_kphase(const View<T>* __restrict__ vs, G2Dev g) {
  const View<T>& w = vs[0];
  const int Nc = w.Nc;
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t >= Nc * Nc) return;
  const int K = t / Nc, a = t % Nc;
  double s, c;
  sincos(-(w.Kp[2 * K] * (double)w.sites[2 * a] + w.Kp[2 * K + 1] * (double)w.sites[2 * a + 1]), &s, &c);
  g.ph[t] = make_double2(c, s);
}

// T1[b][c][i'] = sum_{j' in b} Ms[i'][j'] P[j'][c] on the FP64 matrix cores.
// Workgroup (row group of 256, site b, tile of 16 frequencies); its four
// wavefronts take the 16-row blocks of the group in turn.  A wavefront keeps a chunk of b's phase rows
// P[j][c] (G2_NB blocks of 16 columns) in registers, the lane supplying
// column j = jc + 16 q + 4 u + (lane >> 4) of frequency c0 + (lane & 15), and
// streams the rows of Ms: per 16 rows D[c][i'] = sum_j P[j][c] Ms[i'][j]
// (real and imaginary parts of P separately), stored as T1[b][c][i'] by the
// first chunk of b and added by later ones.
constexpr int G2_NB = 4, G2_RG = 256;
template <typename T>
__global__ void __launch_bounds__(WG) k_g2_t1m(const View<T>* __restrict__ vs, int sp, G2Dev g) {
  const View<T>& w = vs[0];
  const auto off = gp(w.m_off);
  const int kp = off[w.Nc];
  const int b = blockIdx.y, c0 = blockIdx.z * 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = blockIdx.x * G2_RG;
  if (r0 >= kp) return;
  const int nw = g.nw;
  const int ca = c0 + li < nw ? c0 + li : 0;       // rows past nw are computed and never stored
  const auto Ms = gp(w.m_Ms[sp]);
  const size_t ldm = w.kpad_cap;
  const double2* __restrict__ P = g.P;
  double2* __restrict__ T1 = g.T1;
  const int jb0 = off[b], jb1 = off[b + 1];
  const size_t tb = (size_t)b * nw;
  if (jb0 == jb1) {
    // no vertex on site b: its T1 rows are zero
    for (int ib = r0 + wv * 16; ib < r0 + G2_RG && ib < kp; ib += 64)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = c0 + Mfma<double>::row(lane, r);
        if (c < nw) T1[(tb + c) * g.kpad + ib + li] = make_double2(0.0, 0.0);
      }
    return;
  }
  for (int jc = jb0; jc < jb1; jc += 16 * G2_NB) {
    const int blocks = (jb1 - jc) / 16 < G2_NB ? (jb1 - jc) / 16 : G2_NB;
    const bool add = jc > jb0;
    double er[G2_NB][4], ei[G2_NB][4];
#pragma unroll
    for (int q = 0; q < G2_NB; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = jc + 16 * q + 4 * u + lk;
        const double2 p = P[(size_t)(q < blocks ? j : jc) * nw + ca];
        er[q][u] = q < blocks ? p.x : 0.0;
        ei[q][u] = q < blocks ? p.y : 0.0;
      }
    for (int ib = r0 + wv * 16; ib < r0 + G2_RG && ib < kp; ib += 64) {
      const size_t ip = (size_t)ib + li;
      double m[G2_NB][4];
#pragma unroll
      for (int q = 0; q < G2_NB; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = jc + 16 * q + 4 * u + lk;
          m[q][u] = (double)Ms[ip + (size_t)(q < blocks ? j : jc) * ldm];
        }
      typename Mfma<double>::acc_t dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < G2_NB; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          dr = Mfma<double>::run(er[q][u], m[q][u], dr);
          di = Mfma<double>::run(ei[q][u], m[q][u], di);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = c0 + Mfma<double>::row(lane, r);
        if (c < nw) {
          double2* o = T1 + (tb + c) * g.kpad + ip;
          const double2 prev = add ? *o : make_double2(0.0, 0.0);
          *o = make_double2(prev.x + dr[r], prev.y + di[r]);
        }
      }
    }
  }
}

// F[a][c1][b][c2] = sum_{i' in a} conj(P[i'][c1]) T1[b][c2][i']; thread per
// (c1, b, c2) with c1 fastest; grid (ceil(nw^2 Nc / WG), Nc a).
template <typename T>
__global__ void __launch_bounds__(WG) k_g2_f(const View<T>* __restrict__ vs, G2Dev g) {
  const View<T>& w = vs[0];
  const auto off = gp(w.m_off);
  const int Nc = w.Nc, nw = g.nw;
  const int a = blockIdx.y;
  const long long t = (long long)blockIdx.x * WG + threadIdx.x;
  if (t >= (long long)nw * Nc * nw) return;
  const int c1 = (int)(t % nw);
  const long long bc2 = t / nw;                 // b nw + c2
  const double2* t1 = g.T1 + (size_t)bc2 * g.kpad;
  double2 acc = make_double2(0.0, 0.0);
  for (int ip = off[a]; ip < off[a + 1]; ++ip) {
    const double2 x = cmulc(g.P[(size_t)ip * nw + c1], t1[ip]);
    acc.x += x.x;
    acc.y += x.y;
  }
  g.F[((size_t)a * nw + c1) * (size_t)Nc * nw + bc2] = acc;
}

// H[K1][c1][b][c2] = sum_a e^{-i K1 r_a} F[a][c1][b][c2]; thread per
// (c1, b, c2) with c2 fastest; grid (ceil(nw^2 Nc / WG), Nc K1).
template <typename T>
__global__ void __launch_bounds__(WG) k_g2_k1(const View<T>* __restrict__ vs, G2Dev g) {
  const View<T>& w = vs[0];
  const int Nc = w.Nc, nw = g.nw;
  const int K1 = blockIdx.y;
  const long long t = (long long)blockIdx.x * WG + threadIdx.x;
  const long long per = (long long)nw * Nc * nw;
  if (t >= per) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < Nc; ++a) {
    const double2 e = g.ph[K1 * Nc + a];
    const double c = e.x, s = e.y;
    const double2 f = g.F[(size_t)a * per + t];
    acc.x += c * f.x - s * f.y;
    acc.y += c * f.y + s * f.x;
  }
  g.H[(size_t)K1 * per + t] = acc;
}

// G0(K, i w_n) for any fermionic index n (negative ones by conjugation).
template <typename T>
__device__ inline double2 g0_any(const View<T>& w, int sp, int K, int n) {
  double gr, gi;
  if (n >= 0) {
    g0_K_iw(w, sp, K, n, gr, gi);
    return make_double2(gr, gi);
  }
  g0_K_iw(w, sp, K, -n - 1, gr, gi);
  return make_double2(gr, -gi);
}

// G[K1][c1][K2][c2] = G0(k1) delta - G0(k1) M(k1, k2) G0(k2) / beta with
// M(k1, k2) = (1/Nc) sum_b H[K1][c1][b][c2] e^{i K2 r_b}; thread per
// (c1, K2, c2) with c2 fastest; grid (ceil(nw^2 Nc / WG), Nc K1).
template <typename T>
__global__ void __launch_bounds__(WG) k_g2_g(const View<T>* __restrict__ vs, int sp, G2Dev g) {
  const View<T>& w = vs[0];
  const int Nc = w.Nc, nw = g.nw;
  const int K1 = blockIdx.y;
  const long long t = (long long)blockIdx.x * WG + threadIdx.x;
  const long long per = (long long)nw * Nc * nw;
  if (t >= per) return;
  const int c2 = (int)(t % nw);
  const int K2 = (int)((t / nw) % Nc);
  const int c1 = (int)(t / ((long long)nw * Nc));
  const double2* h = g.H + (size_t)K1 * per + (size_t)c1 * Nc * nw + c2;
  double2 m = make_double2(0.0, 0.0);
  for (int b = 0; b < Nc; ++b) {
    const double2 e = g.ph[K2 * Nc + b];     // e^{+i K2 r_b} = conj
    const double c = e.x, s = -e.y;
    const double2 x = h[(size_t)b * nw];
    m.x += c * x.x - s * x.y;
    m.y += c * x.y + s * x.x;
  }
  m.x /= (double)Nc;
  m.y /= (double)Nc;
  const double2 g1 = g0_any(w, sp, K1, g.n_lo + c1), g2 = g0_any(w, sp, K2, g.n_lo + c2);
  double2 v = cmul(cmul(g1, m), g2);
  v.x = -v.x / w.beta;
  v.y = -v.y / w.beta;
  if (K1 == K2 && c1 == c2) {
    v.x += g1.x;
    v.y += g1.y;
  }
  g.G[sp][(size_t)K1 * per + t] = v;
}

// G2[iq][K1][c1][K2][c2] += sign G_up(k1, k2) G_down(q - k1, q - k2) over the
// output grid c < 2 n_w4 (n = n_lo + c); q - k = (dK[Q][K], m - 1 - n).
// Thread per (c1, K2, c2); grid (ceil((2 n_w4)^2 Nc / WG), Nc K1, n_q).
template <typename T>
__global__ void __launch_bounds__(WG) k_g2_acc(const View<T>* __restrict__ vs, G2Dev g, int n4, int wm,
                                               const int* __restrict__ qs, const int* __restrict__ dK,
                                               double2* __restrict__ G2) {
  const View<T>& w = vs[0];
  const int Nc = w.Nc, nw = g.nw;
  const int K1 = blockIdx.y, iq = blockIdx.z;
  const long long t = (long long)blockIdx.x * WG + threadIdx.x;
  const long long per = (long long)n4 * Nc * n4;
  if (t >= per) return;
  const int c2 = (int)(t % n4);
  const int K2 = (int)((t / n4) % Nc);
  const int c1 = (int)(t / ((long long)n4 * Nc));
  const int Q = qs[iq];
  const int Kq1 = dK[Q * Nc + K1], Kq2 = dK[Q * Nc + K2];
  const int cq1 = (wm - 1 - (g.n_lo + c1)) - g.n_lo, cq2 = (wm - 1 - (g.n_lo + c2)) - g.n_lo;
  const long long gper = (long long)nw * Nc * nw;
  const double2 up = g.G[0][(size_t)K1 * gper + ((size_t)c1 * Nc + K2) * nw + c2];
  const double2 dn = g.G[1][(size_t)Kq1 * gper + ((size_t)cq1 * Nc + Kq2) * nw + cq2];
  const double s = w.ctl->sign;
  const double2 x = cmul(up, dn);
  double2* o = G2 + (size_t)iq * Nc * per + (size_t)K1 * per + t;
  o->x += s * x.x;
  o->y += s * x.y;
}

template <typename T>
__global__ void k_g2_sign(const View<T>* __restrict__ vs, double* sign_acc) {
  sign_acc[0] += vs[0].ctl->sign;
}

#define DCAX_INSTANTIATE_G2(T)                                                                   \
  template __global__ void k_g2_phase<T>(const View<T>*, G2Dev);                                 \
  template __global__ void k_g2_kphase<T>(const View<T>*, G2Dev);                                \
  template __global__ void k_g2_t1m<T>(const View<T>*, int, G2Dev);                              \
  template __global__ void k_g2_f<T>(const View<T>*, G2Dev);                                     \
  template __global__ void k_g2_k1<T>(const View<T>*, G2Dev);                                    \
  template __global__ void k_g2_g<T>(const View<T>*, int, G2Dev);                                \
  template __global__ void k_g2_acc<T>(const View<T>*, G2Dev, int, int, const int*, const int*, double2*); \
  template __global__ void k_g2_sign<T>(const View<T>*, double*);

DCAX_INSTANTIATE_G2(double)
DCAX_INSTANTIATE_G2(float)

}  // namespace dcax

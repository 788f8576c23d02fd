// Green's-function measurement, Sec. 2.3: per configuration and spin,
// M = (e^V - 1) N and
//   M(K, i w_n) = (1/Nc) sum_{ij} e^{i (w_n tau_i - K r_i)} M_ij e^{-i (w_n tau_j - K r_j)},
// accumulated with the configuration's sign; G = G0 - G0 <M> G0 / beta.
//
// The contraction is site-blocked: vertices are bucketed by site (each
// bucket padded to a multiple of 16), M is copied into that order, and
//   M(a, b; w_n) = sum_{i in a} e^{i w_n tau_i} sum_{j in b} M_ij e^{-i w_n tau_j}
// is formed for every pair of sites, the inner sum on the matrix cores (4 k^2
// N_w flops per spin rather than the 4 k^2 Nc N_w of the unblocked form): a
// wavefront takes one site b, a group of sites a and a tile of 16
// frequencies.  A small kernel then applies the momentum phases and adds
// sign * M(K, i w_n) to the caller's buffer.
#include "dcax_dev.h"

namespace dcax {

// Counting sort of the vertices by site, buckets padded to 16 rows.  The
// sites are staged in LDS; one wavefront per site places its vertices in
// their original order (stable).
constexpr int SORT_MAX = 32768 + 128;
template <typename T>
__global__ void __launch_bounds__(WG) k_meas_sort(const View<T>* __restrict__ vs, int gated) {
  const View<T>& w = vs[blockIdx.z];
  if (meas_skip(w.ctl, gated)) return;
  const auto order = gp(w.m_order);
  const auto off = gp(w.m_off);
  const auto v_site = gp(w.v_site);
  const int kpad_cap = w.kpad_cap;
  const int k = w.ctl->k;
  const int Nc = w.Nc;
  __shared__ int cnt_s[4097];  // [Nc + 1], Nc <= 4096
  __shared__ unsigned short site_s[SORT_MAX];
  for (int a = threadIdx.x; a <= Nc; a += WG) cnt_s[a] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += WG) {
    const int a = v_site[i];
    site_s[i] = (unsigned short)a;
    atomicAdd(&cnt_s[a], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int o = 0;
    for (int a = 0; a < Nc; ++a) {
      const int c = cnt_s[a];
      cnt_s[a] = o;
      o += (c + 15) & ~15;
    }
    cnt_s[Nc] = o;
  }
  __syncthreads();
  const int kpad = cnt_s[Nc];
  for (int a = threadIdx.x; a <= Nc; a += WG) off[a] = cnt_s[a];
  for (int i = threadIdx.x; i < kpad && i < kpad_cap; i += WG) order[i] = -1;
  __syncthreads();
  // stable placement: one wavefront per site at a time, the vertices in
  // chunks of 64 ranked by a ballot
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int a = threadIdx.x >> 6; a < Nc; a += WG / 64) {
    int o = cnt_s[a];
    for (int i0 = 0; i0 < k; i0 += 64) {
      const int i = i0 + lane;
      const bool hit = i < k && site_s[i] == a;
      const unsigned long long msk = __ballot(hit);
      if (hit) order[o + __popcll(msk & below)] = i;
      o += __popcll(msk);
    }
  }
}

// Ms[i'][j'] = (e^{V_i} - 1) N[i][j] in sorted order (zero on padding).
// Column by column: column j of N is read in its own order (coalesced) and
// scaled into LDS, then column j' of Ms is written in sorted order from LDS.
// One walker of the measurement's work list per blockIdx.y, columns
// grid-strided over blockIdx.x; orders up to MCOPY_ROWS.
constexpr int MCOPY_ROWS = 8192;
template <typename T>
__global__ void __launch_bounds__(WG) k_meas_copy(const View<T>* __restrict__ vs, const int* __restrict__ list) {
  if ((int)blockIdx.y >= list[0]) return;
  const View<T>& w = vs[list[1 + blockIdx.y]];
  __shared__ T col_s[MCOPY_ROWS];
  const auto order = gp(w.m_order);
  const auto off = gp(w.m_off);
  const auto v_s = gp(w.v_s);
  const int kpad = off[w.Nc];
  const int k = w.ctl->k;
  const size_t ldm = w.kpad_cap;
  const int t = threadIdx.x;
  for (int jp = blockIdx.x; jp < kpad; jp += gridDim.x) {
    const int j = order[jp];
#pragma unroll 1
    for (int sp = 0; sp < 2; ++sp) {
      const auto Ms = gp(w.m_Ms[sp]) + (size_t)jp * ldm;
      if (j < 0) {
        for (int ip = t; ip < kpad; ip += WG) Ms[ip] = (T)0;
        continue;
      }
      const auto Nj = gp(w.N[sp]) + (size_t)j * w.ld;
      const double fu = w.ev[sp][0] - 1.0, fd = w.ev[sp][1] - 1.0;
      // sixteen loads per thread in flight (two passes at most for the
      // largest order the LDS column holds)
      for (int i0 = t; i0 < k; i0 += 16 * WG) {
        T v[16];
        int sv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = i0 + u * WG < k ? i0 + u * WG : i0;
          v[u] = Nj[i];
          sv[u] = v_s[i];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (i0 + u * WG < k) col_s[i0 + u * WG] = (T)((sv[u] > 0 ? fu : fd) * (double)v[u]);
      }
      __syncthreads();
      for (int ip0 = t; ip0 < kpad; ip0 += 8 * WG) {
        int iv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) iv[u] = ip0 + u * WG < kpad ? order[ip0 + u * WG] : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (ip0 + u * WG < kpad) Ms[ip0 + u * WG] = iv[u] >= 0 ? col_s[iv[u]] : (T)0;
      }
      __syncthreads();
    }
  }
}

// The same copy for orders above MCOPY_ROWS: a gather from N by sorted row,
// in groups of 16 sorted columns (grid-strided over blockIdx.y, rows over x).
constexpr int MCOLS = 16;
template <typename T>
__global__ void __launch_bounds__(WG) k_meas_copy_wide(const View<T>* __restrict__ vs, int gated) {
  const View<T>& w = vs[blockIdx.z];
  if (meas_skip(w.ctl, gated)) return;
  const auto order = gp(w.m_order);
  const auto off = gp(w.m_off);
  const auto Ms0 = gp(w.m_Ms[0]);
  const auto Ms1 = gp(w.m_Ms[1]);
  const auto N0 = gp(w.N[0]);
  const auto N1 = gp(w.N[1]);
  const int ldm = w.kpad_cap;
  const int kpad = off[w.Nc];
  for (int ip = blockIdx.x * WG + threadIdx.x; ip < kpad; ip += gridDim.x * WG) {
    const int i = order[ip];
    double f0 = 0.0, f1 = 0.0;
    if (i >= 0) {
      const int si = s01(w.v_s[i]);
      f0 = w.ev[0][si] - 1.0;
      f1 = w.ev[1][si] - 1.0;
    }
    for (int j0 = blockIdx.y * MCOLS; j0 < kpad; j0 += gridDim.y * MCOLS)
      for (int jp = j0; jp < j0 + MCOLS && jp < kpad; ++jp) {
        const int j = order[jp];
        T v0 = 0, v1 = 0;
        if (i >= 0 && j >= 0) {
          const size_t o = i + (size_t)j * w.ld;
          v0 = (T)(f0 * (double)N0[o]);
          v1 = (T)(f1 * (double)N1[o]);
        }
        Ms0[ip + (size_t)jp * ldm] = v0;
        Ms1[ip + (size_t)jp * ldm] = v1;
      }
  }
}

// Phase table E[j'][n] = e^{-i w_n tau_j} in sorted order, in groups of 16
// rows (grid-strided over blockIdx.y).
template <typename T>
__global__ void __launch_bounds__(WG) k_meas_phase(const View<T>* __restrict__ vs, int gated) {
  const View<T>& w = vs[blockIdx.z];
  if (meas_skip(w.ctl, gated)) return;
  const auto order = gp(w.m_order);
  const auto off = gp(w.m_off);
  const auto E = gp(w.m_E);
  const int n_freq = w.n_freq;
  const int kpad = off[w.Nc];
  const int n = blockIdx.x * WG + threadIdx.x;
  if (n >= n_freq) return;
  const double wn = (2.0 * n + 1.0) * M_PI / w.beta;
  for (int j0 = blockIdx.y * MCOLS; j0 < kpad; j0 += gridDim.y * MCOLS)
    for (int jp = j0; jp < j0 + MCOLS && jp < kpad; ++jp) {
      const int j = order[jp];
      double c = 0.0, s = 0.0;
      if (j >= 0) sincos(wn * w.v_tau[j], &s, &c);
      E[2 * ((size_t)jp * n_freq + n)] = (T)c;
      E[2 * ((size_t)jp * n_freq + n) + 1] = (T)(-s);
    }
}

// Work items of the contraction: one per (walker, spin, site b, group of
// sites a, tile of 16 frequencies).  The sites a are split into groups so
// that even one walker alone gives at least MEAS_ITEMS items (wavefronts).
template <typename T> struct MeasTiles;                 // column blocks of 16 held in registers
template <> struct MeasTiles<float> { static constexpr int NB = 8; };
template <> struct MeasTiles<double> { static constexpr int NB = 4; };
constexpr int MEAS_ITEMS = 4096;

__host__ __device__ inline int meas_groups(int Nc, int n_freq) {
  const int base = 2 * Nc * ((n_freq + 15) / 16);
  const int ng = (MEAS_ITEMS + base - 1) / base;
  return ng < 1 ? 1 : (ng > Nc ? Nc : ng);
}
__host__ __device__ inline long long meas_items(int Nc, int n_freq) {
  return n_freq > 0 ? 2ll * Nc * meas_groups(Nc, n_freq) * ((n_freq + 15) / 16) : 0;
}

// Work list of one measurement launch: the walkers it covers (every walker,
// or under gating those whose sweep has just ended), list[0] = count and
// list[1 + c] = walker, and the prefix sums of their work items,
// pre[c] = items of the listed walkers before the c-th.  One wavefront,
// walkers in chunks of 64 (a scan over lanes per chunk).
template <typename T>
__global__ void __launch_bounds__(64) k_meas_list(const View<T>* __restrict__ vs, int W, int gated,
                                                  int* __restrict__ list, long long* __restrict__ pre) {
  const int lane = threadIdx.x;
  const unsigned long long below = (1ull << lane) - 1ull;
  int cnt = 0;
  long long run = 0;
  for (int z0 = 0; z0 < W; z0 += 64) {
    const int z = z0 + lane;
    bool on = false;
    long long items = 0;
    if (z < W) {
      const View<T>& w = vs[z];
      on = !meas_skip(w.ctl, gated);
      if (on) items = meas_items(w.Nc, w.n_freq);      // none without frequencies
    }
    long long sc = items;     // inclusive scan over the lanes
    for (int o = 1; o < 64; o <<= 1) {
      const long long v = __shfl_up(sc, o, 64);
      if (lane >= o) sc += v;
    }
    const unsigned long long msk = __ballot(on);
    if (on) {
      const int c = cnt + __popcll(msk & below);
      list[1 + c] = z;
      pre[c] = run + sc - items;
    }
    cnt += __popcll(msk);
    run += __shfl(sc, 63, 64);
  }
  if (lane == 0) {
    list[0] = cnt;
    pre[cnt] = run;
  }
}

// One chunk of NB column blocks of site b (columns jc .. jc + 16 NB) for the
// sites a0 .. a1 - 1 and the 16 frequencies from n0, on one wavefront.  The
// lane keeps its share of E[j][n] for the chunk in registers: in the 4-step
// product u of block q it supplies column j = jc + 16 q + 4 u + (lane >> 4)
// of frequency n0 + (lane & 15) (the A' operand) and M[i'][j] of row
// i' = ib + (lane & 15) (the B operand).  Per 16 rows of a:
//   D^T[n][i'] = sum_j E[j][n] Ms[i'][j]      (matrix cores)
// then the row phases e^{i w_n tau_i} = conj E[i'][n] and the sum over i'.
// The first chunk of b stores M(a, b; w_n), later chunks add to it.
// Loads through a buffer resource (base address in scalar registers): a
// lane offset in one vector register plus a wavefront-uniform offset in a
// scalar register, so a block of loads needs no address register each.
constexpr int BUF_WORD3 = 0x00020000;   // data format word of a raw buffer on gfx9
template <typename T> __device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so);
template <> __device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
template <> __device__ inline double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}

// One chunk of NB column blocks of site b (columns jc .. jc + 16 NB) for the
// sites a0 .. a1 - 1 and the 16 frequencies from n0, on one wavefront.  The
// lane keeps its share of E[j][n] for the chunk in registers: in the 4-step
// product u of block q it supplies column j = jc + 16 q + 4 u + (lane >> 4)
// of frequency n0 + (lane & 15) (the A' operand) and M[i'][j] of row
// i' = ib + (lane & 15) (the B operand).  Per 16 rows of a:
//   D^T[n][i'] = sum_j E[j][n] Ms[i'][j]      (matrix cores)
// then the row phases e^{i w_n tau_i} = conj E[i'][n] and the sum over i'.
// The first chunk of b stores M(a, b; w_n), later chunks add to it.  Offsets
// are taken from bases at the chunk's first column and the row block's
// first row, so they stay far below 2^32 bytes.
template <typename T, int NB>
__device__ void meas_chunk(const View<T>& w, int sp, int b, int jc, int a0, int a1, int n0, bool add) {
  typedef T t2 __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int n_freq = w.n_freq, Nc = w.Nc;
  const unsigned ldm = w.kpad_cap;
  const auto off = gp(w.m_off);
  const int na = n0 + li;
  const unsigned nac = na < n_freq ? na : 0;   // rows past n_freq are computed and never stored
  const auto Ej = gp((const t2*)w.m_E + (size_t)jc * n_freq);
  t2 e[NB][4];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) e[q][u] = Ej[(unsigned)(16 * q + 4 * u + lk) * (unsigned)n_freq + nac];
  const T* Mc = w.m_Ms[sp] + (size_t)jc * ldm;
  const size_t rem = ((size_t)w.kpad_cap - jc) * ldm * sizeof(T);
  const __amdgpu_buffer_rsrc_t rM =
      __builtin_amdgcn_make_buffer_rsrc((void*)Mc, (short)0, (int)(rem < 0x7fffffffu ? rem : 0x7fffffffu), BUF_WORD3);
  const unsigned vcol = (unsigned)lk * ldm * (unsigned)sizeof(T);
  unsigned rowph[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int n = n0 + Mfma<T>::row(lane, r);
    rowph[r] = (unsigned)li * n_freq + (n < n_freq ? n : 0);
  }
  const auto Mab = gp(w.m_Mab[sp]);
#pragma unroll 1
  for (int a = a0; a < a1; ++a) {
    double sre[4] = {0, 0, 0, 0}, sim[4] = {0, 0, 0, 0};
#pragma unroll 1
    for (int ib = off[a]; ib < off[a + 1]; ib += 16) {
      const unsigned vo = (unsigned)(ib + li) * (unsigned)sizeof(T) + vcol;
      T m[NB][4];
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) m[q][u] = buf_load<T>(rM, vo, (unsigned)(16 * q + 4 * u) * ldm * (unsigned)sizeof(T));
      const auto Ei = gp((const t2*)w.m_E + (size_t)ib * n_freq);
      t2 ph[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) ph[r] = Ei[rowph[r]];
      typename Mfma<T>::acc_t dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          dr = Mfma<T>::run(e[q][u].x, m[q][u], dr);
          di = Mfma<T>::run(e[q][u].y, m[q][u], di);
        }
      // lane holds D[n = n0 + row(lane, r)][i' = ib + li]; padding rows of
      // Ms and E are zero
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double c = (double)ph[r].x, s = -(double)ph[r].y;
        const double xr = (double)dr[r], xi = (double)di[r];
        sre[r] += c * xr - s * xi;
        sim[r] += c * xi + s * xr;
      }
    }
    // sum over the 16 lanes that share a frequency set (li varies)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      for (int o = 1; o < 16; o <<= 1) {
        sre[r] += __shfl_xor(sre[r], o, 64);
        sim[r] += __shfl_xor(sim[r], o, 64);
      }
    if (li == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + Mfma<T>::row(lane, r);
        if (n < n_freq) {
          const size_t o = 2 * (((size_t)a * Nc + b) * n_freq + n);
          Mab[o] = add ? Mab[o] + sre[r] : sre[r];
          Mab[o + 1] = add ? Mab[o + 1] + sim[r] : sim[r];
        }
      }
    }
  }
}

// The contraction for every pair of sites:
//   M(a, b; w_n) = sum_{i in a} e^{i w_n tau_i} sum_{j in b} Ms_ij e^{-i w_n tau_j}.
// A persistent grid takes the work items of the listed walkers (walker by
// walker: spins, b, groups of a, frequency tiles fastest), one per
// wavefront; the wavefronts working at one time thus share b's columns of
// Ms.  Workgroups are dealt to the eight XCDs in turn, so they are numbered
// here such that each XCD takes a contiguous range of items and its L2 holds
// the columns they share.
constexpr int XCDS = 8;
template <typename T>
__global__ void __launch_bounds__(WG, 2) k_meas_block(const View<T>* __restrict__ vs, const int* __restrict__ list,
                                                   const long long* __restrict__ pre) {
  constexpr int NB = MeasTiles<T>::NB;
  const int cnt = list[0];
  if (cnt == 0) return;
  const long long total = pre[cnt];
  // everything below is uniform over the wavefront (scalar registers)
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;     // a multiple of XCDS
  const int lb = (blockIdx.x % XCDS) * (nb / XCDS) + blockIdx.x / XCDS;
  for (long long it = (long long)lb * (WG / 64) + wv; it < total; it += (long long)nb * (WG / 64)) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const View<T>& w = vs[list[1 + lo]];
    const int n_freq = w.n_freq, Nc = w.Nc;
    const int nft = (n_freq + 15) / 16, ng = meas_groups(Nc, n_freq);
    long long r = it - pre[lo];
    const int n0 = 16 * (int)(r % nft);
    r /= nft;
    const int g = (int)(r % ng);
    r /= ng;
    const int b = (int)(r % Nc);
    const int sp = (int)(r / Nc);
    const int per = (Nc + ng - 1) / ng;
    const int a0 = g * per, a1 = min(Nc, a0 + per);
    if (a0 >= a1) continue;
    const auto off = gp(w.m_off);
    const int jb0 = off[b], jb1 = off[b + 1];
    if (jb0 == jb1) {
      // no vertex on site b
      const auto Mab = gp(w.m_Mab[sp]);
      for (int x = lane; x < (a1 - a0) * 16; x += 64) {
        const int n = n0 + (x & 15);
        if (n < n_freq) {
          const size_t o = 2 * (((size_t)(a0 + (x >> 4)) * Nc + b) * n_freq + n);
          Mab[o] = 0.0;
          Mab[o + 1] = 0.0;
        }
      }
      continue;
    }
    for (int jc = jb0; jc < jb1; jc += 16 * NB) {
      const int blocks = min(NB, (jb1 - jc) / 16);
      const bool add = jc > jb0;
      switch (blocks) {
        case 1: meas_chunk<T, 1>(w, sp, b, jc, a0, a1, n0, add); break;
        case 2: meas_chunk<T, 2>(w, sp, b, jc, a0, a1, n0, add); break;
        case 3: meas_chunk<T, 3>(w, sp, b, jc, a0, a1, n0, add); break;
        case 4: meas_chunk<T, 4>(w, sp, b, jc, a0, a1, n0, add); break;
        case 5: meas_chunk<T, (NB >= 5 ? 5 : 1)>(w, sp, b, jc, a0, a1, n0, add); break;
        case 6: meas_chunk<T, (NB >= 6 ? 6 : 1)>(w, sp, b, jc, a0, a1, n0, add); break;
        case 7: meas_chunk<T, (NB >= 7 ? 7 : 1)>(w, sp, b, jc, a0, a1, n0, add); break;
        default: meas_chunk<T, NB>(w, sp, b, jc, a0, a1, n0, add); break;
      }
    }
  }
}

// acc[sp][K][n] += sign (1/Nc) sum_ab e^{-i K (r_a - r_b)} M(a, b; w_n),
// with the site phases phi(K, a) = e^{-i K r_a} tabulated in LDS:
// e^{-i K (r_a - r_b)} = phi(K, a) conj(phi(K, b)).
constexpr int MEAS_NC_MAX = 256;
template <typename T>
__global__ void __launch_bounds__(WG) k_meas_K(const View<T>* __restrict__ vs, double* acc_all, int gated) {
  const View<T>& w = vs[blockIdx.z >> 1];
  if (meas_skip(w.ctl, gated)) return;
  const int sp = blockIdx.z & 1;
  const int Nc = w.Nc;
  const int n_freq = w.n_freq;
  const int n = blockIdx.x * WG + threadIdx.x;
  __shared__ double pr_s[MEAS_NC_MAX], pi_s[MEAS_NC_MAX];
  const auto Mab = gp(w.m_Mab[sp]);
  const auto acc = gp(acc_all + w.acc_off);
  const double sign = w.ctl->sign;
  // momenta q grid-strided over blockIdx.y
  for (int q = blockIdx.y; q < Nc; q += gridDim.y) {
    for (int a = threadIdx.x; a < Nc; a += WG) {
      const double ph = -(w.Kp[2 * q] * (double)w.sites[2 * a] + w.Kp[2 * q + 1] * (double)w.sites[2 * a + 1]);
      double s, c;
      sincos(ph, &s, &c);
      pr_s[a] = c;
      pi_s[a] = s;
    }
    __syncthreads();
    if (n < n_freq) {
      double re = 0.0, im = 0.0;
      for (int a = 0; a < Nc; ++a) {
        // t = sum_b conj(phi_b) M(a, b), sixteen loads of a row in flight
        // together and four independent partial sums
        double tr[4] = {0, 0, 0, 0}, ti[4] = {0, 0, 0, 0};
        const auto row = Mab + 2 * ((size_t)a * Nc * n_freq + n);
        int b = 0;
        for (; b + 16 <= Nc; b += 16) {
          double mr[16], mi[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            mr[u] = row[2 * (size_t)(b + u) * n_freq];
            mi[u] = row[2 * (size_t)(b + u) * n_freq + 1];
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            tr[u & 3] += pr_s[b + u] * mr[u] + pi_s[b + u] * mi[u];
            ti[u & 3] += pr_s[b + u] * mi[u] - pi_s[b + u] * mr[u];
          }
        }
        for (; b + 4 <= Nc; b += 4) {
          double mr[4], mi[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            mr[u] = row[2 * (size_t)(b + u) * n_freq];
            mi[u] = row[2 * (size_t)(b + u) * n_freq + 1];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            tr[u] += pr_s[b + u] * mr[u] + pi_s[b + u] * mi[u];
            ti[u] += pr_s[b + u] * mi[u] - pi_s[b + u] * mr[u];
          }
        }
        for (; b < Nc; ++b) {
          const double mr = row[2 * (size_t)b * n_freq], mi = row[2 * (size_t)b * n_freq + 1];
          tr[0] += pr_s[b] * mr + pi_s[b] * mi;
          ti[0] += pr_s[b] * mi - pi_s[b] * mr;
        }
        const double trs = (tr[0] + tr[1]) + (tr[2] + tr[3]), tis = (ti[0] + ti[1]) + (ti[2] + ti[3]);
        re += pr_s[a] * trs - pi_s[a] * tis;
        im += pr_s[a] * tis + pi_s[a] * trs;
      }
      const size_t o = 2 * (((size_t)sp * Nc + q) * n_freq + n);
      acc[o] += sign * re / (double)Nc;
      acc[o + 1] += sign * im / (double)Nc;
    }
    __syncthreads();      // the phase table is rewritten for the next momentum
  }
}

// aux += [sign, sign tr(M_up)/Nc, sign tr(M_dn)/Nc]; one block per spin.
template <typename T>
__global__ void __launch_bounds__(WG) k_meas_diag(const View<T>* __restrict__ vs, double* aux_all, int gated) {
  const View<T>& w = vs[blockIdx.z];
  if (meas_skip(w.ctl, gated)) return;
  double* aux = aux_all + 3 * (size_t)w.wid;
  const int sp = blockIdx.x;
  const double sign = w.ctl->sign;
  __shared__ double red[WG];
  const int k = w.ctl->k;
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += WG)
    s += (w.ev[sp][s01(w.v_s[i])] - 1.0) * (double)w.N[sp][i + (size_t)i * w.ld];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    aux[1 + sp] += sign * red[0] / (double)w.Nc;
    if (sp == 0) aux[0] += sign;
  }
}

// G0(K, i w_n): the caller's when it gave the propagator, else the isolated
// cluster's 1 / (i w_n - xi_K) = (-xi - i w) / (xi^2 + w^2).
template <typename T>
__device__ inline void g0_K_iw(const View<T>& w, int sp, int q, int n, double& gr, double& gi) {
  if (w.ext_g0) {
    const double* g = w.g0Kw + 2 * (((size_t)(w.spin_tables == 2 ? sp : 0) * w.Nc + q) * w.n_freq + n);
    gr = g[0];
    gi = g[1];
    return;
  }
  const double e = w.xi[q];
  const double wn = (2.0 * n + 1.0) * M_PI / w.beta;
  const double d = e * e + wn * wn;
  gr = -e / d;
  gi = -wn / d;
}

// G0(K, tau) for 0 <= tau <= beta: from the caller's table,
// sum_r e^{-i K r} G0(r, tau) (its real part: the tables of inversion-
// symmetric clusters are even in r), else the isolated cluster's closed form.
template <typename T>
__device__ inline double g0_K_tau(const View<T>& w, int sp, int q, double tau) {
  if (w.ext_g0) {
    const double Kx = w.Kp[2 * q], Ky = w.Kp[2 * q + 1];
    double s = 0.0;
    for (int d = 0; d < w.Nc; ++d)
      s += cos(Kx * w.sites[2 * d] + Ky * w.sites[2 * d + 1]) * g0_interp(w, sp, d, tau);
    return s;
  }
  const double e = w.xi[q], beta = w.beta;
  return (e >= 0.0) ? -exp(-e * tau) / (1.0 + exp(-beta * e)) : -exp(e * (beta - tau)) / (exp(beta * e) + 1.0);
}

// G(K, i w_n) = G0 - G0 <M> G0 / beta and the tail-corrected G(K, tau)
// (blockIdx.z = 2 walker + spin, blockIdx.y = momentum).
template <typename T>
__global__ void __launch_bounds__(WG) k_finalize(const View<T>* __restrict__ vs, const double* acc_all,
                                                 const double* aux_all, double* Giw_all, int n_tau_out,
                                                 double* Gtau_all) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int sp = blockIdx.z & 1;
  const int q = blockIdx.y;
  const int Nc = w.Nc, n_freq = w.n_freq;
  if (q >= Nc) return;
  const double beta = w.beta;
  const double* acc = acc_all + w.acc_off;
  double* Giw = Giw_all + w.acc_off;
  const double* aux = aux_all + 3 * (size_t)w.wid;
  const int x = blockIdx.x * WG + threadIdx.x;
  const double sgn = aux[0];
  if (x < n_freq) {
    double gr, gi;
    g0_K_iw(w, sp, q, x, gr, gi);
    const size_t o = 2 * (((size_t)sp * Nc + q) * n_freq + x);
    const double mr = acc[o] / sgn, mi = acc[o + 1] / sgn;
    const double g2r = gr * gr - gi * gi, g2i = 2.0 * gr * gi;
    Giw[o] = gr - (g2r * mr - g2i * mi) / beta;
    Giw[o + 1] = gi - (g2r * mi + g2i * mr) / beta;
  }
  if (Gtau_all && x < n_tau_out) {
    double* Gtau = Gtau_all + (size_t)2 * w.nc_prefix * n_tau_out;
    const double tau = (x == n_tau_out - 1) ? beta : (double)x * (beta / (double)(n_tau_out - 1));
    const double A = -(aux[1 + sp] / sgn) / beta;
    double s = 0.0;
    for (int n = 0; n < n_freq; ++n) {
      const double wn = (2.0 * n + 1.0) * M_PI / beta;
      double gr, gi;
      g0_K_iw(w, sp, q, n, gr, gi);
      const double g2r = gr * gr - gi * gi, g2i = 2.0 * gr * gi;
      const size_t o = 2 * (((size_t)sp * Nc + q) * n_freq + n);
      const double mr = acc[o] / sgn, mi = acc[o + 1] / sgn;
      const double dgr = -(g2r * mr - g2i * mi) / beta;
      const double dgi = -(g2r * mi + g2i * mr) / beta;
      // subtract the tail A / (i w)^2 = -A / w^2 (real)
      const double rr = dgr + A / (wn * wn), ri = dgi;
      double sn, cs;
      sincos(wn * tau, &sn, &cs);
      // Re[e^{-i w tau} (rr + i ri)] = cs rr + sn ri
      s += cs * rr + sn * ri;
    }
    const double g0 = g0_K_tau(w, sp, q, tau);
    Gtau[((size_t)sp * Nc + q) * n_tau_out + x] = g0 + (2.0 / beta) * s + A * (2.0 * tau - beta) / 4.0;
  }
}

#define DCAX_INSTANTIATE_MEASURE(T)                                                             \
  template __global__ void k_meas_sort<T>(const View<T>*, int);                                 \
  template __global__ void k_meas_copy<T>(const View<T>*, const int*);                          \
  template __global__ void k_meas_copy_wide<T>(const View<T>*, int);                            \
  template __global__ void k_meas_phase<T>(const View<T>*, int);                                \
  template __global__ void k_meas_list<T>(const View<T>*, int, int, int*, long long*);           \
  template __global__ void k_meas_block<T>(const View<T>*, const int*, const long long*);         \
  template __global__ void k_meas_K<T>(const View<T>*, double*, int);                           \
  template __global__ void k_meas_diag<T>(const View<T>*, double*, int);                        \
  template __global__ void k_finalize<T>(const View<T>*, const double*, const double*, double*, int, double*);

DCAX_INSTANTIATE_MEASURE(double)
DCAX_INSTANTIATE_MEASURE(float)

}  // namespace dcax

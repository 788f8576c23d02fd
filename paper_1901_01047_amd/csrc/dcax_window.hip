// Submatrix (delayed) update window of the CT-AUX walker, Sec. 2.3.
//
// A window takes up to k_s proposals.  Insertion candidates are drawn
// independently of the state, so their rows and columns of the extended
// walker matrix can be prepared before any decision; removal targets are
// existing vertices whose G columns follow from N itself through
// G (e^V - 1) = N e^V - 1.  The accept loop then runs every Metropolis
// decision in FP64 against a growing Gamma_S^{-1} (determinant ratios by
// Schur complements), and a rank-m fold brings N up to date:
//   N' = N + (E_S - G_{.S}) Gamma_S^{-1} N_{S.},
// followed by removal of the deleted rows and columns.  With G = N g and
// Delta_p = e^{V'_p - V_p} - 1: Gamma_S = G_SS - diag((1 + Delta)/Delta) and
// det N'^{-1} / det N^{-1} = prod_S (-Delta_p) det Gamma_S.
//
// Kernels, in launch order: k_prep_replay | k_prep_rng, k_gather, k_cand_x,
// k_gram, k_accept (which also plans the compaction and closes the window's
// bookkeeping), k_ygemm, k_fold_prep, k_fold, k_compact_move.  Each reads the
// window sizes from the control block and returns at once when the window is
// inactive, so the host may enqueue windows without reading anything back.
#include "dcax_dev.h"

namespace dcax {

// ------------------------------------------------------------------ prep
// Replay mode: the window's proposals come from a recorded trace with forced
// decisions.  Builds the element list: one element per insertion candidate
// and one per distinct window-start vertex proposed for removal; a removal
// of a vertex inserted earlier in the same window refers to that candidate.
template <typename T>
__global__ void __launch_bounds__(WG) k_prep_replay(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  Ctl* c = w.ctl;
  __shared__ long long tid_s[KS_MAX];
  __shared__ int tslot_s[KS_MAX];
  __shared__ int nP_s, k0_s;
  const int t = threadIdx.x;
  if (t == 0) {
    long long rem = c->end - c->pos;
    int nP = (c->status == 0 && rem > 0) ? (int)(rem < w.ks ? rem : w.ks) : 0;
    nP_s = nP;
    k0_s = c->k;
    if (nP == 0) c->active = 0;
  }
  __syncthreads();
  const int nP = nP_s, k0 = k0_s;
  if (nP == 0) return;
  const long long pos = c->pos;
  if (t < nP) {
    const dcax_proposal& r = w.replay[pos + t];
    tid_s[t] = (r.kind == 1) ? r.id : -2;
    tslot_s[t] = -1;
  }
  __syncthreads();
  for (int i = t; i < k0; i += WG) {
    long long id = w.v_id[i];
    for (int j = 0; j < nP; ++j)
      if (tid_s[j] == id) tslot_s[j] = i;
  }
  __syncthreads();
  if (t != 0) return;
  int nE = 0, nC = 0;
  long long next_id = c->next_id;
  for (int j = 0; j < nP; ++j) {
    const dcax_proposal& r = w.replay[pos + j];
    WinProp p;
    p.kind = r.kind;
    p.forced = r.accepted ? 1 : 0;
    p.carried = 0;
    p.u = r.u_accept;
    p.ridx = pos + j;
    p.gidx = pos + j;
    p.el = -1;
    if (r.kind == 0) {
      int e = nE++, cc = nC++;
      w.el_site[e] = r.site;
      w.el_tau[e] = r.tau;
      w.el_s[e] = r.aux_spin;
      w.el_slot[e] = -1;
      w.el_cand[e] = cc;
      w.cand_el[cc] = e;
      w.cand_id[cc] = r.accepted ? r.id : -1;
      if (r.accepted && r.id >= next_id) next_id = r.id + 1;
      p.el = e;
    } else if (r.id >= 0) {
      int e = -1;
      for (int cc = 0; cc < nC; ++cc)
        if (w.cand_id[cc] == r.id) e = w.cand_el[cc];
      if (e < 0) {
        int slot = tslot_s[j];
        if (slot < 0) {
          latch(c, ST_TRACE);
          c->active = 0;
          return;
        }
        for (int x = 0; x < nE; ++x)
          if (w.el_slot[x] == slot) e = x;
        if (e < 0) {
          e = nE++;
          w.el_site[e] = w.v_site[slot];
          w.el_tau[e] = w.v_tau[slot];
          w.el_s[e] = w.v_s[slot];
          w.el_slot[e] = slot;
          w.el_cand[e] = -1;
        }
      }
      p.el = e;
    }
    w.wp[j] = p;
  }
  c->next_id = next_id;
  c->nP = nP;
  c->nE = nE;
  c->nC = nC;
  c->k0 = k0;
  c->active = 1;
}


// Generator mode.  Proposal g draws: slot 0 -> (u_kind, u_site), slot 1 ->
// (u_tau, u_spin), slot 2 -> (u_accept, -), slot 3 + a -> the a-th attempt
// (u_branch, u_index) of a removal target.  Insertions are state-independent
// and become candidates; a removal pre-selects the window-start vertex its
// first attempt would hit (floor(u_index k0)).  A removal carried over from
// an aborted window keeps the target it had already chosen.
template <typename T>
__global__ void __launch_bounds__(WG) k_prep_rng(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const uint64_t seed = w.seed;
  Ctl* c = w.ctl;
  __shared__ int nP_s, k0_s, carry_slot_s;
  __shared__ long long carry_s;
  const int t = threadIdx.x;
  if (t == 0) {
    long long rem = c->end - c->pos;
    int nP = (c->status == 0 && rem > 0) ? (int)(rem < w.ks ? rem : w.ks) : 0;
    nP_s = nP;
    k0_s = c->k;
    carry_s = c->carry_id;
    carry_slot_s = -1;
    if (nP == 0) c->active = 0;
  }
  __syncthreads();
  const int nP = nP_s, k0 = k0_s;
  if (nP == 0) return;
  const long long carry = carry_s;
  if (carry >= 0)
    for (int i = t; i < k0; i += WG)
      if (w.v_id[i] == carry) carry_slot_s = i;
  // the window's uniforms, one proposal per thread
  __shared__ double u_s[KS_MAX][5];
  __shared__ int slot0_s[KS_MAX];
  const long long pos = c->pos;
  if (t < nP) {
    const long long g = pos + t;
    double u_dummy;
    uniforms2(seed, g, 0u, u_s[t][0], u_s[t][1]);
    uniforms2(seed, g, 1u, u_s[t][2], u_s[t][3]);
    uniforms2(seed, g, 2u, u_s[t][4], u_dummy);
    int slot = -1;
    if (k0 > 0) {
      double ub, ui;
      uniforms2(seed, g, 3u, ub, ui);
      slot = (int)(ui * (double)k0);
      if (slot >= k0) slot = k0 - 1;
    }
    slot0_s[t] = slot;
  }
  __syncthreads();
  if (t != 0) return;
  int nE = 0, nC = 0;
  for (int j = 0; j < nP; ++j) {
    const long long g = pos + j;
    const double u_kind = u_s[j][0], u_site = u_s[j][1], u_tau = u_s[j][2], u_spin = u_s[j][3];
    const double u_acc = u_s[j][4];
    WinProp p;
    p.forced = -1;
    p.carried = 0;
    p.u = u_acc;
    p.ridx = -1;
    p.gidx = g;
    p.el = -1;
    int slot = -1;
    if (j == 0 && carry >= 0) {
      p.kind = 1;
      p.carried = 1;
      slot = carry_slot_s;
      if (slot < 0) {
        latch(c, ST_TRACE);
        c->active = 0;
        return;
      }
    } else if (u_kind < 0.5) {
      p.kind = 0;
      int site = (int)(u_site * (double)w.Nc);
      if (site >= w.Nc) site = w.Nc - 1;
      const int e = nE++, cc = nC++;
      w.el_site[e] = site;
      w.el_tau[e] = u_tau * w.beta;
      w.el_s[e] = (u_spin < 0.5) ? 1 : -1;
      w.el_slot[e] = -1;
      w.el_cand[e] = cc;
      w.cand_el[cc] = e;
      w.cand_id[cc] = -1;
      p.el = e;
    } else {
      p.kind = 1;
      slot = slot0_s[j];     // the first attempt's window-start vertex
    }
    if (slot >= 0) {
      int e = -1;
      for (int x = 0; x < nE; ++x)
        if (w.el_slot[x] == slot) e = x;
      if (e < 0) {
        e = nE++;
        w.el_site[e] = w.v_site[slot];
        w.el_tau[e] = w.v_tau[slot];
        w.el_s[e] = w.v_s[slot];
        w.el_slot[e] = slot;
        w.el_cand[e] = -1;
      }
      p.el = e;
    }
    w.wp[j] = p;
  }
  c->carry_id = -1;
  c->nP = nP;
  c->nE = nE;
  c->nC = nC;
  c->k0 = k0;
  c->active = 1;
}

// ---------------------------------------------------------------- gather
// Candidate columns g_{I,c}, candidate rows W_c = g_{c,I} (e^{V_I} - 1) for
// both spins, candidate-candidate entries g_{c,c'}, and the rows N_{p.} of
// the removal targets copied out contiguously.
template <typename T>
__global__ void __launch_bounds__(WG) k_gather(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  T* R0 = w.R[0];
  T* R1 = w.R[1];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int e = blockIdx.y;
  if (e >= c->nE) return;
  const int k0 = c->k0;
  const int i = blockIdx.x * WG + threadIdx.x;
  const int cc = w.el_cand[e];
  if (cc >= 0) {
    const int rc = w.el_site[e];
    const double tc = w.el_tau[e];
    if (i < k0) {
      const int ri = w.v_site[i];
      const double ti = w.v_tau[i];
      const int si = s01(w.v_s[i]);
      const double gic = gfun(w, ri, ti, rc, tc);
      const double gci = gfun(w, rc, tc, ri, ti);
      const size_t o = (size_t)cc * w.cap + i;
      w.gcol[o] = (T)gic;
      w.W[0][o] = (T)(gci * (w.ev[0][si] - 1.0));
      w.W[1][o] = (T)(gci * (w.ev[1][si] - 1.0));
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < c->nC) {
      const int e2 = w.cand_el[threadIdx.x];
      w.gCC[cc * KS_MAX + threadIdx.x] = gfun(w, rc, tc, w.el_site[e2], w.el_tau[e2]);
    }
  } else if (i < k0) {
    const int p = w.el_slot[e];
    const size_t o = (size_t)e * w.cap + i;
    R0[o] = w.N[0][p + (size_t)i * w.ld];
    R1[o] = w.N[1][p + (size_t)i * w.ld];
  }
}

// ------------------------------------------------------- candidate rows
// X_c = W_c N for all candidates and both spins (an nC x k0 x k0 GEMM on the
// matrix cores), written as rows e = element(c) of R.  Tiles of N are staged
// through LDS so that HBM reads run down the columns.
template <typename T>
__global__ void __launch_bounds__(WG) k_cand_x(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int nC = c->nC;
  const int k0 = c->k0;
  const int j0 = blockIdx.x * 64;
  if (nC == 0 || j0 >= k0) return;
  const int sp = blockIdx.y;
  const T* N = w.N[sp];
  const T* Wm = w.W[sp];
  T* R = w.R[sp];
  __shared__ T As[64][17];
  __shared__ T Bs[16][65];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nRB = (nC + 15) >> 4;
  typename Mfma<T>::acc_t acc[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) acc[rb] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  for (int i0 = 0; i0 < k0; i0 += 16) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = t & 15, col = (t >> 4) + 16 * p;
      const int gi = i0 + r, gj = j0 + col;
      Bs[r][col] = (gi < k0 && gj < k0) ? N[gi + (size_t)gj * w.ld] : (T)0;
      const int cr = (t >> 4) + 16 * p;
      As[cr][r] = (cr < nC && gi < k0) ? Wm[(size_t)cr * w.cap + gi] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const T b = Bs[kk * 4 + (lane >> 4)][wv * 16 + (lane & 15)];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        if (rb < nRB) {
          const T a = As[rb * 16 + (lane & 15)][kk * 4 + (lane >> 4)];
          acc[rb] = Mfma<T>::run(a, b, acc[rb]);
        }
    }
    __syncthreads();
  }
  const int col = j0 + wv * 16 + (lane & 15);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
    if (rb < nRB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cr = rb * 16 + Mfma<T>::row(lane, r);
        if (cr < nC && col < k0) R[(size_t)w.cand_el[cr] * w.cap + col] = acc[rb][r];
      }
    }
}

// -------------------------------------------------------------- Gram
// G restricted to the window elements, both spins, in FP64:
//   column of a candidate c:  G_{x,c} = R_x . g_{I,c} (+ g_{x,c} for candidate rows x)
//   column of a target p:     G_{x,p} = (e^{V_p} R_x[p] - delta_{xp}) / (e^{V_p} - 1)
// where R_x is row x of the extended N (X_c for candidates, N_{p.} for targets).
template <typename T>
__global__ void __launch_bounds__(WG) k_gram(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int x = blockIdx.x, sp = blockIdx.y;
  const int nE = c->nE;
  if (x >= nE) return;
  const int k0 = c->k0, nC = c->nC;
  const int cx = w.el_cand[x];
  const T* Rx = w.R[sp] + (size_t)x * w.cap;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* G = w.gram[sp] + x * KS_MAX;
  for (int cc = wv; cc < nC; cc += WG / 64) {
    const T* gc = w.gcol + (size_t)cc * w.cap;
    double s = 0.0;
    for (int i = lane; i < k0; i += 64) s += (double)Rx[i] * (double)gc[i];
    s = wave_sum(s);
    if (lane == 0) G[w.cand_el[cc]] = s + (cx >= 0 ? w.gCC[cx * KS_MAX + cc] : 0.0);
  }
  for (int y = threadIdx.x; y < nE; y += WG) {
    const int py = w.el_slot[y];
    if (py < 0) continue;
    const double ev = w.ev[sp][s01(w.el_s[y])];
    G[y] = (ev * (double)Rx[py] - (y == x ? 1.0 : 0.0)) / (ev - 1.0);
  }
}

// ---------------------------------------------------------- accept loop
// The sequential Metropolis decisions of the window (one workgroup, FP64).
// Adding q to S multiplies the determinant ratio by
//   (-Delta_q) (Gamma_qq - Gamma_qS Gamma_S^{-1} Gamma_Sq);
// taking an inserted spin out again (its removal later in the same window)
// multiplies it by (Gamma_S^{-1})_qq / (-Delta_q).  The acceptance ratio is
// K/(k+1) or k/K times the product over both spins (Sec. 2.3 weights).
//
// Generator mode picks a removal target uniformly among the current vertices
// by rejection: attempt a draws (u_b, u_i); with u_b (k0 + n_ins) < k0 it
// proposes window-start slot floor(u_i k0) and redraws if that vertex was
// already removed, otherwise the floor(u_i n_ins)-th spin inserted in this
// window.  Each current vertex has probability 1 / (k0 + n_ins) per attempt.
// A later attempt that lands on a window-start vertex whose rows were not
// prepared closes the window before this proposal and carries the chosen
// target into the next one (the paper's "abort" treatment; exact, since the
// state does not change in between).
constexpr int MAX_ATTEMPTS = 1 << 16;

template <typename T>
__global__ void __launch_bounds__(WG) k_accept(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  int* el_row = w.el_row;
  int* remap = w.remap;
  int* moves = w.moves;
  const uint64_t seed = w.seed;
  Ctl* c = w.ctl;
  if (!c->active) return;
  // LDS rows are padded to LS doubles: with a stride of 64 doubles every lane
  // reading one column of a tile would hit the same bank.
  constexpr int LS = KS_MAX + 1;
  __shared__ double gram_s[2][KS_MAX * LS];
  __shared__ double ginv_s[2][KS_MAX * LS];
  __shared__ double Lv[2][KS_MAX], Rv[2][KS_MAX], dl_s[2][KS_MAX];
  __shared__ int S_s[KS_MAX], pos_s[KS_MAX], insl_s[KS_MAX];
  __shared__ double rat_s[2], schur_s[2], D_s[2];
  __shared__ int m_s, acc_s, kcur_s, q_s, abort_s, nins_s;
  __shared__ double sign_s;
  // everything the sequential loop touches per proposal lives in LDS
  __shared__ WinProp wp_s[KS_MAX];
  __shared__ int cand_s[KS_MAX], spin_s[KS_MAX], slot_s[KS_MAX];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nE = c->nE, nP = c->nP, k0 = c->k0;
  for (int idx = t; idx < 2 * KS_MAX * KS_MAX; idx += WG) {
    const int sp = idx / (KS_MAX * KS_MAX), r = idx % (KS_MAX * KS_MAX);
    const int ra = r / KS_MAX, rb = r % KS_MAX;
    gram_s[sp][ra * LS + rb] = (ra < nE && rb < nE) ? w.gram[sp][r] : 0.0;
  }
  if (t < KS_MAX) pos_s[t] = -1;
  if (t < nP) wp_s[t] = w.wp[t];
  if (t < nE) {
    cand_s[t] = w.el_cand[t];
    spin_s[t] = w.el_s[t];
    slot_s[t] = w.el_slot[t];
  }
  if (t == 0) {
    m_s = 0;
    nins_s = 0;
    kcur_s = k0;
    sign_s = c->sign;
  }
  __syncthreads();
  long long n_ins = 0, n_rem = 0, n_mis = 0;
  long long next_id = c->next_id;
  long long carry = -1;
  int bad = 0, n_done = nP;
  for (int j = 0; j < nP; ++j) {
    const WinProp p = wp_s[j];
    if (t == 0) {
      int q = p.el, ab = 0;
      if (p.forced < 0 && p.kind == 1 && !p.carried) {
        q = -1;
        const int kc = kcur_s, ni = nins_s;
        if (kc > 0) {
          for (int a = 0; a < MAX_ATTEMPTS; ++a) {
            double ub, ui;
            uniforms2(seed, p.gidx, 3u + (uint32_t)a, ub, ui);
            if (ub * (double)(k0 + ni) < (double)k0) {
              int slot = (int)(ui * (double)k0);
              if (slot >= k0) slot = k0 - 1;
              int e = -1;
              if (a == 0) {
                e = p.el;
              } else {
                for (int x = 0; x < nE; ++x)
                  if (slot_s[x] == slot) e = x;
              }
              if (e >= 0 && pos_s[e] >= 0) continue;
              if (e < 0) {
                ab = 1;
                carry = w.v_id[slot];
                break;
              }
              q = e;
              break;
            }
            int idx = (int)(ui * (double)ni);
            if (idx >= ni) idx = ni - 1;
            q = insl_s[idx];
            break;
          }
          if (q < 0 && !ab) bad = 1;
        }
      }
      q_s = q;
      abort_s = ab;
    }
    __syncthreads();
    if (abort_s) {
      n_done = j;
      break;
    }
    const int q = q_s;
    const int m = m_s;
    if (q < 0) {
      if (t == 0 && p.ridx >= 0) w.ratio_out[p.ridx] = 0.0;
      continue;
    }
    const int pq = pos_s[q];
    const int is_c = cand_s[q] >= 0;
    if (pq >= 0) {
      if (t < 2) rat_s[t] = ginv_s[t][pq * LS + pq] / (-dl_s[t][pq]);
    } else if (wv < 2) {
      const int sp = wv;
      const double ev = w.ev[sp][s01(spin_s[q])];
      const double D = is_c ? ev - 1.0 : 1.0 / ev - 1.0;
      double L = 0.0;
      if (lane < m) {
        for (int b = 0; b < m; ++b) L += ginv_s[sp][lane * LS + b] * gram_s[sp][S_s[b] * LS + q];
        Lv[sp][lane] = L;
      }
      double part = (lane < m) ? gram_s[sp][q * LS + S_s[lane]] * L : 0.0;
      part = wave_sum(part);
      if (lane == 0) {
        const double sch = gram_s[sp][q * LS + q] - (1.0 + D) / D - part;
        schur_s[sp] = sch;
        D_s[sp] = D;
        rat_s[sp] = -D * sch;
      }
    }
    __syncthreads();
    if (t == 0) {
      const int kc = kcur_s;
      const double fac = (p.kind == 0) ? w.K_exp / (double)(kc + 1) : (double)kc / w.K_exp;
      const double R = fac * rat_s[0] * rat_s[1];
      int dec;
      if (!isfinite(R)) {
        bad = 1;
        dec = 0;
      } else {
        const int mine = p.u < fabs(R);
        dec = (p.forced >= 0) ? p.forced : mine;
        if (p.forced >= 0 && mine != p.forced) ++n_mis;
      }
      if (p.ridx >= 0) w.ratio_out[p.ridx] = R;
      if (dec && p.kind == 0 && kc + 1 > w.max_order) {
        latch(c, ST_CAPACITY);
        dec = 0;
      }
      acc_s = dec;
      if (dec) {
        kcur_s = kc + (p.kind == 0 ? 1 : -1);
        if (R < 0.0) sign_s = -sign_s;
        if (p.kind == 0) {
          ++n_ins;
          const int cc = cand_s[q];
          if (p.forced < 0) w.cand_id[cc] = next_id++;
          insl_s[nins_s++] = q;
        } else {
          ++n_rem;
          if (pq >= 0) {
            int x = 0;
            while (insl_s[x] != q) ++x;
            for (; x + 1 < nins_s; ++x) insl_s[x] = insl_s[x + 1];
            --nins_s;
          }
        }
      }
    }
    __syncthreads();
    if (!acc_s) continue;
    if (pq < 0) {
      if (wv < 2) {
        const int sp = wv;
        if (lane < m) {
          double Rr = 0.0;
          for (int a = 0; a < m; ++a) Rr += gram_s[sp][q * LS + S_s[a]] * ginv_s[sp][a * LS + lane];
          Rv[sp][lane] = Rr;
        }
      }
      __syncthreads();
      const int mm = m + 1;
      for (int idx = t; idx < 2 * mm * mm; idx += WG) {
        const int sp = idx / (mm * mm), r = idx % (mm * mm), a = r / mm, b = r % mm;
        const double inv = 1.0 / schur_s[sp];
        double v;
        if (a < m && b < m) v = ginv_s[sp][a * LS + b] + Lv[sp][a] * Rv[sp][b] * inv;
        else if (a == m && b < m) v = -Rv[sp][b] * inv;
        else if (a < m) v = -Lv[sp][a] * inv;
        else v = inv;
        ginv_s[sp][a * LS + b] = v;
      }
      __syncthreads();
      if (t == 0) {
        S_s[m] = q;
        pos_s[q] = m;
        dl_s[0][m] = D_s[0];
        dl_s[1][m] = D_s[1];
        m_s = mm;
      }
      __syncthreads();
    } else {
      const int js = pq, last = m - 1;
      if (t < 2 * m) {
        const int sp = t / m, a = t % m;
        Lv[sp][a] = ginv_s[sp][a * LS + js];
        Rv[sp][a] = ginv_s[sp][js * LS + a];
      }
      __syncthreads();
      for (int idx = t; idx < 2 * m * m; idx += WG) {
        const int sp = idx / (m * m), r = idx % (m * m), a = r / m, b = r % m;
        ginv_s[sp][a * LS + b] -= Lv[sp][a] * Rv[sp][b] / Lv[sp][js];
      }
      __syncthreads();
      if (js != last) {
        for (int idx = t; idx < 2 * m; idx += WG) {
          const int sp = idx / m, b = idx % m;
          ginv_s[sp][js * LS + b] = ginv_s[sp][last * LS + b];
        }
        __syncthreads();
        for (int idx = t; idx < 2 * m; idx += WG) {
          const int sp = idx / m, a = idx % m;
          ginv_s[sp][a * LS + js] = ginv_s[sp][a * LS + last];
        }
      }
      __syncthreads();
      if (t == 0) {
        const int el_last = S_s[last];
        S_s[js] = el_last;
        pos_s[el_last] = js;
        dl_s[0][js] = dl_s[0][last];
        dl_s[1][js] = dl_s[1][last];
        pos_s[q] = -1;
        m_s = last;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const int m = m_s;
  for (int idx = t; idx < 2 * m * m; idx += WG) {
    const int sp = idx / (m * m), r = idx % (m * m), a = r / m, b = r % m;
    w.ginv[sp][a * KS_MAX + b] = ginv_s[sp][a * LS + b];
  }
  // Epilogue: the fold's column order, the new vertex arrays and the plan
  // that removes the deleted rows and columns of N.  Inserted spins take
  // slots k0 .. k0+mi-1; holes left below the new order are filled from the
  // surviving slots above it (remap[dst] = src, moves[] = (dst, src) pairs).
  // Nothing later in the window reads the vertex arrays or the order, so
  // both are final here.
  __shared__ int ins_s[KS_MAX], hole_s[KS_MAX], src_s[KS_MAX], rem[KS_MAX], mi_s, nh_s;
  const int knew = kcur_s;
  if (t == 0) {
    int mi = 0, mr = 0;
    for (int s = 0; s < m; ++s) {
      const int e = S_s[s];
      w.S[s] = e;
      if (cand_s[e] >= 0) {
        ins_s[mi] = e;
        w.ins_el[mi] = e;
        el_row[e] = k0 + mi;
        ++mi;
      } else {
        el_row[e] = slot_s[e];
        rem[mr++] = slot_s[e];
      }
    }
    for (int a = 1; a < mr; ++a)
      for (int b = a; b > 0 && rem[b - 1] > rem[b]; --b) {
        const int x = rem[b];
        rem[b] = rem[b - 1];
        rem[b - 1] = x;
      }
    const int kx = k0 + mi;
    int nh = 0, ns = 0, r = 0;
    for (int a = 0; a < mr; ++a)
      if (rem[a] < knew) hole_s[nh++] = rem[a];
    for (int i = knew; i < kx; ++i) {
      while (r < mr && rem[r] < i) ++r;
      if (r < mr && rem[r] == i) continue;
      src_s[ns++] = i;
    }
    for (int h = 0; h < nh; ++h) {
      moves[2 * h] = hole_s[h];
      moves[2 * h + 1] = src_s[h];
    }
    moves[2 * KS_MAX] = nh;
    mi_s = mi;
    nh_s = nh;
    if (bad) latch(c, ST_NUMERIC);
    c->m = m;
    c->mi = mi;
    c->mr = mr;
    c->kx = kx;
    c->knew = knew;
    c->k = knew;
    c->sign = sign_s;
    c->next_id = next_id;
    c->n_prop += n_done;
    c->n_acc_ins += n_ins;
    c->n_acc_rem += n_rem;
    c->n_mismatch += n_mis;
    c->pos += n_done;
    c->n_windows += 1;
    if (carry >= 0) {
      c->carry_id = carry;
      c->n_abort += 1;
    }
    if (m > 0) {
      const double x = (double)kx;
      c->fold_flops += 2.0 * 2.0 * x * x * (double)m;
      c->fold_bytes += 2.0 * 2.0 * x * x * (double)sizeof(T);
      c->n_folds += 1;
      c->sum_m += m;
    } else {
      c->active = 0;      // nothing to fold: the window ends here
    }
  }
  __syncthreads();
  const int mi = mi_s, nh = nh_s;
  if (m == 0) return;
  for (int i = t; i < knew; i += WG) remap[i] = i;
  if (t < mi) {
    const int e = ins_s[t];
    w.v_site[k0 + t] = w.el_site[e];
    w.v_tau[k0 + t] = w.el_tau[e];
    w.v_s[k0 + t] = spin_s[e];
    w.v_id[k0 + t] = w.cand_id[cand_s[e]];
  }
  __syncthreads();
  if (t < nh) {
    const int d = hole_s[t], sidx = src_s[t];
    remap[d] = sidx;
    w.v_site[d] = w.v_site[sidx];
    w.v_tau[d] = w.v_tau[sidx];
    w.v_s[d] = w.v_s[sidx];
    w.v_id[d] = w.v_id[sidx];
  }
}

// --------------------------------------------------------- Y = N g_{I,c}
// Columns G_{I,c} = N g_{I,c} for the inserted spins (a k0 x k0 x mi GEMM).
template <typename T>
__global__ void __launch_bounds__(WG) k_ygemm(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int mi = c->mi, k0 = c->k0;
  const int i0 = blockIdx.x * 64;
  if (mi == 0 || i0 >= k0) return;
  const int sp = blockIdx.y;
  const T* N = w.N[sp];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ncb = (mi + 15) >> 4;
  const T* gp[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int jj = cb * 16 + (lane & 15);
    gp[cb] = (jj < mi) ? w.gcol + (size_t)w.el_cand[w.ins_el[jj]] * w.cap : nullptr;
  }
  typename Mfma<T>::acc_t acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  const int ii = i0 + wv * 16 + (lane & 15);
  for (int j = 0; j < k0; j += 4) {
    const int jk = j + (lane >> 4);
    const T a = (ii < k0 && jk < k0) ? N[ii + (size_t)jk * w.ld] : (T)0;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      if (cb < ncb) {
        const T b = (gp[cb] != nullptr && jk < k0) ? gp[cb][jk] : (T)0;
        acc[cb] = Mfma<T>::run(a, b, acc[cb]);
      }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
    if (cb < ncb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wv * 16 + Mfma<T>::row(lane, r);
        const int jj = cb * 16 + (lane & 15);
        if (i < k0 && jj < mi) w.Y[sp][(size_t)jj * w.cap + i] = acc[cb][r];
      }
    }
}

// ------------------------------------------------------------ fold prep
// Fold factors in the extended index space (window-start vertices, then the
// inserted spins at rows k0 .. k0+mi-1):
//   A = E_S - G_{.S}: an inserted spin's column is e - [N g_{I,c}; G_{C,c}],
//     a removed vertex p's column is (e^{V_p} / (e^{V_p} - 1)) (e_p - N_{.p});
//   B = Gamma_S^{-1} N_{S.} with the rows of the extended N;
// and the extension of N itself: row k0+j = X_c, column k0+j = e_{k0+j}.
template <typename T>
__global__ void __launch_bounds__(WG) k_fold_prep(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const int* el_row = w.el_row;
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int m = c->m;
  const int sp = blockIdx.y;
  const int k0 = c->k0, mi = c->mi, kx = k0 + mi;
  __shared__ double gi_s[KS_MAX * KS_MAX];
  __shared__ int e_s[KS_MAX], row_s[KS_MAX], cand_s[KS_MAX], slot_s[KS_MAX], ins_s[KS_MAX];
  __shared__ double f_s[KS_MAX];
  const int t = threadIdx.x;
  // the product below runs over all KS_MAX columns: entries beyond m must be
  // zero, not whatever an earlier kernel left in LDS
  for (int idx = t; idx < KS_MAX * KS_MAX; idx += WG) {
    const int a = idx / KS_MAX, b = idx % KS_MAX;
    gi_s[idx] = (a < m && b < m) ? w.ginv[sp][idx] : 0.0;
  }
  if (t < m) {
    const int e = w.S[t];
    e_s[t] = e;
    row_s[t] = el_row[e];
    cand_s[t] = w.el_cand[e];
    slot_s[t] = w.el_slot[e];
    const double ev = w.ev[sp][s01(w.el_s[e])];
    f_s[t] = ev / (ev - 1.0);
  }
  if (t < mi) ins_s[t] = w.ins_el[t];
  __syncthreads();
  const int i = blockIdx.x * WG + t;
  if (i >= kx) return;
  const T* R = w.R[sp];
  T* N = w.N[sp];
  const size_t ld = w.ld;
  // A, column-major [s][i]
  for (int s = 0; s < m; ++s) {
    double v;
    if (cand_s[s] >= 0) {
      const int jj = row_s[s] - k0;
      if (i < k0) v = -(double)w.Y[sp][(size_t)jj * w.cap + i];
      else v = -w.gram[sp][ins_s[i - k0] * KS_MAX + e_s[s]] + (i - k0 == jj ? 1.0 : 0.0);
    } else {
      const int p = slot_s[s];
      const double nip = (i < k0) ? (double)N[i + (size_t)p * ld] : (double)R[(size_t)ins_s[i - k0] * w.cap + p];
      v = f_s[s] * ((i == p ? 1.0 : 0.0) - nip);
    }
    w.A[sp][(size_t)s * w.cap + i] = (T)v;
  }
  // B, row-major [a][i] = sum_b Gamma^{-1}[a][b] Row_{S_b}[i]
  double rv[KS_MAX];
#pragma unroll
  for (int b = 0; b < KS_MAX; ++b) {
    double x = 0.0;
    if (b < m) {
      if (i < k0) x = (double)R[(size_t)e_s[b] * w.cap + i];
      else x = (cand_s[b] >= 0 && row_s[b] == i) ? 1.0 : 0.0;
    }
    rv[b] = x;
  }
  for (int a = 0; a < m; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < KS_MAX; ++b) s += gi_s[a * KS_MAX + b] * rv[b];
    w.B[sp][(size_t)a * w.cap + i] = (T)s;
  }
  // extension of N (reads above touch only rows and columns < k0 of N)
  for (int jj = 0; jj < mi; ++jj) {
    if (i < k0) N[(k0 + jj) + (size_t)i * ld] = R[(size_t)ins_s[jj] * w.cap + i];
    N[i + (size_t)(k0 + jj) * ld] = (i == k0 + jj) ? (T)1 : (T)0;
  }
}

// ---------------------------------------------------------------- fold
// In-place rank-K update C += A B on the matrix cores.  A is column-major
// (lda), B row-major (ldb), C column-major (ldc).  The MFMA computes the
// transposed tile, D = B^T A^T, so that the 16 lanes of a row group walk
// down a column of C (contiguous 128-byte reads and writes).
template <typename T>
__device__ inline void fold_tile(T* C, int ldc, const T* A, int lda, const T* B, int ldb, int M, int Nn, int K,
                                 int i0, int j0) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jb = j0 + wv * 16;
  const int li = lane & 15, lk = lane >> 4;
  typename Mfma<T>::acc_t acc[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int ii = i0 + rb * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = jb + Mfma<T>::row(lane, r);
      acc[rb][r] = (ii < M && jj < Nn) ? C[ii + (size_t)jj * ldc] : (T)0;
    }
  }
  for (int s = 0; s < K; s += 4) {
    const int sk = s + lk;
    const T a = (sk < K && jb + li < Nn) ? B[(size_t)sk * ldb + jb + li] : (T)0;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int ii = i0 + rb * 16 + li;
      const T b = (sk < K && ii < M) ? A[(size_t)sk * lda + ii] : (T)0;
      acc[rb] = Mfma<T>::run(a, b, acc[rb]);
    }
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int ii = i0 + rb * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = jb + Mfma<T>::row(lane, r);
      if (ii < M && jj < Nn) C[ii + (size_t)jj * ldc] = acc[rb][r];
    }
  }
}

// Window fold N_ext += A B for every walker of the batch and both spins
// (blockIdx.z = 2 walker + spin).
template <typename T>
__global__ void __launch_bounds__(WG) k_fold(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int sp = blockIdx.z & 1;
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int kx = c->kx, m = c->m;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (m == 0 || i0 >= kx || j0 >= kx) return;
  fold_tile<T>(w.N[sp], w.ld, w.A[sp], w.cap, w.B[sp], w.cap, kx, kx, m, i0, j0);
}

// ----------------------------------------------------------- compaction
// Drop the rows and columns of removed vertices: with remap and moves from
// the accept kernel, N[i][d] = N[remap(i)][s] and N[d][i] = N[s][remap(i)]
// for every move (d, s).  Sources lie at or above the new order and are
// never written, so the copy is race-free in place.
template <typename T>
__global__ void __launch_bounds__(WG) k_compact_move(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const int* remap = w.remap;
  const int* moves = w.moves;
  Ctl* c = w.ctl;
  if (!c->active) return;
  const int h = blockIdx.y, sp = blockIdx.z & 1;
  const int nh = moves[2 * KS_MAX];
  const int knew = c->knew;
  const int i = blockIdx.x * WG + threadIdx.x;
  if (h < nh && i < knew) {
    const int d = moves[2 * h], s = moves[2 * h + 1];
    T* N = w.N[sp];
    const size_t ld = w.ld;
    const int si = remap[i];
    N[i + (size_t)d * ld] = N[si + (size_t)s * ld];
    N[d + (size_t)i * ld] = N[s + (size_t)si * ld];
  }
}

#define DCAX_INSTANTIATE(T)                                              \
  template __global__ void k_prep_replay<T>(const View<T>*);             \
  template __global__ void k_prep_rng<T>(const View<T>*);                \
  template __global__ void k_gather<T>(const View<T>*);                  \
  template __global__ void k_cand_x<T>(const View<T>*);                  \
  template __global__ void k_gram<T>(const View<T>*);                    \
  template __global__ void k_accept<T>(const View<T>*);                  \
  template __global__ void k_ygemm<T>(const View<T>*);                   \
  template __global__ void k_fold_prep<T>(const View<T>*);               \
  template __global__ void k_fold<T>(const View<T>*);                    \
  template __global__ void k_compact_move<T>(const View<T>*);

DCAX_INSTANTIATE(double)
DCAX_INSTANTIATE(float)

}  // namespace dcax

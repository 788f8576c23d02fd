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
// det N'^{-1} / det N^{-1} = prod_S (-Delta_p) det Gamma_S.  The kernels carry
// the column-scaled Gt = Gamma diag(-Delta), finite also where Delta = 0:
// det Gt is the ratio and N' = N + (E_S - G_{.S}) diag(-Delta) Gt^{-1} N_{S.}.
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
// and one per distinct (window-start vertex, removal or flip) target; a
// removal of a vertex inserted earlier in the same window refers to that
// candidate, a second flip of a vertex to its flip element.  A proposal that
// would change a spin the window has already changed otherwise (a flip of a
// spin inserted in the window, a removal of a flipped spin) ends the window
// before it, so that it opens the next one: the forced decisions make these
// cases known here.
template <typename T>
__global__ void __launch_bounds__(WG) k_prep_replay(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  Ctl* c = w.ctl;
  __shared__ long long tid_s[KS_MAX];
  __shared__ int tslot_s[KS_MAX];
  __shared__ int on_s[KS_MAX];      // element changed by the window so far (odd count)
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
  int nP = nP_s;
  const int k0 = k0_s;
  if (nP == 0) return;
  const long long pos = c->pos;
  if (t < nP) {
    const dcax_proposal& r = w.replay[pos + t];
    tid_s[t] = (r.kind >= 1) ? r.id : -2;
    tslot_s[t] = -1;
  }
  if (t < KS_MAX) on_s[t] = 0;
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
    p.ub0 = 0.0;
    p.ui0 = 0.0;
    p.ridx = pos + j;
    p.gidx = pos + j;
    p.el = -1;
    if (r.kind == 0) {
      int e = nE++, cc = nC++;
      w.el_site[e] = r.site;
      w.el_tau[e] = r.tau;
      w.el_s[e] = r.aux_spin;
      w.el_slot[e] = -1;
      w.el_flip[e] = 0;
      w.el_cand[e] = cc;
      w.cand_el[cc] = e;
      w.cand_id[cc] = r.accepted ? r.id : -1;
      if (r.accepted && r.id >= next_id) next_id = r.id + 1;
      p.el = e;
    } else if (r.id >= 0) {
      const int fl = r.kind == 2 ? 1 : 0;
      int e = -1;
      for (int cc = 0; cc < nC; ++cc)
        if (w.cand_id[cc] == r.id) e = w.cand_el[cc];
      if (e >= 0 && fl) {
        nP = j;           // a flip of a spin inserted in this window
        break;
      }
      if (e < 0) {
        int slot = tslot_s[j];
        if (slot < 0) {
          latch(c, ST_TRACE);
          c->active = 0;
          return;
        }
        int twin = -1;
        for (int x = 0; x < nE; ++x) {
          if (w.el_slot[x] == slot && w.el_flip[x] == fl) e = x;
          if (w.el_slot[x] == slot && w.el_flip[x] != fl) twin = x;
        }
        if (twin >= 0 && on_s[twin]) {
          if (fl) {       // a flip of a vertex the window removed
            latch(c, ST_TRACE);
            c->active = 0;
            return;
          }
          nP = j;         // a removal of a spin flipped in this window
          break;
        }
        if (e < 0) {
          e = nE++;
          w.el_site[e] = w.v_site[slot];
          w.el_tau[e] = w.v_tau[slot];
          w.el_s[e] = w.v_s[slot];
          w.el_slot[e] = slot;
          w.el_flip[e] = fl;
          w.el_cand[e] = -1;
        }
      }
      p.el = e;
    }
    if (p.el >= 0 && r.accepted) on_s[p.el] ^= 1;
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
// an aborted window keeps the target it had already chosen.  One wavefront,
// one lane per proposal; elements are numbered in proposal order (a removal
// whose target an earlier removal of the window already holds shares its
// element) by prefix counts over lane masks.
constexpr int PW = 64;      // prep kernel: one wavefront per walker
static_assert(KS_MAX <= PW, "one lane per proposal");

template <typename T>
__global__ void __launch_bounds__(PW) k_prep_rng(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const uint64_t seed = w.seed;
  Ctl* c = w.ctl;
  const int lane = threadIdx.x;
  const long long left = c->end - c->pos;
  const int nP = uni((c->status == 0 && left > 0) ? (int)(left < w.ks ? left : w.ks) : 0);
  if (nP == 0) {
    if (lane == 0) c->active = 0;
    return;
  }
  const int k0 = uni(c->k);
  const long long pos = uni(c->pos);
  const long long carry = uni(c->carry_id);
  const int carry_kind = uni(c->carry_kind) == 2 ? 2 : 1;
  int carry_slot = -1;
  if (carry >= 0) {
    int found = -1;
    for (int i = lane; i < k0; i += PW)
      if (w.v_id[i] == carry) found = i;
    const unsigned long long hit = __ballot(found >= 0);
    if (hit) carry_slot = __shfl(found, (int)__ffsll((long long)hit) - 1, PW);
    if (carry_slot < 0) {
      if (lane == 0) {
        latch(c, ST_TRACE);
        c->active = 0;
      }
      return;
    }
  }
  const bool act = lane < nP;
  // insertions and removals share 1 - flip_share equally, flips the rest
  const double half = 0.5 * (1.0 - w.flip_share);
  double u_kind = 1.0, u_site = 0.0, u_tau = 0.0, u_spin = 0.0, u_acc = 0.0, u_dummy;
  double ub0 = 0.0, ui0 = 0.0;
  int kind = -1, slot = -1;
  if (act) {
    const long long g = pos + lane;
    uniforms2(seed, g, 0u, u_kind, u_site);
    uniforms2(seed, g, 1u, u_tau, u_spin);
    uniforms2(seed, g, 2u, u_acc, u_dummy);
    if (lane == 0 && carry >= 0) {
      kind = carry_kind;
      slot = carry_slot;
    } else if (u_kind < half) {
      kind = 0;
    } else {
      kind = (u_kind < 2.0 * half) ? 1 : 2;
      uniforms2(seed, g, 3u, ub0, ui0);
      if (k0 > 0) {     // the first attempt's window-start vertex
        slot = (int)(ui0 * (double)k0);
        if (slot >= k0) slot = k0 - 1;
      }
    }
  }
  // A target's element belongs to a (slot, kind) pair: a removal and a flip
  // of one vertex change it differently and need their own columns.  Keys
  // 2 slot + (flip).  A target's second attempt is prepared too (as long as
  // elements remain), so that a redraw after hitting an already removed
  // vertex rarely has to close the window.  Its slot does not depend on the
  // state; whether the attempt happens does, and an unused element costs
  // nothing.
  const int fl = (kind == 2) ? 1 : 0;
  const int key_r = (kind >= 1 && slot >= 0) ? 2 * slot + fl : -1;
  int key1 = -1;
  if (kind >= 1 && !(lane == 0 && carry >= 0) && k0 > 0) {
    double ub1, ui1;
    uniforms2(seed, pos + lane, 4u, ub1, ui1);
    int slot1 = (int)(ui1 * (double)k0);
    if (slot1 >= k0) slot1 = k0 - 1;
    key1 = 2 * slot1 + fl;
  }
  // duplicates, by register broadcasts: the first proposal aiming at a key
  // owns its element; a second attempt is fresh unless some first attempt or
  // an earlier second attempt already prepares its key
  int first = lane;
  bool fresh1 = key1 >= 0;
  for (int x = 0; x < nP; ++x) {
    const int sx = __builtin_amdgcn_readlane(key_r, x), s1x = __builtin_amdgcn_readlane(key1, x);
    if (x < first && sx >= 0 && sx == key_r) first = x;
    fresh1 &= sx != key1;
    fresh1 &= !(x < lane && s1x == key1);
  }
  const bool fresh = (kind == 0) || (key_r >= 0 && first == lane);
  const unsigned long long fresh_m = __ballot(fresh), ins_m = __ballot(kind == 0);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int e_own = fresh ? __popcll(fresh_m & below) : -1;
  const int cc = (kind == 0) ? __popcll(ins_m & below) : -1;
  const int e_first = __shfl(e_own, first, PW);
  const int e = (key_r >= 0 && !fresh) ? e_first : e_own;
  const int nE0 = __popcll(fresh_m);
  const unsigned long long fresh1_m = __ballot(fresh1);
  const int e1 = nE0 + __popcll(fresh1_m & below);
  const int nE = min(nE0 + __popcll(fresh1_m), KS_MAX);
  if (kind == 0) {
    int site = (int)(u_site * (double)w.Nc);
    if (site >= w.Nc) site = w.Nc - 1;
    w.el_site[e] = site;
    w.el_tau[e] = u_tau * w.beta;
    w.el_s[e] = (u_spin < 0.5) ? 1 : -1;
    w.el_slot[e] = -1;
    w.el_flip[e] = 0;
    w.el_cand[e] = cc;
    w.cand_el[cc] = e;
    w.cand_id[cc] = -1;
  } else if (fresh) {
    w.el_site[e] = w.v_site[slot];
    w.el_tau[e] = w.v_tau[slot];
    w.el_s[e] = w.v_s[slot];
    w.el_slot[e] = slot;
    w.el_flip[e] = fl;
    w.el_cand[e] = -1;
  }
  if (fresh1 && e1 < KS_MAX) {
    const int slot1 = key1 >> 1;
    w.el_site[e1] = w.v_site[slot1];
    w.el_tau[e1] = w.v_tau[slot1];
    w.el_s[e1] = w.v_s[slot1];
    w.el_slot[e1] = slot1;
    w.el_flip[e1] = key1 & 1;
    w.el_cand[e1] = -1;
  }
  if (act) {
    WinProp p;
    p.kind = kind;
    p.el = e;
    p.forced = -1;
    p.carried = (lane == 0 && carry >= 0) ? 1 : 0;
    p.u = u_acc;
    p.ub0 = ub0;
    p.ui0 = ui0;
    p.ridx = -1;
    p.gidx = pos + lane;
    w.wp[lane] = p;
  }
  if (lane == 0) {
    c->carry_id = -1;
    c->nP = nP;
    c->nE = nE;
    c->nC = __popcll(ins_m);
    c->k0 = k0;
    c->active = 1;
  }
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
  const int nE = c->nE, k0 = c->k0;
  // elements over blockIdx.y, rows over blockIdx.x (both grid-strided)
  for (int e = blockIdx.y; e < nE; e += gridDim.y) {
    const int cc = w.el_cand[e];
    if (cc >= 0) {
      const int rc = w.el_site[e];
      const double tc = w.el_tau[e];
      for (int i = blockIdx.x * WG + threadIdx.x; i < k0; i += gridDim.x * WG) {
        const int ri = w.v_site[i];
        const double ti = w.v_tau[i];
        const int si = s01(w.v_s[i]);
        const size_t o = (size_t)cc * w.cap + i;
        const double gic = gfun(w, 0, ri, ti, rc, tc);
        const double gci = gfun(w, 0, rc, tc, ri, ti);
        w.gcol[0][o] = (T)gic;
        w.W[0][o] = (T)(gci * (w.ev[0][si] - 1.0));
        if (w.spin_tables == 2) {
          w.gcol[1][o] = (T)gfun(w, 1, ri, ti, rc, tc);
          w.W[1][o] = (T)(gfun(w, 1, rc, tc, ri, ti) * (w.ev[1][si] - 1.0));
        } else {
          w.W[1][o] = (T)(gci * (w.ev[1][si] - 1.0));
        }
      }
      if (blockIdx.x == 0 && (int)threadIdx.x < c->nC) {
        const int e2 = w.cand_el[threadIdx.x];
        for (int sp = 0; sp < w.spin_tables; ++sp)
          w.gCC[sp][cc * KS_MAX + threadIdx.x] = gfun(w, sp, rc, tc, w.el_site[e2], w.el_tau[e2]);
      }
    } else {
      const int p = w.el_slot[e];
      for (int i = blockIdx.x * WG + threadIdx.x; i < k0; i += gridDim.x * WG) {
        const size_t o = (size_t)e * w.cap + i;
        R0[o] = w.N[0][p + (size_t)i * w.ld];
        R1[o] = w.N[1][p + (size_t)i * w.ld];
      }
    }
  }
}

// Four consecutive elements of a global array (16-byte aligned) in one or
// two vector loads.
template <typename T> struct Load4;
template <> struct Load4<double> {
  __device__ static inline void run(const __attribute__((address_space(1))) double* p, double (&v)[4]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const auto q = (const __attribute__((address_space(1))) d2*)p;
    const d2 a = q[0], b = q[1];
    v[0] = a[0];
    v[1] = a[1];
    v[2] = b[0];
    v[3] = b[1];
  }
};
template <> struct Load4<float> {
  __device__ static inline void run(const __attribute__((address_space(1))) float* p, float (&v)[4]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 a = *(const __attribute__((address_space(1))) f4*)p;
    v[0] = a[0];
    v[1] = a[1];
    v[2] = a[2];
    v[3] = a[3];
  }
};

// Four consecutive elements p[i0 .. i0+3] (i0 a multiple of 4, the row
// 16-byte aligned) by one vector load, those at or past n zeroed by selects
// unless the caller knows them all valid (full).  The load is made whatever
// `full` says (every caller's rows are allocated at least 16 elements past
// the order), so no branch separates the loads of a step: they issue
// together and are waited for once.
template <typename T, typename P>
__device__ inline void load4_row(P p, int i0, int n, bool full, T (&v)[4]) {
  Load4<T>::run(p + i0, v);
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = (full || i0 + s < n) ? v[s] : (T)0;
}

// The candidate GEMMs and the Gram kernel split the inner dimension (the
// order k) over the NW wavefronts of a workgroup: 16 (8 for the Y product,
// whose registers need it) when a launch has few workgroups (a single
// walker: short chains of dependent loads per wavefront, many loads in
// flight), 4 for large batches (enough workgroups already; fewer idle
// wavefronts on small walkers).

// ------------------------------------------------------- candidate rows
// X_c = W_c N for all candidates and both spins (an nC x k0 x k0 product on
// the matrix cores), written as rows e = element(c) of R.  A workgroup owns
// 16 columns of X; its wavefronts split the inner dimension and their
// partial tiles are summed in LDS in a fixed order, so the result does not
// depend on scheduling.  Small tiles and the split keep the dependent chain
// of loads short: at the orders of a single walker this product is bound by
// load latency, not by bandwidth.
template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) k_cand_x(const View<T>* __restrict__ vs) {
  constexpr int GWV = NW;
  typedef typename Mfma<T>::acc_t acc_t;
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  // sizes read as wavefront-uniform values, so that the loops below branch
  // on scalars and their loads can be issued together
  const int nC = uni(c->nC);
  const int k0 = uni(c->k0);
  if (nC == 0) return;
  const int sp = blockIdx.y;
  const auto N = gp(w.N[sp]);
  const auto Wm = gp(w.W[sp]);
  const auto R = gp(w.R[sp]);
  const auto cand_el = gp(w.cand_el);
  const size_t ld = uni((long long)w.ld), cap = uni((long long)w.cap);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nRB = (nC + 15) >> 4;
  __shared__ acc_t red[GWV][4][64];
  // column tiles of 16, grid-strided over blockIdx.x
  for (int j0 = blockIdx.x * 16; j0 < k0; j0 += gridDim.x * 16) {
    const int jc = j0 + li;
    acc_t acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = acc_t{0, 0, 0, 0};
    // The inner dimension in blocks of 16 rows of N, dealt to the
    // wavefronts in turn.  Step s of a block pairs row i0 + 4 lk + s with
    // k-slot lk, so that each lane reads four consecutive rows of its column
    // of N and of its row of W (vector loads; the 16 rows of a column are
    // one 128-byte line); columns and candidates beyond the sizes are read
    // from valid ones and zeroed.
    const int jcc = jc < k0 ? jc : 0;
    const T jmask = (T)(jc < k0 ? 1 : 0);
    if constexpr (NW < 8) {
      // batches: two steps per pass, lighter on registers (occupancy matters
      // more than vector loads when many workgroups share a compute unit)
      for (int i0 = 4 * wv; i0 < k0; i0 += 8 * GWV) {
        T bv[2], av[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int ik = i0 + 4 * GWV * u + lk;
          const bool kin = ik < k0;
          const int ikc = kin ? ik : 0;
          bv[u] = N[ikc + (size_t)jcc * ld] * (T)(kin ? 1 : 0) * jmask;
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            const int cr = rb * 16 + li;
            av[u][rb] = Wm[(size_t)(cr < nC ? cr : 0) * cap + ikc] * (T)((kin && cr < nC) ? 1 : 0);
          }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            if (rb < nRB) acc[rb] = Mfma<T>::run(av[u][rb], bv[u], acc[rb]);
      }
    } else
    for (int i0 = 16 * uni(wv); i0 < k0; i0 += 16 * GWV) {
      const int ib = i0 + 4 * lk;
      const bool full = i0 + 16 <= k0;      // the same in every lane
      // every load of the step first (rows ib .. ib + 3 < k0 + 16 lie in
      // the allocations; candidates past nC read row 0), then the masks, so
      // that the loads issue together
      T bv[4], av[4][4];
      Load4<T>::run(N + (size_t)jcc * ld + ib, bv);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int cr = rb * 16 + li;
        Load4<T>::run(Wm + (size_t)(cr < nC ? cr : 0) * cap + ib, av[rb]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool row = full || ib + u < k0;
        bv[u] = (row && jc < k0) ? bv[u] : (T)0;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) av[rb][u] = (row && rb * 16 + li < nC) ? av[rb][u] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          if (rb < nRB) acc[rb] = Mfma<T>::run(av[rb][u], bv[u], acc[rb]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) red[wv][rb][lane] = acc[rb];
    __syncthreads();
    const int rb = wv;
    if (rb < nRB) {
      acc_t sum = red[0][rb][lane];
      for (int v = 1; v < GWV; ++v) sum += red[v][rb][lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cr = rb * 16 + Mfma<T>::row(lane, r);
        if (cr < nC && jc < k0) R[(size_t)cand_el[cr] * cap + jc] = sum[r];
      }
    }
    __syncthreads();      // red is rewritten by the next tile
  }
}

// Candidate rows for launches with many workgroups (batches of walkers): a
// workgroup owns 64 columns of X and runs over the whole inner dimension in
// chunks of 32 rows of N, staged in LDS by coalesced loads (each column's
// chunk is one or two 128-byte lines), with W_C's chunk beside it: W_C is
// then read once per 64 columns instead of once per 16.  The next chunk's
// loads are in flight while the current chunk's MFMA steps run.  Wavefront
// v computes the 16-column block v for every candidate block.
constexpr int XT_COLS = 64, XT_KC = 32, XT_GROUP = 8;
template <typename T> struct LdsPad { static constexpr int P = sizeof(T) == 8 ? 34 : 36; };

template <typename T>
__device__ inline void lds_read4(const T* p, T (&v)[4]) {
  if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = ((const d2*)p)[0], b = ((const d2*)p)[1];
    v[0] = a[0];
    v[1] = a[1];
    v[2] = b[0];
    v[3] = b[1];
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 a = *(const f4*)p;
    v[0] = a[0];
    v[1] = a[1];
    v[2] = a[2];
    v[3] = a[3];
  }
}

// Eight consecutive elements p[i0 .. i0+7] (i0 a multiple of 8, 16-byte
// aligned) by two vector loads, whatever lies there: the callers' rows are
// allocated at least 32 elements past the order, and they zero the elements
// past it when they store the values.  No branch separates the loads from
// their use, so a chunk's loads issue together and are waited for once.
template <typename T, typename P>
__device__ inline void load8_raw(P p, int i0, T (&v)[8]) {
  T a[4], b[4];
  Load4<T>::run(p + i0, a);
  Load4<T>::run(p + i0 + 4, b);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    v[u] = a[u];
    v[4 + u] = b[u];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_cand_xt(const View<T>* __restrict__ vs) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int P = LdsPad<T>::P;
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int nC = uni(c->nC), k0 = uni(c->k0);
  if (nC == 0) return;
  const int sp = blockIdx.y;
  const auto N = gp(w.N[sp]);
  const auto Wm = gp(w.W[sp]);
  const auto R = gp(w.R[sp]);
  const auto cand_el = gp(w.cand_el);
  const size_t ld = uni((long long)w.ld), cap = uni((long long)w.cap);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nRB = (nC + 15) >> 4;
  __shared__ __attribute__((aligned(16))) T Ns[XT_COLS * P];
  __shared__ __attribute__((aligned(16))) T Ws[KS_MAX * P];
  // loader role: column (and candidate row) t / 4, chunk rows 8 (t % 4) .. + 7
  const int lc = t >> 2, lr = (t & 3) * 8;
  const bool wrow = lc < nC;
  const auto wsrc = Wm + (size_t)(wrow ? lc : 0) * cap;
  for (int j0 = blockIdx.x * XT_COLS; j0 < k0; j0 += gridDim.x * XT_COLS) {
    const bool jin = j0 + lc < k0;
    const auto nsrc = N + (size_t)(jin ? j0 + lc : 0) * ld;
    // two-level sums: the MFMA steps of XT_GROUP chunks accumulate in acc,
    // which is then added to tot (in FP32 a single chain over an order of
    // thousands would carry k/4 roundings per entry)
    acc_t acc[4], tot[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = tot[rb] = acc_t{0, 0, 0, 0};
    T nv[8], wr[8];
    // rows i0 + lr .. + 7 < k0 + 32 lie inside N's and W_C's rows of cap
    // elements; columns past k0 read column 0 and candidates past nC row 0,
    // all zeroed when stored
    auto fetch = [&](int i0) {
      load8_raw(nsrc, i0 + lr, nv);
      load8_raw(wsrc, i0 + lr, wr);
    };
    fetch(0);
    for (int i0 = 0; i0 < k0; i0 += XT_KC) {
      __syncthreads();      // the previous chunk's LDS reads are done
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool row = i0 + lr + u < k0;
        Ns[lc * P + lr + u] = (jin && row) ? nv[u] : (T)0;
        Ws[lc * P + lr + u] = (wrow && row) ? wr[u] : (T)0;
      }
      __syncthreads();
      if (i0 + XT_KC < k0) fetch(i0 + XT_KC);
#pragma unroll
      for (int kb = 0; kb < XT_KC / 16; ++kb) {
        // step s pairs chunk row 16 kb + 4 lk + s with k-slot lk (any
        // bijection of rows onto k-slots sums the same terms)
        T b4[4];
        lds_read4(&Ns[(wv * 16 + li) * P + kb * 16 + 4 * lk], b4);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          if (rb < nRB) {
            T a4[4];
            lds_read4(&Ws[(rb * 16 + li) * P + kb * 16 + 4 * lk], a4);
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) acc[rb] = Mfma<T>::run(a4[s2], b4[s2], acc[rb]);
          }
        }
      }
      if ((i0 / XT_KC) % XT_GROUP == XT_GROUP - 1) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          tot[rb] += acc[rb];
          acc[rb] = acc_t{0, 0, 0, 0};
        }
      }
    }
    const int j = j0 + wv * 16 + li;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      if (rb < nRB) {
        tot[rb] += acc[rb];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cr = rb * 16 + Mfma<T>::row(lane, r);
          if (cr < nC && j < k0) R[(size_t)cand_el[cr] * cap + j] = tot[rb][r];
        }
      }
    }
    __syncthreads();        // LDS is rewritten by the next column tile
  }
}

// -------------------------------------------------------------- Gram
// The column-scaled Gamma of the window elements, both spins, in FP64:
//   Gt_{x,y} = -Delta_y G_{x,y} + delta_xy (1 + Delta_y),  G = N_ext g,
// finite also where Delta = 0 (U = 0).  Its columns:
//   candidate c:  G_{x,c} = R_x . g_{I,c} (+ g_{x,c} for candidate rows x),
//                 Delta_c = e^{V'_c} - 1;
//   target p:     Gt_{x,p} = R_x[p], from G (e^V - 1) = N e^V - 1 with
//                 Delta_p = e^{-V_p} - 1 (removal; a flip: target_column);
// where R_x is row x of the extended N (X_c for candidates, N_{p.} for targets).
// Gt_{x,y} for a target y at slot p of the window-start vertices, from
// r = R_x[p] = N_ext{x,p}: a removal (Delta_p = e^{-V_p} - 1) gives r itself;
// a flip of the auxiliary spin (Delta_p = e^{-2 V_p} - 1) gives
// (1 + e^{-V_p}) r - delta_xy e^{-V_p}, by the same identity
// G (e^V - 1) = N e^V - 1.
template <typename T>
__device__ inline double target_column(const View<T>& w, int sp, int y, int x, double r) {
  if (!w.el_flip[y]) return r;
  const double em = w.ev[sp][1 - s01(w.el_s[y])];       // e^{-V_p}
  return (1.0 + em) * r - (y == x ? em : 0.0);
}

// Row form of the Gram kernel for launches with few walkers: a workgroup
// owns one row x of Gt, its wavefronts take the candidate columns in turn
// (each a k0-long dot product summed across the lanes), so a single walker
// spreads over nE workgroups per spin.
template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) k_gram_rows(const View<T>* __restrict__ vs) {
  constexpr int GWV = NW, GW = NW * 64;
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int sp = blockIdx.y;
  const int nE = c->nE;
  const int k0 = c->k0, nC = c->nC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // a wavefront takes its candidate columns cc = wv, wv + NW, ... together,
  // so that each entry of the row is loaded once, with four steps of 64
  // entries per pass in flight and a partial sum per step (the last pass
  // weighs the steps beyond the order zero)
  constexpr int MAXC = (KS_MAX + GWV - 1) / GWV;
  const auto gcol = gp(w.gcol[sp]);
  const size_t cap = w.cap;
  for (int x = blockIdx.x; x < nE; x += gridDim.x) {
    const int cx = w.el_cand[x];
    const auto Rx = gp(w.R[sp] + (size_t)x * cap);
    const auto G = gp(w.gram[sp] + x * KS_MAX);
    size_t goff[MAXC];
#pragma unroll
    for (int q = 0; q < MAXC; ++q) {
      const int cc = wv + q * GWV;
      goff[q] = (size_t)(cc < nC ? cc : 0) * cap;
    }
    // columns this wavefront owns (the same count in every lane)
    const int nq = uni(nC > wv ? (nC - wv + GWV - 1) / GWV : 0);
    double acc[MAXC][4];
#pragma unroll
    for (int q = 0; q < MAXC; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[q][u] = 0.0;
    for (int i = lane; i < k0; i += 256) {
      // steps past the order read a valid entry and weigh it zero
      double a[4], g[MAXC][4];
      int ic[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int iu = i + 64 * u;
        ic[u] = iu < k0 ? iu : i;
        a[u] = (double)Rx[ic[u]] * (iu < k0 ? 1.0 : 0.0);
      }
#pragma unroll
      for (int q = 0; q < MAXC; ++q)
        if (q < nq)
#pragma unroll
          for (int u = 0; u < 4; ++u) g[q][u] = (double)gcol[goff[q] + ic[u]];
#pragma unroll
      for (int q = 0; q < MAXC; ++q)
        if (q < nq)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[q][u] += a[u] * g[q][u];
    }
#pragma unroll
    for (int q = 0; q < MAXC; ++q) {
      const int cc = wv + q * GWV;
      const double s = wave_sum((acc[q][0] + acc[q][1]) + (acc[q][2] + acc[q][3]));
      if (lane == 0 && cc < nC) {
        const int ec = w.cand_el[cc];
        const double Dc = w.ev[sp][s01(w.el_s[ec])] - 1.0;
        const double g = s + (cx >= 0 ? w.gCC[sp][cx * KS_MAX + cc] : 0.0);
        G[ec] = -Dc * g + (ec == x ? 1.0 + Dc : 0.0);
      }
    }
    for (int y = threadIdx.x; y < nE; y += GW) {
      const int py = w.el_slot[y];
      if (py >= 0) G[y] = target_column(w, sp, y, x, (double)Rx[py]);
    }
  }
}

// Matrix-core form for batches: one workgroup per 16 candidates and spin.
template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) k_gram(const View<T>* __restrict__ vs) {
  constexpr int GWV = NW, GW = NW * 64;
  typedef typename Mfma<double>::acc_t acc_t;
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int sp = blockIdx.y;
  const int nE = uni(c->nE);
  const int k0 = uni(c->k0), nC = uni(c->nC);
  const size_t cap = uni((long long)w.cap);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nRB = (nE + 15) >> 4;
  const auto R = gp(w.R[sp]);
  const auto gcol = gp(w.gcol[sp]);
  const auto G = gp(w.gram[sp]);
  __shared__ acc_t red[GWV][4][64];
  // candidate columns: R (nE x k0) times gcol^T (k0 x 16 candidates) on the
  // FP64 matrix cores, the wavefronts splitting k0 and summing in LDS in a
  // fixed order; blocks of 16 candidates grid-strided over blockIdx.x
  for (int cc0 = blockIdx.x * 16; cc0 < nC; cc0 += gridDim.x * 16) {
    const int cc = cc0 + li;
    acc_t acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = acc_t{0, 0, 0, 0};
    // blocks of 16 of the inner dimension, four consecutive per lane (as
    // in the candidate rows)
    const int ccc = cc < nC ? cc : 0;
    if constexpr (NW < 8) {
      // batches: two steps per pass (see the candidate rows)
      for (int i0 = 4 * wv; i0 < k0; i0 += 8 * GWV) {
        double bv[2], av[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int ik = i0 + 4 * GWV * u + lk;
          const bool kin = ik < k0;
          const int ikc = kin ? ik : 0;
          bv[u] = (double)gcol[(size_t)ccc * cap + ikc] * ((kin && cc < nC) ? 1.0 : 0.0);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            const int x = rb * 16 + li;
            av[u][rb] = (double)R[(size_t)(x < nE ? x : 0) * cap + ikc] * ((kin && x < nE) ? 1.0 : 0.0);
          }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            if (rb < nRB) acc[rb] = Mfma<double>::run(av[u][rb], bv[u], acc[rb]);
      }
    } else
    for (int i0 = 16 * uni(wv); i0 < k0; i0 += 16 * GWV) {
      const int ib = i0 + 4 * lk;
      const bool full = i0 + 16 <= k0;      // the same in every lane
      // every load of the step first (rows of cap elements, ib + 3 < k0 +
      // 16), then the masks, so that the loads issue together
      T bt[4], at[4][4];
      Load4<T>::run(gcol + (size_t)ccc * cap + ib, bt);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int x = rb * 16 + li;
        Load4<T>::run(R + (size_t)(x < nE ? x : 0) * cap + ib, at[rb]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool row = full || ib + u < k0;
        const double b = (row && cc < nC) ? (double)bt[u] : 0.0;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          if (rb < nRB) acc[rb] = Mfma<double>::run((row && rb * 16 + li < nE) ? (double)at[rb][u] : 0.0, b, acc[rb]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) red[wv][rb][lane] = acc[rb];
    __syncthreads();
    const int rb = wv;
    if (rb < nRB && cc < nC) {
      acc_t sum = red[0][rb][lane];
      for (int v = 1; v < GWV; ++v) sum += red[v][rb][lane];
      const int ec = w.cand_el[cc];
      const double Dc = w.ev[sp][s01(w.el_s[ec])] - 1.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = rb * 16 + Mfma<double>::row(lane, r);
        if (x < nE) {
          const int cx = w.el_cand[x];
          const double g = sum[r] + (cx >= 0 ? w.gCC[sp][cx * KS_MAX + cc] : 0.0);
          G[x * KS_MAX + ec] = -Dc * g + (ec == x ? 1.0 + Dc : 0.0);
        }
      }
    }
    __syncthreads();      // red is rewritten by the next block
  }
  // columns of window-start vertices (removal or flip targets)
  if (blockIdx.x == 0)
    for (int idx = threadIdx.x; idx < nE * nE; idx += GW) {
      const int x = idx / nE, y = idx % nE;
      const int py = w.el_slot[y];
      if (py >= 0) G[x * KS_MAX + y] = target_column(w, sp, y, x, (double)R[(size_t)x * w.cap + py]);
    }
}

// ---------------------------------------------------------- accept loop
// The sequential Metropolis decisions of the window, in FP64, in one
// workgroup per walker.  Gt is the column-scaled Gamma of k_gram,
// Gt_S = Gamma_S diag(-Delta_S): adding q to S multiplies the determinant
// ratio by the Schur complement
//   Gt_qq - Gt_qS Gt_S^{-1} Gt_Sq,
// taking an inserted spin out again (its removal later in the same window)
// multiplies it by (Gt_S^{-1})_qq.  The acceptance ratio is K/(k+1) or k/K
// times the product over both spins (Sec. 2.3 weights).
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
constexpr int AWV = 4;            // accept kernel: wavefronts per walker
constexpr int AW = 64 * AWV;
static_assert(KS_MAX == 64, "the accept kernel maps one lane to one window element");

// Sweep tableau, one per spin, started at the window's scaled Gram matrix Gt.
// A Gauss-Jordan sweep on element q (pivot d = T_qq) maps T to
//   T_qq -> -1/d,  T_qc -> T_qc/d,  T_rq -> T_rq/d,  T_rc -> T_rc - T_rq T_qc/d,
// and the reverse sweep, which undoes it, flips the signs of row and column
// q.  After sweeping the set S, T_SS = -Gt_S^{-1} and every other diagonal
// entry T_qq is the Schur complement Gt_qq - Gt_qS Gt_S^{-1} Gt_Sq.  So
// flipping q has ratio T_qq, unflipping q in S has ratio (Gt_S^{-1})_qq =
// -T_qq, and accepting either is one (reverse) sweep: a rank-1 update with
// no reductions.
//
// The proposal loop runs in all four wavefronts of the workgroup with the
// same uniform control flow; each keeps the window state in registers (lane
// e: element e's position in S, slot, candidate index and diagonal entries;
// lane j: proposal j; lane a: the element at position a of S; lane i: the
// i-th spin inserted in this window), so a rejected proposal costs register
// reads only.  An accepted one is swept with lane c owning column c and the
// rows dealt to the wavefronts in chunks of CH, between two barriers.
template <typename T>
__global__ void __launch_bounds__(AW) k_accept(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  auto el_row = gp(w.el_row);
  auto remap = gp(w.remap);
  auto moves = gp(w.moves);
  const uint64_t seed = w.seed;
  Ctl* c = w.ctl;
  if (!c->active) return;
  // rows padded to LS doubles so that the lanes of a row hit distinct banks
  constexpr int LS = KS_MAX + 1;
  constexpr int CH = 4;
  __shared__ double T_s[2][KS_MAX * LS];
  __shared__ long long cid_s[KS_MAX];
  __shared__ double rout_s[KS_MAX];
  const int t = threadIdx.x, lane = t & 63, wv = uni(t >> 6);
  const bool t0 = t == 0, w0 = wv == 0;
  const int nE = uni(c->nE), nP = uni(c->nP), k0 = uni(c->k0), nC = uni(c->nC);
  const double K_exp = uni(w.K_exp);
  const int max_order = uni(w.max_order);
  {
    // Gram rows x < nE of both spins; wavefront wv loads rows 16 wv .. 16 wv + 15
    const auto gram0 = gp(w.gram[0]), gram1 = gp(w.gram[1]);
    double g0[16], g1[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = wv * 16 + u;
      const bool in = x < nE && lane < nE;
      g0[u] = in ? gram0[x * KS_MAX + lane] : 0.0;
      g1[u] = in ? gram1[x * KS_MAX + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = wv * 16 + u;
      if (x < nE) {
        T_s[0][x * LS + lane] = g0[u];
        T_s[1][x * LS + lane] = g1[u];
      }
    }
  }
  // per-lane window state (identical in every wavefront)
  int p_kind = 0, p_el = -1, p_forced = -1, p_carried = 0;
  double p_u = 0.0, p_ub0 = 0.0, p_ui0 = 0.0;
  long long p_ridx = -1, p_gidx = 0;
  if (lane < nP) {
    const WinProp& x = w.wp[lane];
    p_kind = x.kind;
    p_el = x.el;
    p_forced = x.forced;
    p_carried = x.carried;
    p_u = x.u;
    p_ub0 = x.ub0;
    p_ui0 = x.ui0;
    p_ridx = x.ridx;
    p_gidx = x.gidx;
  }
  // e_twin: the element of the same window-start vertex with the other kind
  // of change (removal / flip) is in S, i.e. that vertex was changed the
  // other way in this window
  int e_cand = -1, e_spin = 0, e_slot = -1, e_flip = 0, e_twin = 0;
  if (lane < nE) {
    e_cand = gp(w.el_cand)[lane];
    e_spin = gp(w.el_s)[lane];
    e_slot = gp(w.el_slot)[lane];
    e_flip = gp(w.el_flip)[lane];
  }
  if (t < nC) cid_s[t] = gp(w.cand_id)[t];
  int pos_r = -1, sa = 0, insl = 0;
  __syncthreads();
  double dg0 = T_s[0][lane * LS + lane], dg1 = T_s[1][lane * LS + lane];
  int m = 0, kcur = k0, nins = 0, bad = 0, n_done = nP;
  double sign = uni(c->sign);
  long long next_id = uni(c->next_id), carry = -1;
  int carry_kind = 1;
  long long n_ins = 0, n_rem = 0, n_mis = 0, n_flip = 0, n_neg = 0;
  const int neglect = uni(w.neglect);
  // Proposals are settled in runs: every lane from the current proposal on
  // evaluates its own proposal against the current state (valid up to the
  // first accepted one, which is what changes the state); the run's
  // rejections are recorded at once and the first acceptance is applied.
  // Proposals whose evaluation needs more than the lane has (a redrawn or
  // unprepared removal target, a non-finite ratio, the order limit) end the
  // run too and go through the wavefront-uniform path.
  int j = 0;
  while (j < nP) {
    const double facI = K_exp / (double)(kcur + 1), facR = (double)kcur / K_exp;
    const bool inr = lane >= j && lane < nP;
    const bool genrem = p_forced < 0 && p_kind == 1 && !p_carried;
    const bool genflip = p_forced < 0 && p_kind == 2 && !p_carried;
    int q_l = p_el, idx_l = 0;
    bool cx = false, use_insl = false;
    if (genflip && kcur <= 0) q_l = -1;   // flip at order 0: a no-op
    if (genrem) {
      if (kcur <= 0) {
        q_l = -1;                       // removal at order 0: a no-op
      } else if (p_ub0 * (double)(k0 + nins) < (double)k0) {
        if (p_el < 0) cx = true;        // the first target was not prepared
      } else {
        int idx = (int)(p_ui0 * (double)nins);
        if (idx >= nins) idx = nins - 1;
        idx_l = idx < 0 ? 0 : idx;
        use_insl = true;
      }
    }
    const int q_ins = __shfl(insl, idx_l, 64);
    if (use_insl) q_l = q_ins;
    const int qs = q_l < 0 ? 0 : q_l;
    const int pq_l = __shfl(pos_r, qs, 64);
    const double d0_l = __hiloint2double(__shfl(__double2hiint(dg0), qs, 64), __shfl(__double2loint(dg0), qs, 64));
    const double d1_l = __hiloint2double(__shfl(__double2hiint(dg1), qs, 64), __shfl(__double2loint(dg1), qs, 64));
    if (genrem && kcur > 0 && !use_insl && p_el >= 0 && pq_l >= 0) cx = true;   // redraw needed
    // a removal of a vertex flipped in this window, and every generator flip
    // (its target search checks both kinds of change), take the uniform path
    // (the shuffle runs in every lane: a lane that skipped it would not serve
    // its value to the others)
    const int tw_l = __shfl(e_twin, qs, 64);
    if (genrem && kcur > 0 && !use_insl && p_el >= 0 && tw_l) cx = true;
    if (genflip && kcur > 0) cx = true;
    const double sgn_l = (pq_l >= 0) ? -1.0 : 1.0;
    const double R_l = ((p_kind == 0) ? facI : (p_kind == 1) ? facR : 1.0) * (sgn_l * d0_l) * (sgn_l * d1_l);
    const int mine_l = p_u < fabs(R_l);
    const int dec_l = (q_l < 0) ? 0 : ((p_forced >= 0) ? p_forced : mine_l);
    if (q_l >= 0 && (!isfinite(R_l) || (dec_l && p_kind == 0 && kcur + 1 > max_order))) cx = true;
    const unsigned long long evm = __ballot(inr && (cx || dec_l));
    const int E = evm ? (int)__ffsll((long long)evm) - 1 : nP;
    // the rejections before the event
    const bool rej = lane >= j && lane < E;
    if (w0 && rej) rout_s[lane] = (q_l < 0) ? 0.0 : R_l;
    n_mis += __popcll(__ballot(rej && q_l >= 0 && p_forced >= 0 && mine_l != p_forced));
    if (E >= nP) break;
    j = E;
    int q, pq, kind, forced, dec;
    double R, d0, d1, sgn;
    if (!lane_value((int)cx, j)) {
      // a plain acceptance: everything the run computed for it holds
      q = lane_value(q_l, j);
      pq = lane_value(pq_l, j);
      kind = lane_value(p_kind, j);
      forced = lane_value(p_forced, j);
      d0 = lane_value(d0_l, j);
      d1 = lane_value(d1_l, j);
      R = lane_value(R_l, j);
      sgn = (pq >= 0) ? -1.0 : 1.0;
      if (forced >= 0 && lane_value(mine_l, j) != forced) ++n_mis;
      if (t0) rout_s[j] = R;
      dec = 1;
    } else {
    kind = lane_value(p_kind, j);
    const int el = lane_value(p_el, j);
    forced = lane_value(p_forced, j);
    const int carried = lane_value(p_carried, j);
    q = el;
    int ab = 0;
    if (forced < 0 && (kind == 1 || kind == 2) && !carried) {
      // the target, uniform among the current vertices (R6); a flip's and a
      // removal's targets alike, each with the element of its own kind
      const int fl = kind == 2 ? 1 : 0;
      int conflict = 0;
      q = -1;
      if (kcur > 0) {
        const long long gidx = lane_value(p_gidx, j);
        for (int a = 0; a < MAX_ATTEMPTS; ++a) {
          double ub = lane_value(p_ub0, j), ui = lane_value(p_ui0, j);
          if (a > 0) {
            uniforms2(seed, gidx, 3u + (uint32_t)a, ub, ui);
            ub = uni(ub);
            ui = uni(ui);
          }
          if (ub * (double)(k0 + nins) < (double)k0) {
            int slot = (int)(ui * (double)k0);
            if (slot >= k0) slot = k0 - 1;
            int e = el;
            if (a > 0) {
              const unsigned long long hit = __ballot(lane < nE && e_cand < 0 && e_slot == slot && e_flip == fl);
              e = hit ? (int)__ffsll((long long)hit) - 1 : -1;
            }
            const bool tgt = lane < nE && e_cand < 0 && e_slot == slot && pos_r >= 0;
            if (__ballot(tgt && !e_flip)) continue;     // removed in this window: redraw
            if (!fl && __ballot(tgt && e_flip)) {      // a removal of a spin flipped in this window
              conflict = 1;
              carry = uni(gp(w.v_id)[slot]);
              break;
            }
            if (e < 0) {
              ab = 1;
              carry = uni(gp(w.v_id)[slot]);
              carry_kind = kind;
              break;
            }
            q = e;
            break;
          }
          int idx = (int)(ui * (double)nins);
          if (idx >= nins) idx = nins - 1;
          q = lane_value(insl, idx);
          if (fl) {                                     // a flip of a spin inserted in this window
            conflict = 1;
            carry = uni(cid_s[lane_value(e_cand, q)]);
            q = -1;
          }
          break;
        }
        if (q < 0 && !ab && !conflict) bad = 1;
      }
      if (conflict) {
        // the spin is touched twice in this window: close the window before
        // this proposal (exact), or reject it (neglect mode)
        if (neglect) {
          ++n_neg;
          carry = -1;
        } else {
          ab = 1;
          carry_kind = kind;
        }
      }
    }
    if (ab) {
      n_done = j;
      break;
    }
    if (q < 0) {
      if (t0) rout_s[j] = 0.0;
      ++j;
      continue;
    }
    pq = lane_value(pos_r, q);
    sgn = (pq >= 0) ? -1.0 : 1.0;
    d0 = lane_value(dg0, q);
    d1 = lane_value(dg1, q);
    const double fac = (kind == 0) ? facI : (kind == 1) ? facR : 1.0;
    R = fac * (sgn * d0) * (sgn * d1);
    if (!isfinite(R)) {
      bad = 1;
      dec = 0;
    } else {
      const int mine = lane_value(p_u, j) < fabs(R);
      dec = (forced >= 0) ? forced : mine;
      if (forced >= 0 && mine != forced) ++n_mis;
    }
    if (t0) rout_s[j] = R;
    if (dec && kind == 0 && kcur + 1 > max_order) {
      if (t0) latch(c, ST_CAPACITY);
      dec = 0;
    }
    }
    ++j;
    if (!dec) continue;
    kcur += (kind == 0) ? 1 : (kind == 1) ? -1 : 0;
    if (R < 0.0) sign = -sign;
    if (kind == 2) {
      ++n_flip;           // a flip, or the unflip of a spin flipped in this window
    } else if (kind == 0) {
      ++n_ins;
      if (forced < 0) {
        const int cq = lane_value(e_cand, q);
        if (t0) cid_s[cq] = next_id;
        ++next_id;
      }
      if (lane == nins) insl = q;
      ++nins;
    } else {
      ++n_rem;
      if (pq >= 0) {
        // an unflipped insertion leaves the list of inserted spins
        const unsigned long long at = __ballot(lane < nins && insl == q);
        const int x = (int)__ffsll((long long)at) - 1;
        const int next = __shfl(insl, lane + 1, 64);
        if (lane >= x) insl = next;
        --nins;
      }
    }
    {
      const double inv0 = 1.0 / d0, inv1 = 1.0 / d1;
      const bool isq = lane == q;
      const double tq0 = T_s[0][q * LS + lane], tq1 = T_s[1][q * LS + lane];
      // new row q; lane q's own column becomes sgn T_rq / d, which the update
      // below produces with a zero weight on the old value
      const double rq0 = isq ? -inv0 : sgn * (tq0 * inv0), rq1 = isq ? -inv1 : sgn * (tq1 * inv1);
      const double f0 = isq ? -sgn * inv0 : tq0 * inv0, f1 = isq ? -sgn * inv1 : tq1 * inv1;
      const double a_l = isq ? 0.0 : 1.0;
      __syncthreads();      // row q has been read everywhere
      for (int r0_ = wv * CH; r0_ < nE; r0_ += AWV * CH) {
        double pc0[CH], pc1[CH], v0[CH], v1[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int r = r0_ + u;
          pc0[u] = T_s[0][r * LS + q];
          pc1[u] = T_s[1][r * LS + q];
          v0[u] = T_s[0][r * LS + lane];
          v1[u] = T_s[1][r * LS + lane];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int r = r0_ + u;
          T_s[0][r * LS + lane] = fma(-pc0[u], f0, a_l * v0[u]);
          T_s[1][r * LS + lane] = fma(-pc1[u], f1, a_l * v1[u]);
        }
      }
      if ((q / CH) % AWV == wv) {
        // this wavefront swept row q above; its final values
        T_s[0][q * LS + lane] = rq0;
        T_s[1][q * LS + lane] = rq1;
      }
    }
    if (pq < 0) {
      // q joins S at position m
      if (lane == q) pos_r = m;
      if (lane == m) sa = q;
      ++m;
    } else {
      // the last position of S moves into the hole
      const int js = pq, last = m - 1;
      const int el_last = lane_value(sa, last);
      if (lane == el_last) pos_r = js;
      if (lane == q) pos_r = -1;
      if (lane == js) sa = el_last;
      m = last;
    }
    {
      // the other-kind element of q's vertex learns whether q is in S
      const int qslot = lane_value(e_slot, q), qcand = lane_value(e_cand, q), qflip = lane_value(e_flip, q);
      const int qin = pq < 0 ? 1 : 0;
      if (qcand < 0 && lane < nE && e_cand < 0 && e_slot == qslot && e_flip != qflip) e_twin = qin;
    }
    __syncthreads();
    dg0 = T_s[0][lane * LS + lane];
    dg1 = T_s[1][lane * LS + lane];
  }
  {
    // Gt_S^{-1} in the order of S: -T over the rows and columns of S
    const auto gi0 = gp(w.ginv[0]), gi1 = gp(w.ginv[1]);
    for (int a = wv; a < m; a += AWV) {
      const int ea = lane_value(sa, a);
      if (lane < m) {
        gi0[a * KS_MAX + lane] = -T_s[0][ea * LS + sa];
        gi1[a * KS_MAX + lane] = -T_s[1][ea * LS + sa];
      }
    }
  }
  __syncthreads();
  if (w0) {
    if (lane < n_done && p_ridx >= 0) gp(w.ratio_out)[p_ridx] = rout_s[lane];
    if (lane < nC) gp(w.cand_id)[lane] = cid_s[lane];
  }
  // Epilogue: the fold's column order, the new vertex arrays and the plan
  // that removes the deleted rows and columns of N.  Inserted spins take
  // slots k0 .. k0+mi-1; holes left below the new order are filled from the
  // surviving slots above it (remap[dst] = src, moves[] = (dst, src) pairs).
  // Nothing later in the window reads the vertex arrays or the order, so
  // both are final here.  Every wavefront computes the plan (their registers
  // agree); the first one stores it.
  __shared__ int ins_s[KS_MAX], hole_s[KS_MAX], src_s[KS_MAX], rem[KS_MAX], row_s[KS_MAX];
  const int knew = kcur;
  // lane s < m looks at the element in position s of S; inserted spins are
  // numbered in S order, removed slots ranked by value (they are distinct)
  // (the shuffles run in every lane: a lane that skips one would not serve
  // its value to the others)
  const int e_l = lane < m ? sa : 0;
  const int cand_l = __shfl(e_cand, e_l, 64), eslot_l = __shfl(e_slot, e_l, 64);
  const int flip_l = __shfl(e_flip, e_l, 64);
  const bool isc = lane < m && cand_l >= 0;
  const bool isf = lane < m && !isc && flip_l;      // flipped: stays, with s -> -s
  const bool isr = lane < m && !isc && !flip_l;
  const unsigned long long cmask = __ballot(isc), rmask = __ballot(isr);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int mi = __popcll(cmask), mr = __popcll(rmask);
  const int slot_l = isr ? eslot_l : 0x7fffffff;
  int rank = 0;
  for (int b = 0; b < m; ++b) rank += __builtin_amdgcn_readlane(slot_l, b) < slot_l;
  if (w0) {
    if (isc) {
      const int x = __popcll(cmask & below);
      ins_s[x] = e_l;
      row_s[lane] = k0 + x;
    }
    if (isr) {
      row_s[lane] = slot_l;
      rem[rank] = slot_l;
    }
    if (isf) row_s[lane] = eslot_l;
  }
  __syncthreads();
  const int kx = k0 + mi;
  // holes: the removed slots below the new order, in increasing order;
  // sources: the surviving slots in [knew, kx) (there are as many)
  const int nh = __popcll(__ballot(isr && slot_l < knew));
  bool surv = false;
  if (lane < kx - knew) {
    surv = true;
    for (int a = 0; a < mr; ++a) surv &= rem[a] != knew + lane;
  }
  const unsigned long long smask = __ballot(surv);
  if (w0) {
    if (lane < nh) hole_s[lane] = rem[lane];
    if (surv) src_s[__popcll(smask & below)] = knew + lane;
  }
  if (t0) {
    moves[2 * KS_MAX] = nh;
    if (bad) latch(c, ST_NUMERIC);
    c->m = m;
    c->mi = mi;
    c->mr = mr;
    c->kx = kx;
    c->knew = knew;
    c->k = knew;
    c->sign = sign;
    c->next_id = next_id;
    c->n_prop += n_done;
    c->n_acc_ins += n_ins;
    c->n_acc_rem += n_rem;
    c->n_acc_flip += n_flip;
    c->n_neglect += n_neg;
    c->n_mismatch += n_mis;
    c->pos += n_done;
    c->n_windows += 1;
    c->m_hist[(m + 3) >> 2] += 1;
    if (carry >= 0) {
      c->carry_id = carry;
      c->carry_kind = carry_kind;
      c->n_abort += 1;
    }
    {
      // both spins: X_C reads N and W_C, writes X_C; Y reads N and the
      // inserted spins' g columns, writes Y
      const double kk = (double)k0, b = (double)sizeof(T);
      if (nC > 0) {
        c->cand_flops += 2.0 * 2.0 * kk * kk * (double)nC;
        c->cand_bytes += 2.0 * (kk * kk + 2.0 * nC * kk) * b;
      }
      if (mi > 0) {
        c->y_flops += 2.0 * 2.0 * kk * kk * (double)mi;
        c->y_bytes += 2.0 * (kk * kk + 2.0 * mi * kk) * b;
      }
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
  if (m == 0) return;
  for (int i = t; i < knew; i += AW) remap[i] = i;
  if (w0) {
    if (lane < m) {
      gp(w.S)[lane] = sa;
      el_row[sa] = row_s[lane];
    }
    if (lane < mi) gp(w.ins_el)[lane] = ins_s[lane];
    if (lane < nh) {
      moves[2 * lane] = hole_s[lane];
      moves[2 * lane + 1] = src_s[lane];
    }
  }
  const auto v_site = gp(w.v_site), v_s = gp(w.v_s);
  const auto v_tau = gp(w.v_tau);
  const auto v_id = gp(w.v_id);
  // flipped vertices keep their slots with the opposite auxiliary spin (the
  // fold's factors use the element's spin from before the window)
  if (w0 && isf) v_s[eslot_l] = -v_s[eslot_l];
  __syncthreads();
  // window-start vertices that fill holes keep their values: read them
  // before the inserted spins land on slots >= k0
  int h_site = 0, h_s = 0;
  double h_tau = 0.0;
  long long h_id = 0;
  const bool hole = w0 && lane < nh && src_s[lane] < k0;
  if (hole) {
    const int sidx = src_s[lane];
    h_site = v_site[sidx];
    h_tau = v_tau[sidx];
    h_s = v_s[sidx];
    h_id = v_id[sidx];
  }
  __syncthreads();
  const int e_ins = lane < mi ? ins_s[lane] : 0;
  const int s_ins = __shfl(e_spin, e_ins, 64), c_ins = __shfl(e_cand, e_ins, 64);
  if (w0 && lane < mi) {
    v_site[k0 + lane] = gp(w.el_site)[e_ins];
    v_tau[k0 + lane] = gp(w.el_tau)[e_ins];
    v_s[k0 + lane] = s_ins;
    v_id[k0 + lane] = cid_s[c_ins];
  }
  // an inserted spin that moves into a hole: its element's values
  int e_h = 0;
  if (lane < nh && src_s[lane] >= k0) e_h = ins_s[src_s[lane] - k0];
  const int s_h = __shfl(e_spin, e_h, 64), c_h = __shfl(e_cand, e_h, 64);
  __syncthreads();
  if (w0 && lane < nh) {
    const int d = hole_s[lane], sidx = src_s[lane];
    remap[d] = sidx;
    if (sidx >= k0) {
      h_site = gp(w.el_site)[e_h];
      h_tau = gp(w.el_tau)[e_h];
      h_s = s_h;
      h_id = cid_s[c_h];
    }
    v_site[d] = h_site;
    v_tau[d] = h_tau;
    v_s[d] = h_s;
    v_id[d] = h_id;
  }
}

// --------------------------------------------------------- Y = N g_{I,c}
// Columns N g_{I,c} for the inserted spins (a k0 x k0 x mi product).  A
// workgroup owns 16 rows; its wavefronts split the inner dimension and their
// partial tiles are summed in LDS in a fixed order.
template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) k_ygemm(const View<T>* __restrict__ vs) {
  constexpr int GWV = NW;
  typedef typename Mfma<T>::acc_t acc_t;
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int mi = uni(c->mi), k0 = uni(c->k0);
  if (mi == 0) return;
  const int sp = blockIdx.y;
  const size_t ld = uni((long long)w.ld);
  const auto N = gp(w.N[sp]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ncb = (mi + 15) >> 4;
  // the inserted spins' columns g_{I,c}; absent columns read a zero column
  // offset of -1 (never dereferenced)
  const auto gcol = gp(w.gcol[sp]);
  long long goff[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int jj = cb * 16 + li;
    goff[cb] = (jj < mi) ? (long long)w.el_cand[w.ins_el[jj]] * w.cap : -1;
  }
  __shared__ acc_t red[GWV][4][64];
  // row tiles of 16, grid-strided over blockIdx.x
  for (int r0 = blockIdx.x * 16; r0 < k0; r0 += gridDim.x * 16) {
    const int ir = r0 + li;
    acc_t acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = acc_t{0, 0, 0, 0};
    // blocks of 16 columns of N, four consecutive per lane: the lane's four
    // column entries (each load coalesced over the 16 rows of the tile) and
    // four consecutive entries of each g column (vector loads)
    const int irc = ir < k0 ? ir : 0;
    const T imask = (T)(ir < k0 ? 1 : 0);
    if constexpr (NW < 8) {
      // batches: two steps per pass (see the candidate rows)
      for (int j0 = 4 * wv; j0 < k0; j0 += 8 * GWV) {
        T av[2], bv[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int jk = j0 + 4 * GWV * u + lk;
          const bool kin = jk < k0;
          const int jkc = kin ? jk : 0;
          av[u] = N[irc + (size_t)jkc * ld] * (T)(kin ? 1 : 0) * imask;
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            bv[u][cb] = gcol[(goff[cb] >= 0 ? goff[cb] : 0) + jkc] * (T)((kin && goff[cb] >= 0) ? 1 : 0);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            if (cb < ncb) acc[cb] = Mfma<T>::run(av[u], bv[u][cb], acc[cb]);
      }
    } else
    for (int j0 = 16 * uni(wv); j0 < k0; j0 += 16 * GWV) {
      const int jb = j0 + 4 * lk;
      const bool full = j0 + 16 <= k0;      // the same in every lane
      // every load of the step first (columns jb + 3 < k0 + 16 lie inside N
      // and the g columns), then the masks, so that the loads issue together
      T av[4], bt[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = N[irc + (size_t)(jb + u) * ld];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) Load4<T>::run(gcol + (goff[cb] >= 0 ? goff[cb] : 0) + jb, bt[cb]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool col = full || jb + u < k0;
        av[u] = col ? av[u] * imask : (T)0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) bt[cb][u] = (col && goff[cb] >= 0) ? bt[cb][u] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          if (cb < ncb) acc[cb] = Mfma<T>::run(av[u], bt[cb][u], acc[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) red[wv][cb][lane] = acc[cb];
    __syncthreads();
    const int cb = wv;
    if (cb < ncb) {
      acc_t sum = red[0][cb][lane];
      for (int v = 1; v < GWV; ++v) sum += red[v][cb][lane];
      const int jj = cb * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + Mfma<T>::row(lane, r);
        if (i < k0 && jj < mi) gp(w.Y[sp])[(size_t)jj * w.cap + i] = sum[r];
      }
    }
    __syncthreads();      // red is rewritten by the next tile
  }
}

// Y columns for launches with many workgroups: a workgroup owns 64 rows of
// Y and runs over the inner dimension in chunks of 32 columns of N (a
// column's 64 rows are two or four 128-byte lines, loaded coalesced),
// staged in LDS transposed beside the chunk of the inserted spins' g
// columns, which are then read once per 64 rows instead of once per 16.  Wavefront v computes
// rows 16 v .. 16 v + 15 of the tile for every block of inserted spins.
template <typename T>
__global__ void __launch_bounds__(256) k_ygemm_t(const View<T>* __restrict__ vs) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int P = LdsPad<T>::P;
  const View<T>& w = vs[blockIdx.z];
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int mi = uni(c->mi), k0 = uni(c->k0);
  if (mi == 0) return;
  const int sp = blockIdx.y;
  const auto N = gp(w.N[sp]);
  const auto Y = gp(w.Y[sp]);
  const auto gcol = gp(w.gcol[sp]);
  const size_t ld = uni((long long)w.ld), cap = uni((long long)w.cap);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ncb = (mi + 15) >> 4;
  __shared__ __attribute__((aligned(16))) T Ns[64 * P];        // [row][chunk column]
  __shared__ __attribute__((aligned(16))) T Gs[KS_MAX * P];    // [inserted spin][chunk column]
  // loader roles: N column t / 8 of the chunk, tile rows 8 (t % 8) .. + 7;
  // g column of inserted spin t / 4, chunk columns 8 (t % 4) .. + 7
  const int nj = t >> 3, nr = (t & 7) * 8;
  const int gc = t >> 2, gj = (t & 3) * 8;
  const bool gin = gc < mi;
  const auto gsrc = gcol + (gin ? (size_t)w.el_cand[w.ins_el[gc]] * cap : (size_t)0);
  for (int r0 = blockIdx.x * 64; r0 < k0; r0 += gridDim.x * 64) {
    acc_t acc[4], tot[4];     // two-level sums, as in the candidate rows
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = tot[cb] = acc_t{0, 0, 0, 0};
    T nv[8], gv[8];
    // rows r0 + nr .. + 7 < k0 + 64 and columns j0 + gj .. + 7 < k0 + 32 lie
    // inside the allocations (rows of cap elements); what lies past k0 is
    // zeroed when stored
    auto fetch = [&](int j0) {
      const int jj = j0 + nj;
      load8_raw(N + (size_t)(jj < k0 ? jj : 0) * ld, r0 + nr, nv);
      load8_raw(gsrc, j0 + gj, gv);
    };
    fetch(0);
    for (int j0 = 0; j0 < k0; j0 += XT_KC) {
      __syncthreads();
      const bool jin = j0 + nj < k0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        Ns[(nr + u) * P + nj] = (jin && r0 + nr + u < k0) ? nv[u] : (T)0;
        Gs[gc * P + gj + u] = (gin && j0 + gj + u < k0) ? gv[u] : (T)0;
      }
      __syncthreads();
      if (j0 + XT_KC < k0) fetch(j0 + XT_KC);
#pragma unroll
      for (int kb = 0; kb < XT_KC / 16; ++kb) {
        T a4[4];
        lds_read4(&Ns[(wv * 16 + li) * P + kb * 16 + 4 * lk], a4);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if (cb < ncb) {
            T b4[4];
            lds_read4(&Gs[(cb * 16 + li) * P + kb * 16 + 4 * lk], b4);
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) acc[cb] = Mfma<T>::run(a4[s2], b4[s2], acc[cb]);
          }
        }
      }
      if ((j0 / XT_KC) % XT_GROUP == XT_GROUP - 1) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          tot[cb] += acc[cb];
          acc[cb] = acc_t{0, 0, 0, 0};
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb < ncb) {
        tot[cb] += acc[cb];
        const int cc = cb * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = r0 + wv * 16 + Mfma<T>::row(lane, r);
          if (i < k0 && cc < mi) Y[(size_t)cc * cap + i] = tot[cb][r];
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ fold prep
// Fold factors in the extended index space (window-start vertices, then the
// inserted spins at rows k0 .. k0+mi-1), for N' = N + A B with
// A = (E_S - G_{.S}) diag(-Delta_S) and B = Gt_S^{-1} N_{S.}:
//   rows < k0 of A: an inserted spin c gives Delta_c (N g_{I,c}), a removed
//     vertex p gives e_p - N_{.p}, a flipped one (1 + e^{-V_p})(e_p - N_{.p});
//   B with the rows of the extended N (X_c for the inserted spins).
// The rows of the inserted spins come out of the fold as B itself: for x in
// S, Gt_{x,S} Gt_S^{-1} = e_x, so X_x + (e_x - Gt_{x,S}) B = B_x exactly.
// Evaluating that sum instead cancels X_x against X_x, which loses digits
// whenever the new row is small (e^{V_x} - 1 large), and those errors grow
// in later windows.  So A is zero on the inserted rows and B_x is stored
// there directly; on the rows < k0 the inserted columns (e_{k0+j}) are zero.
// The same holds for the row p of a flipped spin (row p of A is
// e_p - Gt_{p,S}): its folded row is B_p, which the sum would reach only
// through a cancellation of terms up to (1 + e^{gamma}) |N| (flips towards
// e^{V} = e^{gamma}); so A is zero on flipped rows too and B_p is stored
// there, over every column (the inserted ones included).  No workgroup reads
// a flipped row of N here, so the stores cannot race with the loads of A.
// A workgroup covers 64 columns; its four wavefronts share the S rows.
template <typename T>
__global__ void __launch_bounds__(WG) k_fold_prep(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z];
  const int* el_row = w.el_row;
  const Ctl* c = w.ctl;
  if (!c->active) return;
  const int m = c->m;
  const int sp = blockIdx.y;
  const int k0 = c->k0, mi = c->mi, kx = k0 + mi;
  if ((int)blockIdx.x * 64 >= kx) return;
  __shared__ double gi_s[KS_MAX * KS_MAX];
  __shared__ double rv_s[KS_MAX][64];
  __shared__ int e_s[KS_MAX], row_s[KS_MAX], cand_s[KS_MAX], slot_s[KS_MAX], flip_s[KS_MAX];
  __shared__ double d_s[KS_MAX], f_s[KS_MAX];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  {
    // Gt_S^{-1} rows into LDS, the loads of eight entries per thread together
    const auto gi = gp(w.ginv[sp]);
    for (int x0 = t; x0 < m * KS_MAX; x0 += 8 * WG) {
      double gv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = x0 + u * WG;
        gv[u] = gi[idx < m * KS_MAX ? idx : x0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = x0 + u * WG;
        if (idx < m * KS_MAX) gi_s[idx] = (idx % KS_MAX < m) ? gv[u] : 0.0;
      }
    }
  }
  if (t < m) {
    const int e = w.S[t];
    e_s[t] = e;
    row_s[t] = el_row[e];
    cand_s[t] = w.el_cand[e];
    slot_s[t] = w.el_slot[e];
    d_s[t] = w.ev[sp][s01(w.el_s[e])] - 1.0;
    // a target's column of A is f (e_p - N_{.p}): f = 1 for a removal,
    // -Delta_p e^{V_p} / (e^{V_p} - 1) = 1 + e^{-V_p} for a flip (the
    // element's spin is the one before the window)
    f_s[t] = w.el_flip[e] ? 1.0 + w.ev[sp][1 - s01(w.el_s[e])] : 1.0;
    flip_s[t] = w.el_flip[e];
  }
  __syncthreads();
  const T* R = w.R[sp];
  T* N = w.N[sp];
  const size_t ld = w.ld;
  const T* Y = w.Y[sp];
  const auto Ag = gp(w.A[sp]);
  const auto Bg = gp(w.B[sp]);
  constexpr int NWV = WG / 64;
  // groups of 64 columns, grid-strided over blockIdx.x.  A wavefront takes
  // the entries q = wv, wv + 4, ... of S eight at a time: the rows of N for
  // B and the entries of A are loaded together, then stored.
  for (int i0 = blockIdx.x * 64; i0 < kx; i0 += gridDim.x * 64) {
    const int i = i0 + lane;
    const bool live = i < kx;
    const int ic = live ? i : 0;
    const int il = (ic < k0) ? ic : 0;
    // row i is the slot of a flipped spin: its row of A is zero and no entry
    // of it is read (the B phase stores it)
    bool frow = false;
    if (live && i < k0)
      for (int q = 0; q < m; ++q) frow |= flip_s[q] && slot_s[q] == i;
    for (int q0 = wv; q0 < m; q0 += 8 * NWV) {
      T rv[8], tv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * NWV;
        const int sc = q < m ? q : q0;
        rv[u] = R[(size_t)e_s[sc] * w.cap + il];
        // rows < k0 of A: Y for a candidate, column p of N for a removed or
        // flipped vertex
        tv[u] = (cand_s[sc] >= 0) ? Y[(size_t)(row_s[sc] - k0) * w.cap + il]
                                  : (frow ? (T)0 : N[il + (size_t)slot_s[sc] * ld]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * NWV;
        if (q < m) {
          double x = 0.0;
          if (live) x = (i < k0) ? (double)rv[u] : ((cand_s[q] >= 0 && row_s[q] == i) ? 1.0 : 0.0);
          rv_s[q][lane] = x;
        }
        if (live && q < m) {
          // A, column-major [s][i]; zero on the inserted rows
          double v = 0.0;
          if (i < k0 && !frow)
            v = (cand_s[q] >= 0) ? d_s[q] * (double)tv[u] : f_s[q] * ((i == slot_s[q] ? 1.0 : 0.0) - (double)tv[u]);
          Ag[(size_t)q * w.cap + i] = (T)v;
        }
        // inserted columns of the rows < k0 (no workgroup reads columns >= k0
        // of N here); a flipped row gets them from B
        if (live && i < k0 && q < mi && !frow) N[i + (size_t)(k0 + q) * ld] = (T)0;
      }
    }
    __syncthreads();
    if (live) {
      // B, row-major [a][i] = sum_b Gt^{-1}[a][b] Row_{S_b}[i], four rows a
      // per pass over rv_s (each sum runs over b in order); an inserted or
      // flipped spin's row of B is also its row of the folded N
      for (int a0 = wv; a0 < m; a0 += 4 * NWV) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int ar[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ar[u] = (a0 + u * NWV < m) ? a0 + u * NWV : a0;
        for (int b = 0; b < m; ++b) {
          const double r = rv_s[b][lane];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] += gi_s[ar[u] * KS_MAX + b] * r;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = a0 + u * NWV;
          if (a < m) {
            Bg[(size_t)a * w.cap + i] = (T)acc[u];
            if (cand_s[a] >= 0 || flip_s[a]) N[row_s[a] + (size_t)i * ld] = (T)acc[u];
          }
        }
      }
    }
    __syncthreads();      // rv_s is rewritten by the next group
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
  const auto Cg = gp(C);
  const auto Ag = gp(A);
  const auto Bg = gp(B);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jb = j0 + wv * 16;
  const int li = lane & 15, lk = lane >> 4;
  // the tile of C is loaded up front (addresses below cap in both
  // dimensions are inside N) and added after the products, so that its loads
  // and the panels' overlap
  T cv[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int ii = i0 + rb * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) cv[rb][r] = Cg[ii + (size_t)(jb + Mfma<T>::row(lane, r)) * ldc];
  }
  typename Mfma<T>::acc_t acc[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) acc[rb] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  // Sixteen steps of the inner dimension per pass, all their loads issued
  // before the first product; the remaining steps in passes of four.  Rows
  // and columns outside the tile are read (the panels hold KS_MAX rows of cap
  // entries, so every address is in bounds) but never stored; steps beyond K
  // are zeroed, since the panels' unused rows hold earlier windows' data.
  int s0 = 0;
  for (; s0 + 16 <= K; s0 += 16) {
    T bv[4], av[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t sk = (size_t)(s0 + 4 * u + lk);
      bv[u] = Bg[sk * ldb + jb + li];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) av[u][rb] = Ag[sk * lda + i0 + rb * 16 + li];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) acc[rb] = Mfma<T>::run(bv[u], av[u][rb], acc[rb]);
  }
  for (; s0 < K; s0 += 4) {
    const int sk = s0 + lk;
    const bool kin = sk < K;
    const size_t skc = kin ? (size_t)sk : 0;
    const T bb = Bg[skc * ldb + jb + li];
    const T bv = kin ? bb : (T)0;
    T av[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const T aa = Ag[skc * lda + i0 + rb * 16 + li];
      av[rb] = kin ? aa : (T)0;
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = Mfma<T>::run(bv, av[rb], acc[rb]);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int ii = i0 + rb * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = jb + Mfma<T>::row(lane, r);
      if (ii < M && jj < Nn) Cg[ii + (size_t)jj * ldc] = cv[rb][r] + acc[rb][r];
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
  const int kx = uni(c->kx), m = uni(c->m);
  if (m == 0) return;
  // 64 x 64 tiles of N, grid-strided over blockIdx.x
  const int nt = (kx + 63) >> 6;
  for (int t = blockIdx.x; t < nt * nt; t += gridDim.x)
    fold_tile<T>(w.N[sp], w.ld, w.A[sp], w.cap, w.B[sp], w.cap, kx, kx, m, (t % nt) * 64, (t / nt) * 64);
}

// ----------------------------------------------------------- compaction
// Drop the rows and columns of removed vertices: with remap and moves from
// the accept kernel, N[i][d] = N[remap(i)][s] and N[d][i] = N[s][remap(i)]
// for every move (d, s).  Sources lie at or above the new order and are
// never written, so the copy is race-free in place.
template <typename T>
__global__ void __launch_bounds__(WG) k_compact_move(const View<T>* __restrict__ vs) {
  const View<T>& w = vs[blockIdx.z >> 1];
  const auto remap = gp(w.remap);
  const auto moves = gp(w.moves);
  Ctl* c = w.ctl;
  if (!c->active) return;
  const int sp = blockIdx.z & 1;
  const int nh = moves[2 * KS_MAX];
  const int knew = c->knew;
  if (nh == 0) return;
  const auto N = gp(w.N[sp]);
  const size_t ld = w.ld;
  // the moves are read into LDS once; the copies of eight moves are loaded
  // together before they are stored (sources are never destinations)
  __shared__ int mv_s[2 * KS_MAX];
  for (int x = threadIdx.x; x < 2 * nh; x += WG) mv_s[x] = moves[x];
  __syncthreads();
  for (int i = blockIdx.x * WG + threadIdx.x; i < knew; i += gridDim.x * WG) {
    const int si = remap[i];
    for (int h0 = 0; h0 < nh; h0 += 8) {
      T cv[8], rv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (h0 + u < nh) {
          const int s = mv_s[2 * (h0 + u) + 1];
          cv[u] = N[si + (size_t)s * ld];
          rv[u] = N[s + (size_t)si * ld];
        }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (h0 + u < nh) {
          const int d = mv_s[2 * (h0 + u)];
          N[i + (size_t)d * ld] = cv[u];
          N[d + (size_t)i * ld] = rv[u];
        }
    }
  }
}

#define DCAX_INSTANTIATE(T)                                              \
  template __global__ void k_prep_replay<T>(const View<T>*);             \
  template __global__ void k_prep_rng<T>(const View<T>*);                \
  template __global__ void k_gather<T>(const View<T>*);                  \
  template __global__ void k_cand_x<T, 4>(const View<T>*);               \
  template __global__ void k_cand_x<T, 16>(const View<T>*);              \
  template __global__ void k_gram<T, 4>(const View<T>*);                 \
  template __global__ void k_gram_rows<T, 16>(const View<T>*);           \
  template __global__ void k_accept<T>(const View<T>*);                  \
  template __global__ void k_ygemm<T, 4>(const View<T>*);                \
  template __global__ void k_ygemm<T, 8>(const View<T>*);                \
  template __global__ void k_ygemm_t<T>(const View<T>*);                 \
  template __global__ void k_cand_xt<T>(const View<T>*);                 \
  template __global__ void k_fold_prep<T>(const View<T>*);               \
  template __global__ void k_fold<T>(const View<T>*);                    \
  template __global__ void k_compact_move<T>(const View<T>*);

DCAX_INSTANTIATE(double)
DCAX_INSTANTIATE(float)

}  // namespace dcax

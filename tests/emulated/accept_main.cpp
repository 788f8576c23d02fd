// Runs the accept kernel k_accept<double> on the host, one std::thread per
// work-item (see emu_hip.h), for random windows in both modes (replayed
// decisions, own generator), built with AddressSanitizer so that every
// buffer access is bounds-checked.  Checks: all lanes meet at the same
// collectives and barriers; replayed ratios equal determinant ratios of Gram
// submatrices; Gt_S^{-1} inverts Gram[S, S]; the compaction plan and the new
// vertex arrays hold exactly the surviving and the inserted vertices.
// Usage: accept_main <cases>; exit status 0 when every case passes.
#include "k_accept_emu.h"
#include <random>
thread_local emu_dim3 threadIdx, blockIdx;
EmuRendezvous* emu_wave[4];
EmuRendezvous* emu_block;
std::mutex emu_atomic_mu;
using namespace dcax;

template <typename X> X* arr(size_t n, X fill) { X* p = new X[n]; for (size_t i = 0; i < n; ++i) p[i] = fill; return p; }

static double det(std::vector<double> a, int n) {
  double d = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r) if (std::fabs(a[r * n + c]) > std::fabs(a[p * n + c])) p = r;
    if (a[p * n + c] == 0.0) return 0.0;
    if (p != c) { for (int k = 0; k < n; ++k) std::swap(a[p * n + k], a[c * n + k]); d = -d; }
    d *= a[c * n + c];
    for (int r = c + 1; r < n; ++r) {
      double f = a[r * n + c] / a[c * n + c];
      for (int k = c; k < n; ++k) a[r * n + k] -= f * a[c * n + k];
    }
  }
  return d;
}
static double detS(const double* G, const std::vector<int>& S) {
  int n = S.size();
  if (!n) return 1.0;
  std::vector<double> a(n * n);
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) a[i * n + j] = G[S[i] * KS_MAX + S[j]];
  return det(a, n);
}

int main(int argc, char** argv) {
  const int n_cases = argc > 1 ? atoi(argv[1]) : 50;
  int fails = 0;
  for (int cs = 0; cs < n_cases; ++cs) {
    std::mt19937_64 rng(1234 + cs);
    auto U = [&]() { return (double)(rng() >> 11) * (1.0 / 9007199254740992.0); };
    const bool replay = cs % 2;
    const int ks = (int[]){16, 32, 64}[cs % 3];
    const int k0 = (cs % 5 == 0) ? (int)(rng() % 6) : 20 + (int)(rng() % 200);
    const int cap = ((k0 + 2 * KS_MAX + 63) / 64) * 64;
    View<double> v{};
    v.ks = ks; v.cap = cap; v.ld = cap; v.max_order = (cs % 7 == 3) ? k0 + 2 : 100000;
    v.K_exp = 1.0; v.seed = 99 + cs;
    Ctl* c = new Ctl{};
    v.ctl = c;
    // elements: candidates then window-start targets
    int nC = std::min(ks, (int)(rng() % (ks + 1)));
    int nR = std::min(64 - nC, std::min(k0, (int)(rng() % 40)));
    if (cs % 4 == 0) { nC = std::min(ks, 64); nR = std::min(64 - nC, k0); }
    // tiny orders with both kinds of target element for every vertex (so
    // that removals and flips of one vertex meet in a window)
    const bool twins = k0 > 0 && k0 < 6 && cs % 3 != 0;
    if (twins) { nC = std::min(nC, 64 - 2 * k0); nR = 2 * k0; }
    const int nE = nC + nR;
    v.el_cand = arr<int>(KS_MAX, -1); v.el_slot = arr<int>(KS_MAX, -1); v.el_flip = arr<int>(KS_MAX, 0);
    v.neglect = (cs % 4 == 2) ? 1 : 0;
    v.el_s = arr<int>(KS_MAX, 1); v.el_site = arr<int>(KS_MAX, 0); v.el_tau = arr<double>(KS_MAX, 0.0);
    std::vector<int> slots(k0);
    for (int i = 0; i < k0; ++i) slots[i] = i;
    std::shuffle(slots.begin(), slots.end(), rng);
    for (int e = 0; e < nC; ++e) { v.el_cand[e] = e; v.el_s[e] = (rng() & 1) ? 1 : -1; v.el_site[e] = rng() % 16; v.el_tau[e] = U(); }
    for (int e = nC; e < nE && !twins; ++e) v.el_slot[e] = slots[e - nC];
    // a share of the window-start targets are spin-flip elements
    if (cs % 3 != 0)
      for (int e = nC; e < nE; ++e) v.el_flip[e] = (rng() % 3 == 0) ? 1 : 0;
    if (twins)
      for (int e = nC; e < nE; ++e) { v.el_slot[e] = (e - nC) % k0; v.el_flip[e] = (e - nC) >= k0; }
    for (int sp = 0; sp < 2; ++sp) {
      v.gram[sp] = arr<double>(KS_MAX * KS_MAX, 0.0);
      for (int i = 0; i < nE; ++i)
        for (int j = 0; j < nE; ++j)
          v.gram[sp][i * KS_MAX + j] = (i == j) ? ((rng() & 1) ? 1.0 : -1.0) * (1.5 + U()) : 0.25 * (U() - 0.5);
      v.ginv[sp] = arr<double>(KS_MAX * KS_MAX, NAN);
    }
    v.cand_id = arr<long long>(KS_MAX, -1);
    v.S = arr<int>(KS_MAX, -1); v.ins_el = arr<int>(KS_MAX, -1); v.el_row = arr<int>(KS_MAX, -1);
    v.remap = arr<int>(cap, -1); v.moves = arr<int>(2 * KS_MAX + 1, -1);
    v.v_site = arr<int>(cap, -7); v.v_tau = arr<double>(cap, -7.0); v.v_s = arr<int>(cap, 0); v.v_id = arr<long long>(cap, -7);
    for (int i = 0; i < k0; ++i) { v.v_site[i] = rng() % 16; v.v_tau[i] = U(); v.v_s[i] = (rng() & 1) ? 1 : -1; v.v_id[i] = 5000 + i; }
    std::vector<int> s_before(v.v_s, v.v_s + k0);
    // proposals
    const int nP = ks;
    v.wp = new WinProp[KS_MAX];
    std::vector<int> forced_in_S;   // replay: elements flipped so far (for consistent removals)
    std::vector<char> flipped(KS_MAX, 0);
    int next_c = 0;
    std::vector<int> ref_S;
    for (int j = 0; j < nP; ++j) {
      WinProp& p = v.wp[j];
      p = WinProp{};
      p.u = U(); p.ridx = replay ? j : -1; p.gidx = 777 + j; p.forced = -1; p.carried = 0;
      const bool ins = next_c < nC && (rng() % 3 != 0);
      if (ins) { p.kind = 0; p.el = next_c++; }
      else {
        p.kind = (cs % 3 != 0 && rng() % 2) ? 2 : 1;
        p.ub0 = U(); p.ui0 = U();
        int slot = k0 ? std::min((int)(p.ui0 * k0), k0 - 1) : 0;
        p.el = -1;
        for (int e = nC; e < nE; ++e) if (v.el_slot[e] == slot && v.el_flip[e] == (p.kind == 2)) p.el = e;
        if (replay) {
          // removal: a window-start removal element not yet removed, or an
          // inserted candidate; flip: any flip element (a second flip undoes it)
          std::vector<int> opts;
          if (p.kind == 1) {
            for (int e = nC; e < nE; ++e) if (!v.el_flip[e] && !flipped[e]) opts.push_back(e);
            for (int e = 0; e < nC; ++e) if (flipped[e]) opts.push_back(e);
          } else {
            for (int e = nC; e < nE; ++e) if (v.el_flip[e]) opts.push_back(e);
          }
          p.el = opts.empty() ? -1 : opts[rng() % opts.size()];
        }
      }
      if (replay) {
        p.forced = (int)(rng() % 2);
        if (p.el >= 0 && p.forced) flipped[p.el] ^= 1;
      }
    }
    if (!replay && cs % 3 == 1)      // a carried target keeps the kind its element was prepared for
      v.wp[0].carried = 1, v.wp[0].el = nE > nC ? nC : -1, v.wp[0].kind = (nE > nC && v.el_flip[nC]) ? 2 : 1;
    v.ratio_out = replay ? arr<double>(nP, NAN) : nullptr;
    if (!replay) for (int j = 0; j < nP; ++j) v.wp[j].ridx = -1;
    c->k = k0; c->active = 1; c->nP = nP; c->nE = nE; c->nC = nC; c->k0 = k0; c->next_id = 1000000;
    c->sign = 1.0; c->carry_id = -1;
    long long* cid_before = arr<long long>(KS_MAX, -1);
    // launch
    for (int i = 0; i < 4; ++i) emu_wave[i] = new EmuRendezvous(64);
    emu_block = new EmuRendezvous(256);
    std::vector<std::thread> th;
    View<double>* vs = &v;
    for (int t = 0; t < 256; ++t)
      th.emplace_back([t, vs]() { threadIdx.x = t; blockIdx = emu_dim3{}; k_accept<double>(vs); });
    for (auto& x : th) x.join();
    // checks
    const int m = c->m;
    bool ok = true;
    if (c->status) printf("case %d: status %d\n", cs, c->status);
    if (c->m > 0 && c->status == 0) {
      // vertex arrays: the survivors of the window start plus the inserted spins
      std::vector<long long> want, got(v.v_id, v.v_id + c->knew);
      std::vector<char> rm(k0, 0);
      for (int a = 0; a < c->m; ++a) { int e = v.S[a]; if (v.el_cand[e] < 0 && !v.el_flip[e]) rm[v.el_slot[e]] = 1; }
      // flipped vertices keep their slots with the opposite spin (before compaction moves them)
      std::vector<char> fl(k0, 0);
      for (int a = 0; a < c->m; ++a) { int e = v.S[a]; if (v.el_cand[e] < 0 && v.el_flip[e]) fl[v.el_slot[e]] = 1; }
      for (int d = 0; d < c->knew; ++d) {
        long long id = v.v_id[d];
        if (id >= 5000 && id < 5000 + k0) {
          int i = (int)(id - 5000);
          if (v.v_s[d] != (fl[i] ? -s_before[i] : s_before[i])) { printf("case %d: flipped spin of %d\n", cs, i); ok = false; break; }
        }
      }
      for (int i = 0; i < k0; ++i) if (!rm[i]) want.push_back(5000 + i);
      for (int a = 0; a < c->mi; ++a) want.push_back(v.cand_id[v.el_cand[v.ins_el[a]]]);
      std::sort(want.begin(), want.end()); std::sort(got.begin(), got.end());
      if (want != got) { printf("case %d: vertex ids differ\n", cs); ok = false; }
      // remap: destination d < knew takes source remap[d]; sources distinct and survivors
      std::vector<char> seen(cap, 0);
      for (int d = 0; d < c->knew; ++d) {
        int sidx = v.remap[d];
        if (sidx < 0 || sidx >= k0 + c->mi || seen[sidx] || (sidx < k0 && rm[sidx])) { printf("case %d: remap[%d]=%d\n", cs, d, sidx); ok = false; break; }
        seen[sidx] = 1;
      }
      for (int a = 0; a < c->m; ++a) {
        int e = v.S[a];
        int row = v.el_row[e];
        if (v.el_cand[e] >= 0 ? (row < k0 || row >= k0 + c->mi) : row != v.el_slot[e]) { printf("case %d: el_row\n", cs); ok = false; }
      }
    }
    if (replay && c->active && c->status == 0) {
      // reference ratios from determinants of Gram submatrices with the forced decisions
      std::vector<int> S;
      int kcur = k0;
      for (int j = 0; j < (int)c->n_prop; ++j) {
        const WinProp& p = v.wp[j];
        int q = p.el;
        if (q < 0) continue;
        auto it = std::find(S.begin(), S.end(), q);
        double r[2];
        std::vector<int> S2 = S;
        if (it == S.end()) S2.push_back(q); else S2.erase(S2.begin() + (it - S.begin()));
        for (int sp = 0; sp < 2; ++sp) r[sp] = detS(v.gram[sp], S2) / detS(v.gram[sp], S);
        double fac = p.kind == 0 ? 1.0 / (kcur + 1) : p.kind == 1 ? (double)kcur : 1.0;
        double R = fac * r[0] * r[1];
        double e = std::fabs(R - v.ratio_out[j]) / std::max(1.0, std::fabs(R));
        if (!(e < 1e-10)) { printf("case %d: ratio %d ref %.15g got %.15g\n", cs, j, R, v.ratio_out[j]); ok = false; break; }
        if (p.forced) { S = S2; kcur += p.kind == 0 ? 1 : p.kind == 1 ? -1 : 0; }
      }
    }
    if (c->active && m > 0 && c->status == 0) {
      // ginv = inverse of Gram[S,S] in S order
      std::vector<int> S(v.S, v.S + m);
      for (int sp = 0; sp < 2 && ok; ++sp)
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b) {
            double s = 0.0;
            for (int x = 0; x < m; ++x) s += v.gram[sp][S[a] * KS_MAX + S[x]] * v.ginv[sp][x * KS_MAX + b];
            if (std::fabs(s - (a == b)) > 1e-9) { printf("case %d: ginv check %d %d %g\n", cs, a, b, s); ok = false; a = m; break; }
          }
    }
    printf("case %2d %s ks=%2d k0=%3d nC=%2d nE=%2d nP=%2d done=%lld m=%d mi=%d mr=%d knew=%d abort=%lld flips=%lld "
           "neglected=%lld %s\n", cs, replay ? "replay" : "gen   ", ks, k0, nC, nE, nP, c->n_prop, c->m, c->mi, c->mr,
           c->knew, c->n_abort, c->n_acc_flip, c->n_neglect, ok ? "ok" : "FAIL");
    fails += !ok;
  }
  printf("%d failures\n", fails);
  return fails != 0;
}

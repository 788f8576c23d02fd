"""CPU check of the submatrix (delayed) update algebra the HIP kernels use.

Sec. 2.3 fuses k_s single-spin updates into one rank-k_s operation but gives
no formulas; the identities below follow from N^{-1} = e^V - g (e^V - 1).
With G = N g, for a set S of flipped auxiliary spins with
Delta_p = e^{V'_p - V_p} - 1:

* Gamma_S = G_SS - diag((1 + Delta_p) / Delta_p);
* det N'^{-1} / det N^{-1} = prod_{p in S} (-Delta_p) det Gamma_S;
* N' = N + (E_S - G_{.S}) Gamma_S^{-1} N_{S.};
* an insertion flips a non-interacting spin (V = 0) whose N row is
  X_q = g_{q,I} (e^{V_I} - 1) N and column e_q; removing flips V_p -> 0 and
  deletes row and column p.

Gamma_S is singular where Delta = 0 (U = 0, where every flip leaves V
unchanged).  The kernels therefore carry the column-scaled matrix
Gt = Gamma_S diag(-Delta), Gt_xy = -Delta_y G_xy + delta_xy (1 + Delta_y),
which is finite everywhere:

* the ratio is det Gt, so adding q multiplies it by the Schur complement
  Gt_qq - Gt_qS Gt_S^{-1} Gt_Sq and taking q out again by (Gt_S^{-1})_qq;
* N' = N + (E_S - G_{.S}) diag(-Delta) Gt_S^{-1} N_{S.}; the scaled column of
  a removed vertex is exactly e_p - N_{.p} (since (-Delta_p) e^{V_p} /
  (e^{V_p} - 1) = 1), that of an inserted spin -Delta_c (e_c - G_{.c});
* the column of Gt for a removed vertex p is N_ext{x,p} itself, from
  G (e^V - 1) = N e^V - 1; for a flipped vertex (V_p -> -V_p) it is
  (1 + e^{-V_p}) N_ext{x,p} - delta_xp e^{-V_p}, and its scaled column of the
  fold (1 + e^{-V_p}) (e_p - N_{.p});
* for x in S, row x of (E_S - G_{.S}) diag(-Delta) is e_x - Gt_{x,S}, so the
  folded row x is B_x exactly: inserted and flipped rows are taken from B
  (the sum would cancel terms up to (1 + e^{gamma}) |N| for a flip).

``WindowModel`` is a NumPy transcription of the kernel pipeline (gathers,
candidate rows, scaled Gram matrix of the window, sequential Schur loop,
fold with compaction).  It is test code: the HIP library does not import it.
Replaying an oracle trace through it must reproduce every ratio and the
final N, also at U = 0.
"""

import numpy as np
import pytest

from oracle import ctaux
from tests.ctaux_cases import exact_replay_with_flip_conditioning, records


def test_gamma_identities_random():
    rng = np.random.default_rng(0)
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=3.0, n_tau=500)
    for trial in range(20):
        k = int(rng.integers(3, 12))
        r = rng.integers(0, 4, size=k)
        t = rng.random(k) * m.beta
        s = rng.choice([-1, 1], size=k)
        spin = trial % 2
        Ninv = ctaux.n_inverse(m, r, t, s, spin)
        N = np.linalg.inv(Ninv)
        g = m.prop.matrix(r, t)
        G = N @ g
        S = rng.choice(k, size=int(rng.integers(1, k)), replace=False)
        s_new = s.copy()
        s_new[S] = -s[S]
        V = (1 if spin == 0 else -1) * m.gamma * s
        Vn = (1 if spin == 0 else -1) * m.gamma * s_new
        Delta = np.exp(Vn[S] - V[S]) - 1.0
        Gam = G[np.ix_(S, S)] - np.diag((1 + Delta) / Delta)
        ratio = np.prod(-Delta) * np.linalg.det(Gam)
        Ninv_new = ctaux.n_inverse(m, r, t, s_new, spin)
        assert abs(ratio - np.linalg.det(Ninv_new) / np.linalg.det(Ninv)) < 1e-10 * abs(ratio)
        E = np.zeros((k, len(S)))
        E[S, np.arange(len(S))] = 1.0
        N_fold = N + (E - G[:, S]) @ np.linalg.solve(Gam, N[S, :])
        assert np.max(np.abs(N_fold - np.linalg.inv(Ninv_new))) < 1e-11 * np.max(np.abs(N_fold))
        # column-scaled form
        Gt = -Delta[None, :] * G[np.ix_(S, S)] + np.diag(1.0 + Delta)
        assert abs(np.linalg.det(Gt) - ratio) < 1e-10 * abs(ratio)
        A = (E - G[:, S]) * (-Delta)[None, :]
        N_fold2 = N + A @ np.linalg.solve(Gt, N[S, :])
        assert np.max(np.abs(N_fold2 - N_fold)) < 1e-11 * np.max(np.abs(N_fold))
        # columns of removed (here: flipped) vertices from N alone
        ev = np.exp(V[S])
        Gcol = (N[:, S] * ev[None, :] - E) / (ev - 1.0)[None, :]
        assert np.max(np.abs(Gcol - G[:, S])) < 1e-10 * np.max(np.abs(G[:, S]))


def test_scaled_gamma_is_finite_at_u0():
    """At U = 0 every Delta vanishes: Gt = 1, ratio 1, and N stays the identity."""
    rng = np.random.default_rng(3)
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=0.0, beta=3.0, n_tau=500)
    assert m.gamma == 0.0
    k = 7
    r = rng.integers(0, 4, size=k)
    t = rng.random(k) * m.beta
    s = rng.choice([-1, 1], size=k)
    N = np.linalg.inv(ctaux.n_inverse(m, r, t, s, 0))
    assert np.array_equal(N, np.eye(k))
    G = N @ m.prop.matrix(r, t)
    S = np.array([1, 4, 5])
    Delta = np.zeros(len(S))
    Gt = -Delta[None, :] * G[np.ix_(S, S)] + np.diag(1.0 + Delta)
    assert np.array_equal(Gt, np.eye(len(S)))
    E = np.zeros((k, len(S)))
    E[S, np.arange(len(S))] = 1.0
    A = (E - G[:, S]) * (-Delta)[None, :]
    assert np.array_equal(N + A @ np.linalg.solve(Gt, N[S, :]), np.eye(k))


class WindowModel:
    """NumPy transcription of the window pipeline, replaying forced decisions."""

    def __init__(self, model, r, t, s, ids, schur="sweep"):
        self.m = model
        # "sweep": Gauss-Jordan sweeps of the window's Gram matrix (ratios are
        # diagonal entries); "border": the inverse over S grown by bordering
        self.schur = schur
        self.r, self.t, self.s, self.id = (np.array(x) for x in (r, t, s, ids))
        self.N = [np.linalg.inv(ctaux.n_inverse(model, self.r, self.t, self.s, sp)) for sp in (0, 1)]
        self.ratios = []

    def ev(self, s, sp):
        return self.m.ev(s, sp)

    def window(self, props):
        """props: list of (kind, site, tau, s, id, accepted), kind 0 insertion,
        1 removal, 2 flip of an auxiliary spin.  A proposal that would change
        a spin the window has already changed otherwise (a flip of a spin
        inserted in the window, a removal of a flipped one) ends the window
        before it; returns the number of proposals taken."""
        m = self.m
        k0 = len(self.r)
        slot_of = {int(v): i for i, v in enumerate(self.id)}
        # -- element list: candidates and window-start targets --------------
        el_r, el_t, el_s, el_slot, el_flip = [], [], [], [], []      # slot -1 for candidates
        cand_of_id = {}
        prop_el = []
        on = []
        for (kind, site, tau, sq, vid, acc) in props:
            if kind == 0:
                prop_el.append(len(el_r))
                el_r.append(site); el_t.append(tau); el_s.append(sq); el_slot.append(-1); el_flip.append(0)
                on.append(0)
                if acc:
                    cand_of_id[int(vid)] = prop_el[-1]
            else:
                fl = int(kind == 2)
                if int(vid) in cand_of_id:
                    if fl:
                        break
                    prop_el.append(cand_of_id[int(vid)])
                else:
                    p = slot_of[int(vid)]
                    mine = [e for e in range(len(el_r)) if el_slot[e] == p and el_flip[e] == fl]
                    twin = [e for e in range(len(el_r)) if el_slot[e] == p and el_flip[e] != fl]
                    if twin and on[twin[0]]:
                        assert not fl, "a flip of a vertex the window removed"
                        break
                    if mine:
                        prop_el.append(mine[0])
                    else:
                        prop_el.append(len(el_r))
                        el_r.append(self.r[p]); el_t.append(self.t[p]); el_s.append(self.s[p]); el_slot.append(p)
                        el_flip.append(fl)
                        on.append(0)
            if acc:
                on[prop_el[-1]] ^= 1
        props = props[:len(prop_el)]
        nE = len(el_r)
        el_r, el_t, el_s, el_slot, el_flip = map(np.array, (el_r, el_t, el_s, el_slot, el_flip))
        cand = el_slot < 0
        ci = np.where(cand)[0]
        ti = np.where(~cand)[0]
        tslot = el_slot[ti]
        # gathers only for insertion candidates: column g_{I,c}, row g_{c,I}, g_{c,c'}
        gcol = m.prop.g(self.r[:, None], self.t[:, None], el_r[None, ci], el_t[None, ci])  # (k0, nC)
        grow = m.prop.g(el_r[ci, None], el_t[ci, None], self.r[None, :], self.t[None, :])  # (nC, k0)
        gCC = m.prop.g(el_r[ci, None], el_t[ci, None], el_r[None, ci], el_t[None, ci])
        Rw, Gram, Xs = [], [], []
        for sp in (0, 1):
            evI = self.ev(self.s, sp)
            X = (grow * (evI - 1.0)[None, :]) @ self.N[sp]             # candidate rows of N_ext
            R = np.zeros((nE, k0))
            R[ci] = X
            R[ti] = self.N[sp][tslot, :]
            Gm = np.zeros((nE, nE))
            # candidate columns: Gt_{x,c} = -Delta_c G_{x,c} + delta_xc (1 + Delta_c),
            # G_{x,c} = R_x . g_{I,c} (+ g_{x,c} for candidate rows)
            Dc = self.ev(el_s[ci], sp) - 1.0
            Gm[:, ci] = R @ gcol
            Gm[np.ix_(ci, ci)] += gCC
            Gm[:, ci] *= -Dc[None, :]
            Gm[ci, ci] += 1.0 + Dc
            # columns of existing vertices p: Gt_{x,p} = N_ext{x,p} for a
            # removal, (1 + e^{-V_p}) N_ext{x,p} - delta_xp e^{-V_p} for a flip
            Gm[:, ti] = R[:, tslot]
            fi = ti[el_flip[ti] == 1]
            if len(fi):
                emv = 1.0 / self.ev(el_s[fi], sp)
                Gm[:, fi] *= (1.0 + emv)[None, :]
                Gm[fi, fi] -= emv
            Rw.append(R)
            Gram.append(Gm)
        # -- sequential Schur loop ---------------------------------------
        loop = self._sweep_loop if self.schur == "sweep" else self._border_loop
        S, Ginv = loop(props, prop_el, Gram, k0)
        # -- fold in the extended space, then compaction --------------------
        ins = [q for q in S if cand[q]]
        rem = [el_slot[q] for q in S if not cand[q] and not el_flip[q]]
        flips = [el_slot[q] for q in S if el_flip[q]]
        mi = len(ins)
        kx = k0 + mi
        row_of = {}
        for q in S:
            row_of[q] = (k0 + ins.index(q)) if cand[q] else el_slot[q]
        ins_ids = []
        id_iter = iter([p[4] for p in props if p[0] == 0 and p[5]])
        cand_id = {}
        for (kind, site, tau, sq, vid, acc), q in zip(props, prop_el):
            if kind == 0 and acc:
                cand_id[q] = vid
        for sp in (0, 1):
            Next = np.zeros((kx, kx))
            Next[:k0, :k0] = self.N[sp]
            for j, q in enumerate(ins):
                Next[k0 + j, :k0] = Rw[sp][q]
                Next[k0 + j, k0 + j] = 1.0
            if S:
                # A = (E_S - G_ext[:, S]) diag(-Delta) on the rows < k0: existing
                # p: e_p - N_{.p}; candidate c: Delta_c N g_{I,c}
                A = np.zeros((kx, len(S)))
                for j, q in enumerate(S):
                    if cand[q]:
                        Dq = self.ev(el_s[q], sp) - 1.0
                        A[:k0, j] = Dq * (self.N[sp] @ m.prop.g(self.r, self.t, el_r[q], el_t[q]))
                    else:
                        p = el_slot[q]
                        e = np.zeros(kx)
                        e[p] = 1.0
                        A[:, j] = e - Next[:, p]
                        if el_flip[q]:
                            A[:, j] *= 1.0 + 1.0 / self.ev(el_s[q], sp)
                # the inserted and the flipped rows of the result are rows of
                # B (for x in S, row x of A is e_x - Gt_{x,S} and
                # Gt_{x,S} Gt_S^{-1} = e_x): A is zero there
                A[k0:, :] = 0.0
                for q in S:
                    if el_flip[q]:
                        A[el_slot[q], :] = 0.0
                rows = [row_of[q] for q in S]
                B = Ginv[sp] @ Next[rows, :]
                Next = Next + A @ B
                for j, q in enumerate(S):
                    if cand[q] or el_flip[q]:
                        Next[row_of[q], :] = B[j, :]
            keep = np.array([i for i in range(kx) if i not in rem], dtype=int)
            self.N[sp] = Next[np.ix_(keep, keep)]
        new_r = np.concatenate([self.r, el_r[ins]])
        new_t = np.concatenate([self.t, el_t[ins]])
        s_now = self.s.copy()
        s_now[flips] = -s_now[flips]
        new_s = np.concatenate([s_now, el_s[ins]])
        new_id = np.concatenate([self.id, np.array([cand_id[q] for q in ins], dtype=self.id.dtype)])
        keep = np.array([i for i in range(kx) if i not in rem], dtype=int)
        self.r, self.t, self.s, self.id = new_r[keep], new_t[keep], new_s[keep], new_id[keep]
        return len(props)

    def run(self, props, k_s):
        """Windows of at most k_s proposals until every proposal is taken."""
        i = 0
        while i < len(props):
            i += self.window(props[i:i + k_s])

    def _border_loop(self, props, prop_el, Gram, kcur):
        """Inverse over S grown by bordering and shrunk by a rank-1 downdate."""
        m = self.m
        S = []
        Ginv = [np.zeros((0, 0)), np.zeros((0, 0))]
        for (kind, site, tau, sq, vid, acc), q in zip(props, prop_el):
            if q in S:
                j = S.index(q)
                rat = [Ginv[sp][j, j] for sp in (0, 1)]
            else:
                rat, parts = [], []
                for sp in (0, 1):
                    gqS = Gram[sp][q, S]
                    gSq = Gram[sp][S, q]
                    L = Ginv[sp] @ gSq
                    Rr = gqS @ Ginv[sp]
                    schur = Gram[sp][q, q] - gqS @ L
                    rat.append(schur)
                    parts.append((L, Rr, schur))
            fac = m.K_exp / (kcur + 1) if kind == 0 else kcur / m.K_exp if kind == 1 else 1.0
            self.ratios.append(fac * rat[0] * rat[1])
            if not acc:
                continue
            if q in S:
                j = S.index(q)
                for sp in (0, 1):
                    A = Ginv[sp]
                    A = A - np.outer(A[:, j], A[j, :]) / A[j, j]
                    keep = np.arange(len(S)) != j
                    Ginv[sp] = A[np.ix_(keep, keep)]
                S.pop(j)
            else:
                for sp in (0, 1):
                    L, Rr, schur = parts[sp]
                    n = len(S)
                    B = np.empty((n + 1, n + 1))
                    B[:n, :n] = Ginv[sp] + np.outer(L, Rr) / schur
                    B[:n, n] = -L / schur
                    B[n, :n] = -Rr / schur
                    B[n, n] = 1.0 / schur
                    Ginv[sp] = B
                S.append(q)
            kcur += 1 if kind == 0 else -1 if kind == 1 else 0
        return S, Ginv

    def _sweep_loop(self, props, prop_el, Gram, kcur):
        """Sweep tableau T (one per spin), started at the Gram matrix.  After
        sweeping the set S, T_SS = -Gt_S^{-1} and the other diagonal entries
        are the Schur complements Gt_qq - Gt_qS Gt_S^{-1} Gt_Sq: the ratio of
        flipping q is T_qq, that of unflipping q in S is -T_qq, and either
        acceptance is one sweep (reverse sweep for an unflip) on q."""
        T = [Gram[0].copy(), Gram[1].copy()]
        S = []
        for (kind, site, tau, sq, vid, acc), q in zip(props, prop_el):
            sgn = -1.0 if q in S else 1.0
            rat = [sgn * T[sp][q, q] for sp in (0, 1)]
            fac = self.m.K_exp / (kcur + 1) if kind == 0 else kcur / self.m.K_exp if kind == 1 else 1.0
            self.ratios.append(fac * rat[0] * rat[1])
            if not acc:
                continue
            for sp in (0, 1):
                A = T[sp]
                inv = 1.0 / A[q, q]
                col, row = A[:, q].copy(), A[q, :] * inv
                A -= np.outer(col, row)
                A[q, :] = sgn * row
                A[:, q] = sgn * col * inv
                A[q, q] = -inv
            if sgn < 0:
                j = S.index(q)
                S[j] = S[-1]             # the last position fills the hole
                S.pop()
            else:
                S.append(q)
            kcur += 1 if kind == 0 else -1 if kind == 1 else 0
        return S, [-T[sp][np.ix_(S, S)] for sp in (0, 1)]

    def canonical(self):
        o = np.argsort(self.id)
        return self.id[o], self.N[0][np.ix_(o, o)], self.N[1][np.ix_(o, o)]


@pytest.mark.parametrize("schur", ["sweep", "border"])
@pytest.mark.parametrize("k_s,seed,U", [(4, 1, 4.0), (16, 2, 4.0), (64, 3, 4.0), (16, 4, 0.0)])
def test_window_model_replays_oracle(k_s, seed, U, schur):
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=U, beta=5.0, n_tau=1000)
    w = ctaux.Walker(m, seed=seed, k_s=k_s, record=False)
    w.random_config(25)
    for _ in range(20):              # equilibrate, then replay from a refreshed state
        w.sweep()
    w.refresh()
    w.record = True
    r0, t0, s0, id0 = w.r.copy(), w.t.copy(), w.s.copy(), w.id.copy()
    for _ in range(6):
        w.sweep()
    tr = w.trace
    wm = WindowModel(m, r0, t0, s0, id0, schur=schur)
    n_unflip = 0
    for i in range(0, len(tr), k_s):
        chunk = tr[i:i + k_s]
        props = [(rec[0], rec[1], rec[2], rec[3], rec[4], rec[7]) for rec in chunk]
        inserted = {p[4] for p in props if p[0] == 0 and p[5]}
        n_unflip += sum(1 for p in props if p[0] == 1 and p[4] in inserted)
        # removal at k = 0 carries no target; the model skips such records
        props = [p for p in props if not (p[0] == 1 and p[4] < 0)]
        wm.window(props)
    ref = np.array([rec[6] for rec in tr if not (rec[0] == 1 and rec[4] < 0)])
    assert len(ref) > 50
    got = np.array(wm.ratios)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-10
    ids, Nu, Nd = w.canonical()
    ids2, Nu2, Nd2 = wm.canonical()
    assert np.array_equal(ids, ids2)
    for A, B in ((Nu, Nu2), (Nd, Nd2)):
        assert A.shape == B.shape
        if A.size:
            assert np.max(np.abs(A - B)) / np.max(np.abs(A)) < 1e-10
    if k_s == 64:
        assert n_unflip > 0      # the exact "spin touched twice" path was exercised
    if U == 0.0:
        assert np.array_equal(Nu2, np.eye(len(ids2))) and np.array_equal(Nd2, np.eye(len(ids2)))


@pytest.mark.parametrize("k_s,seed", [(16, 5), (32, 6), (64, 7)])
def test_window_model_replays_oracle_with_flips(k_s, seed):
    """Flips of auxiliary spins in the window: the flip element's Gram column
    (1 + e^{-V_p}) N_ext{x,p} - delta_xp e^{-V_p} and fold column
    (1 + e^{-V_p}) (e_p - N_{.p}) reproduce the single-spin chain; windows
    end before a second change of one spin.  A flip ratio is a difference of
    terms up to e^{gamma} N_pp: it is held to 1e-10 times its condition
    number kappa with respect to N_pp (insertions and removals: kappa = 1),
    against the extended-precision chain, as is the FP64 oracle."""
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=5.0, n_tau=1000)
    w = ctaux.Walker(m, seed=seed, k_s=k_s, p_flip=0.3)
    w.random_config(25)
    for _ in range(20):
        w.sweep()
    w.refresh()
    w.record = True
    init = (w.r.copy(), w.t.copy(), w.s.copy(), w.id.copy())
    for _ in range(30):
        w.sweep()
    rec, ro = records(w.trace)
    good = ~((rec["kind"] >= 1) & (rec["id"] < 0))
    rx, ch, kap = exact_replay_with_flip_conditioning(m, init, rec)
    props = [(int(r["kind"]), int(r["site"]), float(r["tau"]), int(r["aux_spin"]), int(r["id"]), int(r["accepted"]))
             for r in rec[good]]
    assert sum(1 for p in props if p[0] == 2 and p[5]) > 20
    wm = WindowModel(m, *init)
    n_win = 0
    i = 0
    while i < len(props):
        i += wm.window(props[i:i + k_s])
        n_win += 1
    assert n_win > -(-len(props) // k_s)          # some windows ended early
    got = np.array(wm.ratios)
    for r in (got, ro[good]):
        assert np.all(np.abs(r - rx[good]) <= 1e-10 * kap[good] * np.abs(rx[good]))
    ids_x, Xu, Xd = ch.canonical()
    ids2, Nu2, Nd2 = wm.canonical()
    assert np.array_equal(ids_x, ids2)
    assert np.array_equal(ch.s[np.argsort(ch.id)], wm.s[np.argsort(wm.id)])
    for A, X in ((Nu2, Xu), (Nd2, Xd)):
        assert float(np.max(np.abs(A.astype(np.longdouble) - X)) / np.max(np.abs(X))) < 1e-10

"""Extended-precision replay of a recorded single-vertex chain (Sec. 2.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The FP64 oracle chain and any FP64 submatrix evaluation both carry rounding
that the conditioning of N amplifies: on doped clusters the determinant
ratio of a proposal is a Schur complement of terms of size e^{gamma} that
cancel to O(1e-2).  To tell which of two FP64 evaluations is right, this
module replays the same proposals in x87 extended precision
(numpy.longdouble: 64-bit significand, eps = 1.1e-19, 2^11 times finer than
FP64's 2.2e-16) with the textbook single-vertex algebra:

* N_sigma = [e^{V_sigma} - g (e^{V_sigma} - 1)]^{-1} by Gauss-Jordan
  elimination with partial pivoting, at the start and after every
  `reinvert_every` accepted moves;
* insertion ratio d - W N Q (bordered inverse), removal ratio N_pp
  (cofactor identity), R = K/(k+1) or k/K times the product over spins;
  the flip of an auxiliary spin changes one column of N^{-1}: ratio
  1 + (N d)_p per spin (matrix determinant lemma), R the product;
* the bordered-inverse, rank-one-downdate and Sherman-Morrison updates of N.

The propagator g between vertices is the same linear interpolation of the
FP64 table as ``g0.interp``, evaluated in extended precision.  Results are
returned rounded to FP64 (ratios) and in extended precision (N).
"""
import numpy as np

LD = np.longdouble


def gj_inverse(A):
    """Inverse of a square matrix by Gauss-Jordan elimination with partial
    pivoting, in the dtype of A (vectorised over rows)."""
    n = A.shape[0]
    M = np.concatenate([A.copy(), np.eye(n, dtype=A.dtype)], axis=1)
    for c in range(n):
        p = c + int(np.argmax(np.abs(M[c:, c])))
        if M[p, c] == 0:
            raise np.linalg.LinAlgError("singular matrix")
        if p != c:
            M[[c, p]] = M[[p, c]]
        M[c] = M[c] / M[c, c]
        f = M[:, c].copy()
        f[c] = 0
        M -= np.outer(f, M[c])
    return M[:, n:]


class ExactChain:
    """The single-vertex chain in extended precision, replaying forced decisions."""

    def __init__(self, model, r, t, s, ids, reinvert_every=64):
        if getattr(model, "h", 0.0) != 0.0:
            raise ValueError("the extended-precision replay takes one propagator for both spins (h = 0)")
        self.m = model
        self.r = np.asarray(r, np.int64).copy()
        self.t = np.asarray(t, np.float64).copy()
        self.s = np.asarray(s, np.int64).copy()
        self.id = np.asarray(ids, np.int64).copy()
        self.reinvert_every = reinvert_every
        self.table = np.asarray(model.table, dtype=LD)
        self.h = LD(model.beta) / LD(model.table.shape[1] - 1)
        self.n_acc = 0
        self.reinvert()

    # -- propagator and weights -----------------------------------------
    def _G0(self, d, dtau):
        x = np.asarray(dtau, dtype=LD) / self.h
        l = np.clip(np.floor(x).astype(np.int64), 0, self.table.shape[1] - 2)
        f = x - l.astype(LD)
        return (LD(1) - f) * self.table[d, l] + f * self.table[d, l + 1]

    def g(self, ri, ti, rj, tj):
        """g(i, j) = -G0(r_i - r_j, tau_i - tau_j) (0+ at equal times), with
        the antiperiodic image for tau_i < tau_j."""
        ri, rj = np.broadcast_arrays(np.asarray(ri), np.asarray(rj))
        ti, tj = np.broadcast_arrays(np.asarray(ti, LD), np.asarray(tj, LD))
        d = self.m.diff[ri, rj]
        dt = ti - tj
        neg = dt < 0
        val = self._G0(d, np.where(neg, dt + LD(self.m.beta), dt))
        return np.where(neg, val, -val)

    def ev(self, s, spin):
        sig = 1 if spin == 0 else -1
        return np.exp(LD(sig) * LD(self.m.gamma) * np.asarray(s, dtype=LD))

    def n_inverse(self, spin):
        ev = self.ev(self.s, spin)
        g = self.g(self.r[:, None], self.t[:, None], self.r[None, :], self.t[None, :])
        return np.diag(ev) - g * (ev - LD(1))[None, :]

    def reinvert(self):
        k = len(self.r)
        self.N = [gj_inverse(self.n_inverse(sp)) if k else np.zeros((0, 0), LD) for sp in (0, 1)]

    @property
    def k(self):
        return len(self.r)

    # -- moves ------------------------------------------------------------
    def insert_ratio(self, rq, tq, sq):
        g_Iq = self.g(self.r, self.t, rq, tq)
        g_qI = self.g(rq, tq, self.r, self.t)
        g_qq = self.g(rq, tq, rq, tq)
        parts = []
        for sp in (0, 1):
            evq = self.ev(sq, sp)
            Q = -g_Iq * (evq - LD(1))
            W = -g_qI * (self.ev(self.s, sp) - LD(1))
            d = evq - g_qq * (evq - LD(1))
            NQ = self.N[sp] @ Q
            WN = W @ self.N[sp]
            parts.append((d - W @ NQ, NQ, WN))
        return parts

    def flip_ratio(self, p):
        """Flip of the auxiliary spin at row p: only column p of N^{-1}
        changes, by d = (e^{V'_p} - e^{V_p}) (e_p - g_{.p}), so per spin the
        ratio is 1 + (N d)_p (matrix determinant lemma) and N' = N - N d
        N_{p.} / ratio (Sherman-Morrison)."""
        g_p = self.g(self.r, self.t, self.r[p], self.t[p])
        parts = []
        for sp in (0, 1):
            dv = self.ev(-self.s[p], sp) - self.ev(self.s[p], sp)
            d = -dv * g_p
            d[p] += dv
            Nd = self.N[sp] @ d
            parts.append((LD(1) + Nd[p], Nd))
        return parts

    def step(self, kind, site, tau, aux_spin, vid, accepted):
        """Replay one record; returns the full acceptance ratio R (FP64)."""
        m = self.m
        k = self.k
        if kind == 0:
            parts = self.insert_ratio(site, tau, aux_spin)
            R = LD(m.K_exp) / LD(k + 1) * parts[0][0] * parts[1][0]
            if accepted:
                for sp in (0, 1):
                    ratio, NQ, WN = parts[sp]
                    Nn = np.empty((k + 1, k + 1), LD)
                    Nn[:k, :k] = self.N[sp] + np.outer(NQ, WN) / ratio
                    Nn[:k, k] = -NQ / ratio
                    Nn[k, :k] = -WN / ratio
                    Nn[k, k] = LD(1) / ratio
                    self.N[sp] = Nn
                self.r = np.append(self.r, site)
                self.t = np.append(self.t, tau)
                self.s = np.append(self.s, aux_spin)
                self.id = np.append(self.id, vid)
        elif kind == 2:
            if vid < 0:
                return 0.0
            p = int(np.nonzero(self.id == vid)[0][0])
            parts = self.flip_ratio(p)
            R = parts[0][0] * parts[1][0]
            if accepted:
                for sp in (0, 1):
                    ratio, Nd = parts[sp]
                    self.N[sp] = self.N[sp] - np.outer(Nd, self.N[sp][p]) / ratio
                self.s[p] = -self.s[p]
        else:
            if vid < 0:
                return 0.0
            p = int(np.nonzero(self.id == vid)[0][0])
            R = LD(k) / LD(m.K_exp) * self.N[0][p, p] * self.N[1][p, p]
            if accepted:
                keep = np.arange(k) != p
                for sp in (0, 1):
                    N = self.N[sp]
                    self.N[sp] = N[np.ix_(keep, keep)] - np.outer(N[keep, p], N[p, keep]) / N[p, p]
                self.r, self.t, self.s, self.id = (x[keep] for x in (self.r, self.t, self.s, self.id))
        if accepted:
            self.n_acc += 1
            if self.reinvert_every and self.n_acc % self.reinvert_every == 0:
                self.reinvert()
        return float(R)

    def canonical(self):
        """(ids, N_up, N_dn) in id order, extended precision."""
        o = np.argsort(self.id)
        return self.id[o], self.N[0][np.ix_(o, o)], self.N[1][np.ix_(o, o)]


def replay(model, init, records, reinvert_every=64):
    """Ratios (FP64) of every record and the final chain, in extended precision.

    init: (r, t, s, ids); records: rows with fields kind, site, tau, aux_spin,
    id, accepted (kind 0 insertion, 1 removal, 2 flip; a removal or flip with
    id < 0 is the no-op at order 0, ratio 0)."""
    ch = ExactChain(model, *init, reinvert_every=reinvert_every)
    out = np.array([ch.step(int(x["kind"]), int(x["site"]), float(x["tau"]), int(x["aux_spin"]), int(x["id"]),
                            int(x["accepted"])) for x in records])
    return out, ch


class RefinedChain:
    """The single-vertex chain at large orders, its ratios solved to extended
    precision by iterative refinement.

    A Gauss-Jordan inverse in extended precision costs O(k^3) numpy steps on
    80-bit numbers, too slow at k ~ 2000-6000.  Here A_sigma = N_sigma^{-1}
    = e^V - g (e^V - 1) is assembled exactly as the FP64 oracle assembles it
    (the same rounded propagator values), an FP64 inverse of it serves as the
    preconditioner, and each ratio needs one solve: x = A^{-1} b is refined
    with residuals b - A x accumulated in extended precision until the
    correction is below 1e-18 of x, or stalls below 1e-12 of it: at the
    floor set by the extended-precision residual (eps_80 |A| |x|, which the
    column scales e^{+-gamma} of A make ~1e-16 at k ~ 2000), about 1e-14 of x
    on the random 6x6 configurations of order 2000.  So the ratios are exact for the FP64
    entries of A (to eps_80 times the conditioning), and the first-order
    bound of a ratio's change under a relative perturbation eps of every entry
    of A (the rounding any FP64 evaluation starts from) is returned beside
    each ratio:
        insertion, rho = d - W A^{-1} Q:  |W| |x| + |y| |Q| + |y| |A| |x| + |d|,
            x = A^{-1} Q, y^T = W A^{-1};
        removal, rho = (A^{-1})_pp:       |y| |A| |x|, x = A^{-1} e_p,
            y = A^{-T} e_p;
    for each spin, combined for R = fac rho_up rho_dn as
    |R| (b_up / |rho_up| + b_dn / |rho_dn|).
    """

    def __init__(self, model, r, t, s, ids, reinvert_every=32, refine=True):
        if getattr(model, "h", 0.0) != 0.0:
            raise ValueError("the extended-precision replay takes one propagator for both spins (h = 0)")
        self.m = model
        self.refine = refine
        self.r = np.asarray(r, np.int64).copy()
        self.t = np.asarray(t, np.float64).copy()
        self.s = np.asarray(s, np.int64).copy()
        self.id = np.asarray(ids, np.int64).copy()
        self.reinvert_every = reinvert_every
        self.n_acc = 0
        self.A = [self._n_inverse(sp) for sp in (0, 1)]
        self.Al = [a.astype(LD) if refine else None for a in self.A]
        self.P = [np.linalg.inv(a) for a in self.A]
        self.iterations = 0

    def _n_inverse(self, spin):
        ev = self.m.ev(self.s, spin)
        g = self.m.prop.matrix(self.r, self.t)
        return np.diag(ev) - g * (ev - 1.0)[None, :]

    @property
    def k(self):
        return len(self.r)

    def _solve(self, sp, b, transpose=False):
        P = self.P[sp].T if transpose else self.P[sp]
        x = (P @ np.asarray(b, np.float64)).astype(LD)
        if not self.refine:
            return x
        Al = self.Al[sp].T if transpose else self.Al[sp]
        bl = np.asarray(b, LD)
        prev = np.inf
        for _ in range(16):
            res = bl - Al @ x
            dx = (P @ res.astype(np.float64)).astype(LD)
            x += dx
            self.iterations += 1
            step = float(np.max(np.abs(dx)) / np.max(np.abs(x)))
            # converged, or stalled at the extended-precision residual's floor
            if step <= 1e-18 or (step > 0.25 * prev and step < 1e-12):
                break
            prev = step
        else:
            raise ArithmeticError("iterative refinement did not converge")
        return x

    def _insert_parts(self, rq, tq, sq):
        m = self.m
        g_Iq = m.prop.g(self.r, self.t, rq, tq)
        g_qI = m.prop.g(rq, tq, self.r, self.t)
        g_qq = float(m.prop.g(rq, tq, rq, tq))
        out = []
        for sp in (0, 1):
            evq = float(m.ev(sq, sp))
            Q = -g_Iq * (evq - 1.0)
            W = -g_qI * (m.ev(self.s, sp) - 1.0)
            d = evq - g_qq * (evq - 1.0)
            if self.k:
                x = self._solve(sp, Q)
                y = self._solve(sp, W, transpose=True)
                rho = LD(d) - np.asarray(W, LD) @ x
                xa, ya = np.abs(x).astype(np.float64), np.abs(y).astype(np.float64)
                bound = np.abs(W) @ xa + ya @ np.abs(Q) + ya @ (np.abs(self.A[sp]) @ xa) + abs(d)
            else:
                rho, bound = LD(d), abs(d)
            out.append((rho, float(bound), Q, W, d))
        return out

    def flip_ratio(self, p):
        """Flip of the auxiliary spin at row p: only column p of N^{-1}
        changes, by d = (e^{V'_p} - e^{V_p}) (e_p - g_{.p}), so per spin the
        ratio is 1 + (N d)_p (matrix determinant lemma) and N' = N - N d
        N_{p.} / ratio (Sherman-Morrison)."""
        g_p = self.g(self.r, self.t, self.r[p], self.t[p])
        parts = []
        for sp in (0, 1):
            dv = self.ev(-self.s[p], sp) - self.ev(self.s[p], sp)
            d = -dv * g_p
            d[p] += dv
            Nd = self.N[sp] @ d
            parts.append((LD(1) + Nd[p], Nd))
        return parts

    def step(self, kind, site, tau, aux_spin, vid, accepted):
        """Replay one record; returns (R, bound) in FP64 (R = 0, bound 0 for the
        no-op removal at order 0)."""
        m = self.m
        k = self.k
        if kind == 0:
            parts = self._insert_parts(site, tau, aux_spin)
            rho = [p[0] for p in parts]
            R = LD(m.K_exp) / LD(k + 1) * rho[0] * rho[1]
            b = abs(float(R)) * sum(p[1] / abs(float(p[0])) for p in parts)
            if accepted:
                for sp in (0, 1):
                    _, _, Q, W, d = parts[sp]
                    A = np.empty((k + 1, k + 1))
                    A[:k, :k] = self.A[sp]
                    A[:k, k] = Q
                    A[k, :k] = W
                    A[k, k] = d
                    self.A[sp] = A
                    if self.refine:
                        self.Al[sp] = A.astype(LD)
                    # the preconditioner by the FP64 bordered inverse
                    Pm = self.P[sp]
                    NQ, WN = Pm @ Q, W @ Pm
                    ratio = d - W @ NQ
                    Pn = np.empty((k + 1, k + 1))
                    Pn[:k, :k] = Pm + np.outer(NQ, WN) / ratio
                    Pn[:k, k] = -NQ / ratio
                    Pn[k, :k] = -WN / ratio
                    Pn[k, k] = 1.0 / ratio
                    self.P[sp] = Pn
                self.r = np.append(self.r, site)
                self.t = np.append(self.t, tau)
                self.s = np.append(self.s, aux_spin)
                self.id = np.append(self.id, vid)
        else:
            if vid < 0:
                return 0.0, 0.0
            p = int(np.nonzero(self.id == vid)[0][0])
            rho, bnd = [], []
            for sp in (0, 1):
                e = np.zeros(k)
                e[p] = 1.0
                x = self._solve(sp, e)
                y = self._solve(sp, e, transpose=True)
                rho.append(x[p])
                bnd.append(float(np.abs(y).astype(np.float64) @ (np.abs(self.A[sp]) @ np.abs(x).astype(np.float64))))
            R = LD(k) / LD(m.K_exp) * rho[0] * rho[1]
            b = abs(float(R)) * sum(bb / abs(float(rr)) for rr, bb in zip(rho, bnd))
            if accepted:
                keep = np.arange(k) != p
                for sp in (0, 1):
                    self.A[sp] = self.A[sp][np.ix_(keep, keep)]
                    if self.refine:
                        self.Al[sp] = self.Al[sp][np.ix_(keep, keep)]
                    Pm = self.P[sp]
                    self.P[sp] = Pm[np.ix_(keep, keep)] - np.outer(Pm[keep, p], Pm[p, keep]) / Pm[p, p]
                self.r, self.t, self.s, self.id = (x[keep] for x in (self.r, self.t, self.s, self.id))
        if accepted:
            self.n_acc += 1
            if self.reinvert_every and self.n_acc % self.reinvert_every == 0:
                self.P = [np.linalg.inv(a) for a in self.A]
        return float(R), float(b)

    def column(self, sp, j):
        """Column j (list order) of N_sigma = A^{-1}, extended precision."""
        e = np.zeros(self.k)
        e[j] = 1.0
        return self._solve(sp, e)


def replay_refined(model, init, records, refine=True):
    """(ratios, first-order bounds per unit rounding, chain) of a replay at large
    order.  refine=False skips the refinement: the ratios are then the FP64
    single-vertex ones and only the bounds are of interest (they need x and y
    to a few digits)."""
    ch = RefinedChain(model, *init, refine=refine)
    out = [ch.step(int(x["kind"]), int(x["site"]), float(x["tau"]), int(x["aux_spin"]), int(x["id"]),
                   int(x["accepted"])) for x in records]
    return np.array([o[0] for o in out]), np.array([o[1] for o in out]), ch

"""Single-vertex CT-AUX Markov chain (Sec. 2.3), plain NumPy float64.

Weights (Sec. 2.3, the expansion of Z and the auxiliary-field decoupling):

* cosh(gamma) = 1 + U beta Nc / (2 K_exp) for the single-band Hubbard model
  (N_corr = Nc);
* a configuration {(r_i, tau_i, s_i)}, i = 1..k, weighs
  (K_exp / (2 beta Nc))^k prod_sigma det N_sigma^{-1};
* N_sigma^{-1} = e^{V_sigma} - g_sigma (e^{V_sigma} - 1), e^{V_sigma,i} =
  e^{sigma gamma s_i} (sigma = +1 up, -1 down), g = -G0 between vertices
  with the 0+ value on the diagonal (see ``g0.Propagator``).

Moves (Sec. 2.3, the Metropolis updates of the vertex configuration): each
proposal draws five uniforms u0..u4 from a Mersenne-twister stream.  u0 < 1/2
proposes inserting a vertex at site floor(u1 Nc), time u2 beta, auxiliary
spin +1 if u3 < 1/2 else -1, accepted with probability
min(1, |K_exp/(k+1) prod_sigma ratio_sigma|); otherwise the vertex at list
position floor(u1 k) is proposed for removal with factor k/K_exp (a removal
at k = 0 is a rejected no-op).  u4 is compared with |R|; the sign of the
configuration is multiplied by sgn(R) on acceptance.  With a flip share
p_flip > 0 (the spin-flip move of the paper's figure of CT-AUX moves), u0
below (1 - p_flip)/2 inserts, below 1 - p_flip removes, and otherwise the
auxiliary spin of the vertex at list position floor(u1 k) is proposed to
flip, accepted with min(1, |prod_sigma ratio_sigma|) (a symmetric move at
fixed order: no expansion-parameter factor).

Determinant ratios and updates are the textbook single-vertex ones:
insertion is a bordered inverse (Schur complement d - W N Q), removal the
cofactor identity ratio = N_pp followed by the rank-one downdate
N_{-p,-p} - N_{-p,p} N_{p,-p} / N_pp.  The submatrix method of Sec. 2.3 fuses
k_s of these single updates into one rank-k_s operation and, with the "abort"
or exact treatment of a spin touched twice, produces exactly this chain, so
this chain is the plain definition the GPU path must reproduce.

A sweep is max(k_start, 1) proposals rounded up to a multiple of k_s (the
paper counts sweeps between measurements without defining one).
"""
import math
import numpy as np

from . import geometry, g0 as g0mod


class Model:
    """Hubbard model on a periodic cluster, finite-size mode."""

    def __init__(self, a1=(2, 0), a2=(0, 2), t=1.0, tp=0.0, U=4.0, beta=5.0, mu=0.0,
                 K_exp=1.0, n_tau=1000, use_table=True, h=0.0, tables=None):
        """h: a Zeeman field, -h sum_i (n_iup - n_idown) in H0, so that the
        spins see xi_sigma = eps_K - mu - sigma h (sigma = +1 up, -1 down)
        and the walker one bare propagator per spin.
        tables: the bare propagator given as tables (one per spin, each
        (Nc, n_tau), standard convention, the grid of ``g0.tau_grid``), e.g.
        the cluster-excluded G0 of the DCA loop; t, tp, mu and h then only
        describe the lattice."""
        self.a1, self.a2 = tuple(a1), tuple(a2)
        self.t, self.tp, self.U, self.beta, self.mu, self.h = t, tp, U, beta, mu, h
        self.K_exp = K_exp
        self.n_tau = n_tau
        self.sites = geometry.cluster_sites(self.a1, self.a2)
        self.K = geometry.cluster_momenta(self.a1, self.a2)
        self.Nc = len(self.sites)
        self.diff = geometry.diff_table(self.a1, self.a2)
        self.eps = geometry.dispersion(self.K, t, tp)
        self.xis = [self.eps - mu - h, self.eps - mu + h]
        self.xi = self.xis[0]
        self.gamma = math.acosh(1.0 + U * beta * self.Nc / (2.0 * K_exp))
        self.tables, self.props = [], []
        if tables is not None:
            for sp in range(2):
                tab = np.asarray(tables[sp], np.float64)
                if tab.shape != (self.Nc, n_tau):
                    raise ValueError("a table must be (Nc, n_tau)")
                self.tables.append(tab)
                self.props.append(g0mod.Propagator(self.diff, beta, table=tab))
            self.table, self.prop = self.tables[0], self.props[0]
            return
        for sp in range(2 if h != 0.0 else 1):
            tab = g0mod.g0_table(self.sites, self.K, self.xis[sp], beta, n_tau)
            analytic = (lambda d, tau, sp=sp: self._g0_exact(d, tau, sp))
            self.tables.append(tab)
            self.props.append(g0mod.Propagator(self.diff, beta, table=tab if use_table else None,
                                               analytic=analytic))
        if h == 0.0:
            self.tables.append(self.tables[0])
            self.props.append(self.props[0])
        self.table, self.prop = self.tables[0], self.props[0]

    def _g0_exact(self, d, tau, spin=0):
        d = np.asarray(d)
        tau = np.asarray(tau, float)
        flat_d, flat_t = d.ravel(), tau.ravel()
        gk = g0mod.g0_K_tau(self.xis[spin], flat_t, self.beta)        # (NcK, T)
        ph = np.exp(1j * self.sites[flat_d].astype(float) @ self.K.T)  # (T, NcK)
        val = np.einsum("tk,kt->t", ph, gk).real / self.Nc
        return val.reshape(d.shape)

    def ev(self, s, spin):
        """e^{V_sigma} for auxiliary spins s; spin 0 = up (+), 1 = down (-)."""
        sig = 1.0 if spin == 0 else -1.0
        return np.exp(sig * self.gamma * np.asarray(s, dtype=np.float64))


def n_inverse(model, r, t, s, spin):
    """N_sigma^{-1} = e^V - g (e^V - 1) for a vertex list."""
    ev = model.ev(s, spin)
    g = model.props[spin].matrix(r, t)
    return np.diag(ev) - g * (ev - 1.0)[None, :]


class Walker:
    """One CT-AUX Markov chain with single-vertex updates."""

    def __init__(self, model, seed, k_s=16, record=False, p_flip=0.0):
        """p_flip: share of proposals that flip the auxiliary spin of an
        existing vertex (Sec. 2.3's figure of the CT-AUX moves); insertions
        and removals share the rest equally."""
        self.m = model
        self.p_flip = float(p_flip)
        self.n_acc_flip = 0
        self.rng = np.random.Generator(np.random.MT19937(seed))
        self.k_s = int(k_s)
        self.frozen_length = 0
        self.r = np.zeros(0, np.int64)
        self.t = np.zeros(0, np.float64)
        self.s = np.zeros(0, np.int64)
        self.id = np.zeros(0, np.int64)
        self.N = [np.zeros((0, 0)), np.zeros((0, 0))]
        self.sign = 1.0
        self.next_id = 0
        self.record = record
        self.trace = []
        self.n_prop = 0
        self.n_acc_ins = 0
        self.n_acc_rem = 0
        self.drifts = []

    @property
    def k(self):
        return len(self.r)

    # -- configuration ----------------------------------------------------
    def set_config(self, r, t, s, ids=None):
        self.r = np.asarray(r, np.int64).copy()
        self.t = np.asarray(t, np.float64).copy()
        self.s = np.asarray(s, np.int64).copy()
        k = len(self.r)
        self.id = np.arange(k, dtype=np.int64) if ids is None else np.asarray(ids, np.int64).copy()
        self.next_id = int(self.id.max()) + 1 if k else 0
        sgn = 1.0
        for spin in range(2):
            A = n_inverse(self.m, self.r, self.t, self.s, spin)
            self.N[spin] = np.linalg.inv(A) if k else np.zeros((0, 0))
            if k:
                sgn *= np.linalg.slogdet(A)[0]
        self.sign = sgn

    def random_config(self, k):
        """k random interacting vertices (App. B, initial-configuration-size)."""
        u = self.rng.random((k, 3))
        r = np.floor(u[:, 0] * self.m.Nc).astype(np.int64)
        t = u[:, 1] * self.m.beta
        s = np.where(u[:, 2] < 0.5, 1, -1)
        self.set_config(r, t, s)

    def refresh(self):
        """Replace N by a direct float64 inversion; return the relative drift."""
        drift = 0.0
        for spin in range(2):
            if self.k == 0:
                continue
            Nn = np.linalg.inv(n_inverse(self.m, self.r, self.t, self.s, spin))
            drift = max(drift, np.max(np.abs(self.N[spin] - Nn)) / np.max(np.abs(Nn)))
            self.N[spin] = Nn
        self.drifts.append(drift)
        return drift

    # -- moves ------------------------------------------------------------
    def _insert_ratio(self, rq, tq, sq):
        m = self.m
        out = []
        for spin in range(2):
            g_Iq = m.props[spin].g(self.r, self.t, rq, tq)
            g_qI = m.props[spin].g(rq, tq, self.r, self.t)
            g_qq = float(m.props[spin].g(rq, tq, rq, tq))
            evq = float(m.ev(sq, spin))
            evI = m.ev(self.s, spin)
            Q = -g_Iq * (evq - 1.0)
            W = -g_qI * (evI - 1.0)
            d = evq - g_qq * (evq - 1.0)
            NQ = self.N[spin] @ Q
            WN = W @ self.N[spin]
            ratio = d - W @ NQ
            out.append((ratio, NQ, WN))
        return out

    def _do_insert(self, rq, tq, sq, parts):
        for spin in range(2):
            ratio, NQ, WN = parts[spin]
            k = self.k
            Nn = np.empty((k + 1, k + 1))
            Nn[:k, :k] = self.N[spin] + np.outer(NQ, WN) / ratio
            Nn[:k, k] = -NQ / ratio
            Nn[k, :k] = -WN / ratio
            Nn[k, k] = 1.0 / ratio
            self.N[spin] = Nn
        new_id = self.next_id
        self.next_id += 1
        self.r = np.append(self.r, rq)
        self.t = np.append(self.t, tq)
        self.s = np.append(self.s, sq)
        self.id = np.append(self.id, new_id)
        return new_id

    def _do_remove(self, p):
        last = self.k - 1
        for spin in range(2):
            N = self.N[spin]
            if p != last:
                perm = np.arange(self.k)
                perm[p], perm[last] = last, p
                N = N[np.ix_(perm, perm)]
            self.N[spin] = N[:-1, :-1] - np.outer(N[:-1, -1], N[-1, :-1]) / N[-1, -1]
        for name in ("r", "t", "s", "id"):
            a = getattr(self, name)
            a[p] = a[last]
            setattr(self, name, a[:-1].copy())

    def _flip_ratio(self, p):
        """Ratio of det N'^{-1} / det N^{-1} per spin when s_p -> -s_p.

        Only column p of N^{-1} = e^V - g (e^V - 1) changes, by
        d = (e^{V'_p} - e^{V_p}) (e_p - g_{.p}), so the ratio is
        1 + (N d)_p (matrix determinant lemma).  The unchanged column p of
        N^{-1} is e^{V_p} e_p - g_{.p} (e^{V_p} - 1), so N g_{.p} =
        (e^{V_p} N_{.p} - e_p) / (e^{V_p} - 1) and
            N d = c (e_p - N_{.p}),  c = (e^{V'_p} - e^{V_p}) / (e^{V_p} - 1),
        ratio 1 + c (1 - N_pp): the same quantity read off N itself, without
        the sum over k products of size e^{gamma} that N d would take."""
        m = self.m
        out = []
        for spin in range(2):
            ev_old = float(m.ev(self.s[p], spin))
            ev_new = float(m.ev(-self.s[p], spin))
            c = (ev_new - ev_old) / (ev_old - 1.0)
            Nd = -c * self.N[spin][:, p]
            Nd[p] += c
            out.append((1.0 + Nd[p], Nd))
        return out

    def _do_flip(self, p, parts):
        """Sherman-Morrison update of N for the column change d e_p^T."""
        for spin in range(2):
            ratio, Nd = parts[spin]
            N = self.N[spin]
            self.N[spin] = N - np.outer(Nd, N[p]) / ratio
        self.s[p] = -self.s[p]

    def step(self):
        """One proposal; returns (kind, accepted)."""
        m = self.m
        u = self.rng.random(5)
        self.n_prop += 1
        k = self.k
        half = 0.5 * (1.0 - self.p_flip)
        if u[0] >= 2.0 * half:
            # flip of the auxiliary spin of vertex floor(u1 k) (a no-op at k = 0)
            if k == 0:
                if self.record:
                    self.trace.append((2, -1, 0.0, 0, -1, u[4], 0.0, False))
                return 2, False
            p = int(math.floor(u[1] * k))
            parts = self._flip_ratio(p)
            R = parts[0][0] * parts[1][0]
            acc = u[4] < abs(R)
            tid = int(self.id[p])
            if acc:
                self.sign *= math.copysign(1.0, R)
                self._do_flip(p, parts)
                self.n_acc_flip += 1
            if self.record:
                self.trace.append((2, -1, 0.0, 0, tid, u[4], R, bool(acc)))
            return 2, acc
        if u[0] < half:
            rq = int(math.floor(u[1] * m.Nc))
            tq = u[2] * m.beta
            sq = 1 if u[3] < 0.5 else -1
            parts = self._insert_ratio(rq, tq, sq)
            R = m.K_exp / (k + 1) * parts[0][0] * parts[1][0]
            acc = u[4] < abs(R)
            new_id = -1
            if acc:
                self.sign *= math.copysign(1.0, R)
                new_id = self._do_insert(rq, tq, sq, parts)
                self.n_acc_ins += 1
            if self.record:
                self.trace.append((0, rq, tq, sq, new_id, u[4], R, bool(acc)))
            return 0, acc
        if k == 0:
            if self.record:
                self.trace.append((1, -1, 0.0, 0, -1, u[4], 0.0, False))
            return 1, False
        p = int(math.floor(u[1] * k))
        R = k / m.K_exp * self.N[0][p, p] * self.N[1][p, p]
        acc = u[4] < abs(R)
        tid = int(self.id[p])
        if acc:
            self.sign *= math.copysign(1.0, R)
            self._do_remove(p)
            self.n_acc_rem += 1
        if self.record:
            self.trace.append((1, -1, 0.0, 0, tid, u[4], R, bool(acc)))
        return 1, acc

    def sweep_length(self):
        """Proposals in the next sweep, a multiple of k_s.

        The length is frozen by freeze_sweep_length (after the warm-up); until
        then it is max(k, 1) for the current order k.  Measuring between
        sweeps whose length depends on the state would sample a distribution
        other than the weight (the order of the atom shifts visibly), so a
        measured chain uses a frozen length."""
        ks = self.k_s
        L = self.frozen_length if self.frozen_length else max(self.k, 1)
        return int(math.ceil(L / ks) * ks)

    def freeze_sweep_length(self, mean_order):
        """Fix the sweep length at the rounded mean order (at least 1)."""
        self.frozen_length = max(int(round(mean_order)), 1)

    def sweep(self):
        for _ in range(self.sweep_length()):
            self.step()

    def weight_sign(self):
        """Sign of prod_sigma det N_sigma^{-1} recomputed from scratch."""
        sgn = 1.0
        for spin in range(2):
            if self.k:
                sgn *= np.linalg.slogdet(n_inverse(self.m, self.r, self.t, self.s, spin))[0]
        return sgn

    def canonical(self):
        """(ids, N_up, N_dn) with vertices sorted by id."""
        o = np.argsort(self.id)
        return self.id[o], self.N[0][np.ix_(o, o)], self.N[1][np.ix_(o, o)]


TRACE_FIELDS = ("kind", "site", "tau", "aux_spin", "id", "u_accept", "ratio", "accepted")


def trace_arrays(trace):
    """Column arrays from a recorded trace.

    kind 0 insertion, 1 removal, 2 flip of an auxiliary spin; id is the new
    vertex's id for an accepted insertion and the target's id for a removal
    or a flip (-1 otherwise)."""
    if not trace:
        return {f: np.zeros(0) for f in TRACE_FIELDS}
    cols = list(zip(*trace))
    return {
        "kind": np.array(cols[0], np.uint8),
        "site": np.array(cols[1], np.int32),
        "tau": np.array(cols[2], np.float64),
        "aux_spin": np.array(cols[3], np.int8),
        "id": np.array(cols[4], np.int64),
        "u_accept": np.array(cols[5], np.float64),
        "ratio": np.array(cols[6], np.float64),
        "accepted": np.array(cols[7], np.uint8),
    }

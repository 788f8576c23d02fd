"""Two-particle Green's function of the cluster, particle-particle up-down
channel (Sec. 2.5, the Bethe-Salpeter equation's G_2; App. B, four-point
type PARTICLE_PARTICLE_UP_DOWN with a momentum and a frequency transfer).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For one CT-AUX configuration the two spins are independent quadratic
problems, so Wick's theorem gives the configuration's four-point function
of the up-down particle-particle channel as the product of its one-particle
functions (no exchange term between different spins):

  G2(k1, k2; q) = < c_{k1 up} c_{q-k1 down} c^+_{q-k2 down} c^+_{k2 up} >
                = G_up(k1, k2) G_down(q - k1, q - k2),

with k = (K, i w_n) and G_sigma(k1, k2) the configuration's Green's
function, which is not diagonal in k (translation invariance holds only on
average):

  M_sigma(k1, k2) = (1/Nc) sum_ij e^{i (w1 tau_i - K1 r_i)} [(e^V - 1) N]_ij
                                  e^{-i (w2 tau_j - K2 r_j)},
  G_sigma(k1, k2) = G0(k1) delta_{k1 k2} - G0(k1) M_sigma(k1, k2) G0(k2) / beta.

Its diagonal is the single-particle estimator of Sec. 2.3.  The Monte Carlo
estimate is sum_c s_c G2_c / sum_c s_c.

Grids (readings; the paper names the parameters only): the four-point
fermionic frequencies are w_n, n = -n_w4 .. n_w4 - 1 (App. B,
four-point-fermionic-frequencies = n_w4); a transfer q = (Q, i nu_m) is a
cluster momentum Q and a bosonic frequency nu_m = 2 pi m / beta, m >= 0, so
q - k = (Q - K, i w_{m-1-n}); the one-particle functions are needed on
n = -n_w4 .. n_w4 - 1 + m.  Momentum indices follow the cluster
enumeration (``geometry``); Q - K is reduced to the cluster's momenta.

Parity pins: at U = 0 (M = 0) G2 is G0(k1) G0(q - k1) delta_{k1 k2}
exactly; the diagonal of G_sigma(k1, k2) for n >= 0 equals the pinned
single-particle estimator of the same configuration (``measure``).  The
interacting G2 has no independent exact reference here: beyond those two
pins it is "parity unpinned".
"""
import numpy as np

from . import g0 as g0mod


def momentum_index_table(K):
    """d[a, b] = index of K_a - K_b reduced to the cluster momenta."""
    Nc = len(K)
    red = np.mod(K[:, None, :] - K[None, :, :], 2 * np.pi)
    out = np.empty((Nc, Nc), np.int64)
    for a in range(Nc):
        for b in range(Nc):
            dist = np.abs(np.angle(np.exp(1j * (K - red[a, b][None, :])))).sum(axis=1)
            out[a, b] = int(np.argmin(dist))
            if dist[out[a, b]] > 1e-9:
                raise AssertionError("momentum difference outside the cluster momenta")
    return out


class Grid:
    """The four-point grid: n_w4 fermionic frequencies per sign, transfer m."""

    def __init__(self, model, n_w4, m=0):
        if m < 0:
            raise ValueError("the bosonic transfer index is >= 0")
        self.m = model
        self.n_w4, self.w_m = n_w4, m
        self.n_lo = -n_w4
        self.nw = 2 * n_w4 + m                  # one-particle frequencies n_lo .. n_lo + nw - 1
        self.Nc = model.Nc

    def freqs(self):
        n = np.arange(self.n_lo, self.n_lo + self.nw)
        return n, (2 * n + 1) * np.pi / self.m.beta

    def G0(self, spin, g0_Kw=None):
        """G0(K, i w_n) on the one-particle grid, (Nc, nw): the isolated
        cluster's 1/(i w - xi_K), or from positive frequencies given by the
        caller (g0_Kw (Nc, >= n_w4 + m)) with G0(-i w) = conj G0(i w)."""
        n, w = self.freqs()
        if g0_Kw is None:
            xi = self.m.xis[spin]
            return 1.0 / (1j * w[None, :] - xi[:, None])
        out = np.empty((self.Nc, self.nw), complex)
        for c, nn in enumerate(n):
            out[:, c] = g0_Kw[:, nn] if nn >= 0 else np.conj(g0_Kw[:, -nn - 1])
        return out


def config_G(model, grid, walker, spin, g0_Kw=None):
    """G_sigma(k1, k2) of the walker's configuration, (Nc, nw, Nc, nw)."""
    from .measure import M_matrix
    n, w = grid.freqs()
    M = M_matrix(model, walker, spin)                               # (k, k) = (e^V - 1) N
    r = model.sites[walker.r].astype(float)                         # (k, 2)
    ph_t = np.exp(1j * np.outer(walker.t, w))                      # (k, nw): e^{i w tau_i}
    ph_K = np.exp(-1j * r @ model.K.T)                              # (k, Nc): e^{-i K r_i}
    E = (ph_K[:, :, None] * ph_t[:, None, :]).reshape(len(walker.t), -1)   # (k, Nc*nw)
    MK = (E.T @ M @ np.conj(E)) / model.Nc
    G0 = grid.G0(spin, g0_Kw).reshape(-1)
    G = -G0[:, None] * MK * G0[None, :] / model.beta
    G[np.diag_indices_from(G)] += G0
    return G.reshape(model.Nc, grid.nw, model.Nc, grid.nw)


def g2_pp_updown(grid, Gup, Gdn, qs):
    """G2(k1, k2; q) = G_up(k1, k2) G_down(q - k1, q - k2) for the transfers
    q = (Q, m) with Q in qs (momentum indices) and the grid's m; returns
    (len(qs), Nc, 2 n_w4, Nc, 2 n_w4)."""
    Nc, N, m = grid.Nc, grid.n_w4, grid.w_m
    dK = momentum_index_table(grid.m.K)
    out = np.empty((len(qs), Nc, 2 * N, Nc, 2 * N), complex)
    c = np.arange(2 * N)                    # column of n = n_lo + c in the one-particle grid
    nq = (m - 1 - (grid.n_lo + c)) - grid.n_lo      # column of m - 1 - n
    for iq, Q in enumerate(qs):
        kq = dK[Q]                           # Q - K for every K
        up = Gup[:, :2 * N][:, :, :, :2 * N]
        dn = Gdn[kq][:, nq][:, :, kq][:, :, :, nq]
        out[iq] = up * dn
    return out


class Accumulator2:
    """sum_c s_c G2_c and sum_c s_c over measured configurations."""

    def __init__(self, model, n_w4, m, qs, g0_Kw=None):
        self.m = model
        self.grid = Grid(model, n_w4, m)
        self.qs = list(qs)
        self.g0_Kw = g0_Kw
        self.sG2 = 0.0
        self.s = 0.0

    def measure(self, walker):
        Gs = [config_G(self.m, self.grid, walker, sp, None if self.g0_Kw is None else self.g0_Kw[sp])
              for sp in range(2)]
        self.sG2 = self.sG2 + walker.sign * g2_pp_updown(self.grid, Gs[0], Gs[1], self.qs)
        self.s += walker.sign

    def G2(self):
        return self.sG2 / self.s

"""Bare propagator of the isolated periodic cluster (Sec. 2.1 / 2.3).

In finite-size mode (App. B, "do-finite-size-QMC") the cluster solver's bare
propagator is that of the isolated periodic cluster,
G0(K, i w_n) = 1 / (i w_n - xi_K) with xi_K = eps_K - mu_B, where mu_B is the
chemical potential of H0 measured from the Hartree shift U/2 that Sec. 2.3
puts into H0.  Everything is in the standard convention
G(tau) = -<T c(tau) c^dagger(0)>.

The walker uses a tabulated real-space propagator G0(dr, tau_l) on n_tau
points tau_l = l * beta / (n_tau - 1), point 0 standing for 0+ and the last
point for beta-, interpolated linearly.
"""
import numpy as np


def g0_K_tau(xi, tau, beta):
    """G0(K, tau) = -e^{-xi tau} / (1 + e^{-beta xi}) for 0 < tau < beta.

    xi: (Nc,) ; tau: (T,) -> (Nc, T).  Overflow-safe for either sign of xi.
    """
    xi = np.asarray(xi, dtype=np.float64)[:, None]
    tau = np.asarray(tau, dtype=np.float64)[None, :]
    pos = -np.exp(-xi * tau) / (1.0 + np.exp(-beta * np.abs(xi)))
    neg = -np.exp(xi * (beta - tau)) / (np.exp(beta * xi) + 1.0)
    return np.where(xi >= 0, pos, neg)


def g0_K_iw(xi, n_freq, beta):
    """G0(K, i w_n) for n = 0 .. n_freq-1, shape (Nc, n_freq) complex."""
    w = (2 * np.arange(n_freq) + 1) * np.pi / beta
    return 1.0 / (1j * w[None, :] - np.asarray(xi)[:, None])


def g0_r_tau(sites, K, xi, tau, beta):
    """G0(dr, tau) = (1/Nc) sum_K e^{i K dr} G0(K, tau), indexed by site dr.

    Returns (Nc, T) real; the imaginary part vanishes for the inversion-
    symmetric clusters used here and is checked.
    """
    gk = g0_K_tau(xi, tau, beta)                      # (NcK, T)
    ph = np.exp(1j * np.asarray(sites, float) @ K.T)  # (Ncr, NcK)
    gr = ph @ gk / len(K)
    if np.max(np.abs(gr.imag)) > 1e-12 * max(1.0, np.max(np.abs(gr.real))):
        raise AssertionError("G0(r, tau) not real")
    return gr.real


def tau_grid(beta, n_tau):
    return np.linspace(0.0, beta, n_tau)


def g0_table(sites, K, xi, beta, n_tau):
    """Table T[dr, l] = G0(dr, tau_l); tau_0 = 0+ and tau_{n-1} = beta-."""
    t = tau_grid(beta, n_tau)
    # the analytic form is continuous on (0, beta); its limits at the two ends
    # are the one-sided values the table needs.
    return g0_r_tau(sites, K, xi, t, beta)


def interp(table, d, dtau, beta):
    """Linear interpolation of the table at (d, dtau), dtau in [0, beta].

    l = floor(dtau / h), f = dtau / h - l, value (1 - f) T[l] + f T[l + 1],
    with l clamped to n_tau - 2.  dtau == 0 gives the 0+ value.
    """
    n_tau = table.shape[1]
    h = beta / (n_tau - 1)
    x = np.asarray(dtau, dtype=np.float64) / h
    l = np.floor(x).astype(np.int64)
    l = np.clip(l, 0, n_tau - 2)
    f = x - l
    return (1.0 - f) * table[d, l] + f * table[d, l + 1]


class Propagator:
    """The walker's g = -G0 (positive convention) between vertices.

    g(i, j) = -G0(r_i - r_j, tau_i - tau_j) for tau_i >= tau_j (0+ at equal
    times, including the diagonal), and, by antiperiodicity,
    g(i, j) = +G0(r_i - r_j, tau_i - tau_j + beta) for tau_i < tau_j.
    """

    def __init__(self, diff, beta, table=None, analytic=None):
        self.diff = np.asarray(diff)
        self.beta = float(beta)
        self.table = table
        self.analytic = analytic   # callable (d, tau) -> G0 for exact checks

    def _G0(self, d, tau):
        if self.table is not None:
            return interp(self.table, d, tau, self.beta)
        return self.analytic(d, tau)

    def g(self, ri, ti, rj, tj):
        ri, rj = np.broadcast_arrays(np.asarray(ri), np.asarray(rj))
        ti, tj = np.broadcast_arrays(np.asarray(ti, float), np.asarray(tj, float))
        d = self.diff[ri, rj]
        dt = ti - tj
        neg = dt < 0
        dtw = np.where(neg, dt + self.beta, dt)
        val = self._G0(d, dtw)
        return np.where(neg, val, -val)

    def matrix(self, r, t):
        """Full k x k matrix g(i, j) for vertices (r, t)."""
        r = np.asarray(r)
        t = np.asarray(t, float)
        return self.g(r[:, None], t[:, None], r[None, :], t[None, :])

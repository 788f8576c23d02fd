"""The DCA self-consistency loop around the cluster solver (Sec. 2.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loop of Sec. 2.1 (the DCA loop figure and the equations around it):

* patches: the Brillouin zone is cut into Nc patches, one around each cluster
  momentum K, all of one shape (phi_K(k) = phi(k - K)) and inversion
  symmetric; the standard coarse-graining takes the Brillouin zone of the
  superlattice, i.e. the Wigner-Seitz cell of the reciprocal superlattice
  spanned by b1, b2 (a_i . b_j = 2 pi delta_ij);
* Sigma_DCA(k, i w_n) = Sigma_c(K, i w_n) on K's patch (piecewise constant);
* coarse-graining: Gbar(K, i w_n) = (Nc / V_BZ) int dk phi_K(k)
  [G0^{-1}(k, i w_n) - Sigma_DCA(k, i w_n)]^{-1}, the average over the patch,
  with G0(k, i w_n) = 1 / (i w_n - eps_k + mu);
* cluster exclusion: G0cal(K, i w_n) = [Gbar^{-1} + Sigma_c]^{-1}, the bare
  propagator of the effective cluster problem;
* the cluster solver turns G0cal into the cluster G_c(K, i w_n); Dyson's
  equation gives Sigma_QMC = G0cal^{-1} - G_c^{-1};
* mixing: Sigma_c^(n) = alpha Sigma_QMC + (1 - alpha) Sigma_c^(n-1).

Readings where the paper is silent (each a choice of this module, made the
same way by the library):

* quadrature of the patch average: L x L points u = ((i + 1/2)/L - 1/2) b1 +
  ((j + 1/2)/L - 1/2) b2, each moved by a reciprocal-superlattice vector to
  its image of least length (the Wigner-Seitz cell; among images of equal
  length within 1e-12, on the cell's boundary, each takes an equal share of
  the point's weight); the average is the weighted mean over the points.  For Nc = 1 the patch is the
  whole Brillouin zone and the rule is the trapezoidal rule of a periodic
  function;
* chemical potential and field: mu is measured from U/2 as for the walker
  (the Hartree shift sits in H0), and a Zeeman field h enters as
  eps_k - mu - sigma h (sigma = +1 up, -1 down);
* Sigma beyond the measured frequencies: the coarse-graining runs over
  n_cg >= n_freq positive frequencies (the transform to tau needs many);
  for n >= n_freq, Sigma keeps the real part of its last measured value and
  its imaginary part falls as 1/w_n from there:
  Sigma(i w_n) = Re Sigma_last + i Im Sigma_last w_last / w_n;
* G0cal(K, tau) = (1/beta) sum_n e^{-i w_n tau} G0cal(K, i w_n) over all n
  (G0cal(-i w) is the conjugate): the sum over n < n_cg of
  (2/beta) Re[e^{-i w_n tau} R(i w_n)], R = G0cal - 1/(i w) - c2/(i w)^2 -
  c3/(i w)^3, plus the closed forms of the three tail terms, -1/2,
  c2 (2 tau - beta)/4 and c3 tau (beta - tau)/4.  The moments are exact:
  expanding Gbar = <1/(z - eps)>_patch in 1/z gives Gbar^{-1} = z - epsbar_K
  - var_K / z + O(z^-2) (var_K the patch variance of eps), and Sigma cancels
  in G0cal^{-1} = Gbar^{-1} + Sigma up to O(1/w^2), so c2 = epsbar_K - mu -
  sigma h and c3 = c2^2 + var_K.  Phases use the exact reduction of
  w_n tau_l = pi (2n+1) l / (n_tau - 1) modulo 2 pi.
* the table the walker takes: G0cal(r_d, tau_l) = (1/Nc) sum_K e^{i K r_d}
  G0cal(K, tau_l) (real), tau_l = l beta / (n_tau - 1), point 0 the 0+ value
  and the last the beta- value, in the standard convention.
"""
import math

import numpy as np

from . import geometry


def reciprocal_superlattice(a1, a2):
    """b1, b2 with a_i . b_j = 2 pi delta_ij, as rows of a (2, 2) array."""
    A = np.array([a1, a2], dtype=np.float64)          # rows a1, a2
    return 2.0 * np.pi * np.linalg.inv(A).T


def patch_points(a1, a2, L):
    """The quadrature of the standard patch around K = 0: offsets k~ (P, 2)
    and weights (P,) summing to L^2.  A grid point with several images of
    least length (on the cell's boundary) contributes each of them with an
    equal share of its weight, so the rule stays inversion symmetric."""
    B = reciprocal_superlattice(a1, a2)
    f = (np.arange(L) + 0.5) / L - 0.5
    pts, wts = [], []
    for j in range(L):
        for i in range(L):
            u = f[i] * B[0] + f[j] * B[1]
            imgs = [u + n1 * B[0] + n2 * B[1] for n1 in range(-2, 3) for n2 in range(-2, 3)]
            norms = np.array([float(v @ v) for v in imgs])
            best = [v for v, nv in zip(imgs, norms) if nv <= norms.min() + 1e-12]
            for v in best:
                pts.append(v)
                wts.append(1.0 / len(best))
    return np.array(pts), np.array(wts)


class DCA:
    """The steps of one DCA iteration around a cluster solver, in float64."""

    def __init__(self, a1, a2, t=1.0, tp=0.0, beta=5.0, mu=0.0, h=0.0, n_freq=64, n_cg=2048, n_tau=1000, L=8):
        self.a1, self.a2 = tuple(a1), tuple(a2)
        self.t, self.tp, self.beta, self.mu, self.h = t, tp, beta, mu, h
        self.n_freq, self.n_cg, self.n_tau, self.L = n_freq, n_cg, n_tau, L
        if n_cg < n_freq:
            raise ValueError("n_cg < n_freq")
        self.sites = geometry.cluster_sites(self.a1, self.a2)
        self.K = geometry.cluster_momenta(self.a1, self.a2)
        self.Nc = len(self.K)
        self.kt, self.wt = patch_points(self.a1, self.a2, L)                  # (P, 2), (P,)
        kk = self.K[:, None, :] + self.kt[None, :, :]                          # (Nc, P, 2)
        self.eps = geometry.dispersion(kk.reshape(-1, 2), t, tp).reshape(self.Nc, -1)
        self.epsbar = self.eps @ self.wt / (L * L)
        self.epsvar = (self.eps - self.epsbar[:, None]) ** 2 @ self.wt / (L * L)
        self.w = (2 * np.arange(n_cg) + 1) * np.pi / beta

    def spin_shift(self, spin):
        """The field's shift of the chemical potential for spin 0 (up) or 1."""
        return self.h if spin == 0 else -self.h

    def extend_sigma(self, sigma):
        """Sigma (Nc, n_freq) -> (Nc, n_cg) with the high-frequency rule above."""
        sigma = np.asarray(sigma, complex)
        out = np.empty((self.Nc, self.n_cg), complex)
        nf = self.n_freq
        out[:, :nf] = sigma
        if self.n_cg > nf:
            last = sigma[:, nf - 1]
            wl = self.w[nf - 1]
            out[:, nf:] = last.real[:, None] + 1j * last.imag[:, None] * wl / self.w[None, nf:]
        return out

    def coarse_grain(self, sigma, spin=0):
        """(Gbar, G0cal), each (Nc, n_cg) complex, from Sigma_c (Nc, n_freq)."""
        s = self.extend_sigma(sigma)
        z = 1j * self.w[None, :] + self.mu + self.spin_shift(spin) - s      # (Nc, n_cg)
        gbar = np.einsum("p,kpn->kn", self.wt, 1.0 / (z[:, None, :] - self.eps[:, :, None])) / (self.L * self.L)
        g0 = 1.0 / (1.0 / gbar + s)
        return gbar, g0

    def g0_K_tau(self, g0, spin=0):
        """G0cal(K, tau_l) on the table grid, (Nc, n_tau), from (Nc, n_cg)."""
        n_tau, beta = self.n_tau, self.beta
        l = np.arange(n_tau)
        tau = l * beta / (n_tau - 1)
        iw = 1j * self.w
        c2 = self.epsbar - self.mu - self.spin_shift(spin)                    # (Nc,)
        c3 = c2 ** 2 + self.epsvar
        R = g0 - 1.0 / iw[None, :] - c2[:, None] / iw[None, :] ** 2 - c3[:, None] / iw[None, :] ** 3
        n = np.arange(self.n_cg)
        # w_n tau_l = pi (2n+1) l / (n_tau - 1), reduced modulo 2 pi exactly
        red = np.outer(2 * n + 1, l) % (2 * (n_tau - 1))
        ph = np.exp(-1j * np.pi * red / (n_tau - 1))                           # (n_cg, n_tau)
        out = (2.0 / beta) * (R @ ph).real
        out += -0.5 + c2[:, None] * (2 * tau[None, :] - beta) / 4.0 + c3[:, None] * tau * (beta - tau) / 4.0
        return out

    def g0_table(self, g0, spin=0):
        """The walker's table G0cal(r_d, tau_l), (Nc, n_tau), real."""
        gk = self.g0_K_tau(g0, spin)
        ph = np.exp(1j * self.sites.astype(float) @ self.K.T)                 # (Nc r, Nc K)
        gr = ph @ gk / self.Nc
        if np.max(np.abs(gr.imag)) > 1e-10 * max(1.0, np.max(np.abs(gr.real))):
            raise AssertionError("G0cal(r, tau) not real")
        return gr.real

    @staticmethod
    def self_energy(g0, G, sigma_old, alpha):
        """Dyson's equation and mixing on the measured frequencies:
        alpha (G0cal^{-1} - G^{-1}) + (1 - alpha) Sigma_old."""
        nf = G.shape[-1]
        s_qmc = 1.0 / g0[..., :nf] - 1.0 / G
        return alpha * s_qmc + (1.0 - alpha) * sigma_old


def finalize_G_iw(g0, M_avg, beta):
    """G_c(K, i w_n) = G0cal - G0cal <M> G0cal / beta (Sec. 2.3's estimator
    with the cluster-excluded propagator), M_avg (Nc, n_freq)."""
    nf = M_avg.shape[-1]
    g = g0[..., :nf]
    return g - g * M_avg * g / beta


def dca_loop(dca, U, iterations, sweeps, warmup, seed, alpha=1.0, k_s=16, K_exp=1.0, sigma0=None):
    """The plain loop with the oracle's single-vertex chain as the solver
    (slow; small clusters and orders only).  Returns the list of Sigma_c
    iterates, each (2 spins, Nc, n_freq), and the last (G_c, sign)."""
    from . import ctaux, measure
    nf = dca.n_freq
    sig = np.zeros((2, dca.Nc, nf), complex) if sigma0 is None else np.array(sigma0, complex)
    out = [sig.copy()]
    last = None
    for it in range(iterations):
        g0s = [dca.coarse_grain(sig[sp], sp)[1] for sp in range(2)]
        tables = [dca.g0_table(g0s[sp], sp) for sp in range(2)]
        m = ctaux.Model(a1=dca.a1, a2=dca.a2, t=dca.t, tp=dca.tp, U=U, beta=dca.beta, mu=dca.mu, h=dca.h,
                        K_exp=K_exp, n_tau=dca.n_tau, tables=tables)
        w = ctaux.Walker(m, seed=seed + it, k_s=k_s)
        for _ in range(warmup):
            w.sweep()
        acc = measure.Accumulator(m, nf)
        for _ in range(sweeps):
            w.sweep()
            acc.measure(w)
        s, sM, _ = acc.arrays()
        Mavg = sM.sum(axis=0) / s.sum()                                    # (2, Nc, nf)
        G = np.array([finalize_G_iw(g0s[sp], Mavg[sp], dca.beta) for sp in range(2)])
        if dca.h == 0.0:
            G[:] = G.mean(axis=0)
        sig = np.array([DCA.self_energy(g0s[sp], G[sp], sig[sp], alpha) for sp in range(2)])
        out.append(sig.copy())
        last = (G, s.mean())
    return out, last

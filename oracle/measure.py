"""Green's-function measurement from the walker's N matrices (Sec. 2.3).

Per configuration and spin, M = (e^V - 1) N and its Fourier coefficients

    M(K, i w_n) = (1/Nc) sum_{ij} e^{i (w_n tau_i - K r_i)} M_ij e^{-i (w_n tau_j - K r_j)}

are accumulated with the configuration's sign.  The Green's function estimator
of Sec. 2.3 is then G(K, i w_n) = G0 - (1/beta) G0 <M> G0 with
<M> = sum sign M / sum sign; G0 is diagonal in K for the isolated cluster.

The transform is the plain non-uniform DFT: no NFFT gridding (the paper's
delayed-NFFT of Sec. 2.3 is an acceleration of exactly this sum).
"""
import numpy as np


def matsubara(n_freq, beta):
    return (2 * np.arange(n_freq) + 1) * np.pi / beta


def M_matrix(model, walker, spin):
    ev = model.ev(walker.s, spin)
    return (ev - 1.0)[:, None] * walker.N[spin]


def M_K_iw(model, r, t, M, n_freq, freqs=None, Ks=None):
    """M(K, i w_n) for one spin, shape (Nc, n_freq) complex, by direct sums.

    freqs / Ks (optional index arrays) restrict the sums to those Matsubara
    indices n and momentum indices: the result is then (len(Ks), len(freqs)),
    each entry the same direct sum (sampled outputs at large orders)."""
    n_idx = np.arange(n_freq) if freqs is None else np.asarray(freqs, np.int64)
    K_idx = np.arange(model.Nc) if Ks is None else np.asarray(Ks, np.int64)
    w = (2 * n_idx + 1) * np.pi / model.beta
    out = np.zeros((len(K_idx), len(n_idx)), dtype=complex)
    if len(r) == 0:
        return out
    pos = model.sites[np.asarray(r)].astype(np.float64)        # (k, 2)
    for o, iK in enumerate(K_idx):
        K = model.K[iK]
        phi = np.exp(1j * (np.outer(t, w) - (pos @ K)[:, None]))   # (k, n)
        out[o] = np.sum(phi * (M @ phi.conj()), axis=0) / model.Nc
    return out


class Accumulator:
    """sum sign * M(K, i w_n) per spin and sum sign, binned for error bars."""

    def __init__(self, model, n_freq):
        self.m = model
        self.n_freq = n_freq
        self.samples = []     # list of (sign, M[2, Nc, n_freq], Mdiag[2])

    def measure(self, walker):
        Ms = np.zeros((2, self.m.Nc, self.n_freq), dtype=complex)
        diag = np.zeros(2)
        for spin in range(2):
            M = M_matrix(self.m, walker, spin)
            Ms[spin] = M_K_iw(self.m, walker.r, walker.t, M, self.n_freq)
            diag[spin] = np.trace(M) / self.m.Nc if walker.k else 0.0
        self.samples.append((walker.sign, walker.sign * Ms, walker.sign * diag))

    def arrays(self):
        s = np.array([x[0] for x in self.samples])
        sM = np.array([x[1] for x in self.samples])
        sD = np.array([x[2] for x in self.samples])
        return s, sM, sD


def finalize_G_iw(model, M_avg, n_freq, spin=0):
    """G(K, i w_n) = G0 - (1/beta) G0 <M> G0 for one spin; M_avg (Nc, n_freq)."""
    from .g0 import g0_K_iw
    G0 = g0_K_iw(model.xis[spin], n_freq, model.beta)
    return G0 - G0 * M_avg * G0 / model.beta


def G_tau_from_iw(model, M_avg, Mdiag_avg, n_freq, taus, spin=0):
    """G(K, tau) from the frequency estimator with the 1/(i w)^2 tail removed.

    dG = G - G0 behaves as A / (i w)^2 with A = -(1/beta) <(1/Nc) sum_i M_ii>;
    dG(tau) = (2/beta) Re sum_{n>=0} e^{-i w_n tau} [dG(i w_n) - A/(i w_n)^2]
    + A (2 tau - beta) / 4, the last term being the exact transform of the tail.
    """
    from .g0 import g0_K_iw, g0_K_tau
    beta = model.beta
    w = matsubara(n_freq, beta)
    xi = model.xis[spin]
    G0w = g0_K_iw(xi, n_freq, beta)
    dG = -G0w * M_avg * G0w / beta                       # (Nc, n_freq)
    A = -Mdiag_avg / beta
    resid = dG - A / (1j * w[None, :]) ** 2
    taus = np.asarray(taus, float)
    ph = np.exp(-1j * np.outer(w, taus))                 # (n_freq, T)
    dGt = (2.0 / beta) * (resid @ ph).real + A * (2 * taus[None, :] - beta) / 4.0
    return g0_K_tau(xi, taus, beta) + dGt

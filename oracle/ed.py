"""Exact diagonalisation of small Hubbard clusters (test oracle).

The paper validates its QMC solvers against an exact-diagonalisation solver on
small clusters (Sec. 3.1 lists ED among the cluster solvers; App. A, the
cluster_solver_check application).  This module rebuilds that check for the
single-band Hubbard model

    H = sum_{ij,s} t_ij c+_{is} c_{js} - mu_B N + U sum_i (n_iu - 1/2)(n_id - 1/2)

(Sec. 2.3's H0 + H_int up to a constant, with mu_B the chemical potential
measured from the Hartree shift).  Fock states are bit strings over 2 Nc
spin-orbitals, orbital index 2 i + s (s = 0 up, 1 down); fermion signs follow
that ordering.
"""
import numpy as np


def _annihilate(state, orb):
    """c_orb |state> -> (sign, new_state) or (0, None)."""
    if not (state >> orb) & 1:
        return 0, None
    sign = -1 if bin(state & ((1 << orb) - 1)).count("1") % 2 else 1
    return sign, state ^ (1 << orb)


def _create(state, orb):
    if (state >> orb) & 1:
        return 0, None
    sign = -1 if bin(state & ((1 << orb) - 1)).count("1") % 2 else 1
    return sign, state | (1 << orb)


def hamiltonian(tij, U, mu, h=0.0):
    """Dense many-body Hamiltonian on all 4^Nc Fock states; h is a Zeeman
    field, -h sum_i (n_iup - n_idown)."""
    Nc = tij.shape[0]
    n_orb = 2 * Nc
    dim = 1 << n_orb
    H = np.zeros((dim, dim))
    for st in range(dim):
        occ = [(st >> o) & 1 for o in range(n_orb)]
        diag = 0.0
        for i in range(Nc):
            nu, nd = occ[2 * i], occ[2 * i + 1]
            diag += U * (nu - 0.5) * (nd - 0.5) - mu * (nu + nd) - h * (nu - nd)
        H[st, st] += diag
        for s in range(2):
            for i in range(Nc):
                for j in range(Nc):
                    if tij[i, j] == 0.0:
                        continue
                    s1, st1 = _annihilate(st, 2 * j + s)
                    if not s1:
                        continue
                    s2, st2 = _create(st1, 2 * i + s)
                    if not s2:
                        continue
                    H[st2, st] += tij[i, j] * s1 * s2
    return H


def annihilator(Nc, orb):
    dim = 1 << (2 * Nc)
    C = np.zeros((dim, dim))
    for st in range(dim):
        s, new = _annihilate(st, orb)
        if s:
            C[new, st] = s
    return C


class ED:
    """Eigen-decomposition plus single-particle Green's functions."""

    def __init__(self, tij, U, mu, beta, h=0.0):
        self.Nc = tij.shape[0]
        self.beta = beta
        H = hamiltonian(tij, U, mu, h)
        E, V = np.linalg.eigh(H)
        self.E0 = E[0]
        self.E = E - E[0]
        self.V = V
        self.w = np.exp(-beta * self.E)
        self.Z = self.w.sum()

    def expect(self, op):
        """Thermal expectation of a many-body operator (dense matrix)."""
        d = np.einsum("ia,ij,ja->a", self.V, op, self.V)
        return float((self.w * d).sum() / self.Z)

    def _c_eig(self, phases, spin):
        """<m| c_K |n> in the eigenbasis for c_K = sum_r phases[r] c_{r,spin}."""
        C = np.zeros((1 << (2 * self.Nc),) * 2, dtype=complex)
        for r in range(self.Nc):
            C += phases[r] * annihilator(self.Nc, 2 * r + spin)
        return self.V.T @ C @ self.V

    def G_tau(self, phases, spin, tau):
        """G(tau) = -<c(tau) c+(0)> for c = sum_r phases[r] c_r, 0 < tau < beta."""
        A = np.abs(self._c_eig(phases, spin)) ** 2          # |<m|c|n>|^2
        tau = np.atleast_1d(np.asarray(tau, float))
        Em, En = self.E[:, None], self.E[None, :]
        out = np.empty(len(tau))
        for n, t in enumerate(tau):
            out[n] = -(A * np.exp(-(self.beta - t) * Em - t * En)).sum() / self.Z
        return out

    def G_iw(self, phases, spin, n_freq):
        """G(i w_n), n = 0..n_freq-1, same operator convention as G_tau."""
        A = np.abs(self._c_eig(phases, spin)) ** 2
        w = (2 * np.arange(n_freq) + 1) * np.pi / self.beta
        Em, En = self.E[:, None], self.E[None, :]
        num = A * (self.w[:, None] + self.w[None, :])
        mask = num > 0
        numv, dE = num[mask], (Em - En)[mask]
        return np.array([(numv / (1j * wn + dE)).sum() / self.Z for wn in w])


def momentum_phases(sites, K):
    """phases[K_index, r] such that c_K = sum_r phases[r] c_r = Nc^{-1/2} sum_r e^{-iK r} c_r."""
    Nc = len(sites)
    return np.exp(-1j * K @ np.asarray(sites, float).T) / np.sqrt(Nc)

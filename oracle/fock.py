"""Brute-force Fock-space trace of a time-ordered product (test oracle).

Sec. 2.3 writes the weight of a CT-AUX configuration as a trace over
e^{-dtau H0} factors interleaved with exponentials of densities, Z_k, and
states that it equals Z_0 times a product of determinants of N^{-1}.  For one
spin species of spinless fermions on L sites with H0 = c+ h c this module
evaluates

    < T prod_i exp(V_i n_{r_i}(tau_i)) >_0
        = Tr[ e^{-(beta - tau_k) H0} e^{V_k n_{r_k}} ... e^{V_1 n_{r_1}} e^{-tau_1 H0} ] / Z_0

literally, in the 2^L-dimensional Fock space, with times sorted so that later
times stand to the left.  It also gives the single-particle propagator
g(tau) = <T c(tau) c+(0)>_0 from h alone (no many-body algebra), which the
determinant formula consumes.
"""
import numpy as np


def _number_ops(L):
    dim = 1 << L
    occ = np.array([[(s >> r) & 1 for r in range(L)] for s in range(dim)], dtype=np.float64)
    return occ  # (dim, L)


def many_body_h0(h):
    L = h.shape[0]
    dim = 1 << L
    H = np.zeros((dim, dim))
    for st in range(dim):
        for i in range(L):
            for j in range(L):
                if h[i, j] == 0.0:
                    continue
                if not (st >> j) & 1:
                    continue
                s1 = -1 if bin(st & ((1 << j) - 1)).count("1") % 2 else 1
                st1 = st ^ (1 << j)
                if (st1 >> i) & 1:
                    continue
                s2 = -1 if bin(st1 & ((1 << i) - 1)).count("1") % 2 else 1
                H[st1 | (1 << i), st] += h[i, j] * s1 * s2
    return H


def _expm_sym(H, t):
    E, V = np.linalg.eigh(H)
    return (V * np.exp(-t * E)) @ V.T


def time_ordered_trace(h, beta, sites, taus, V):
    """<T prod_i exp(V_i n_{sites_i}(taus_i))>_0 by explicit Fock-space products."""
    L = h.shape[0]
    H = many_body_h0(h)
    occ = _number_ops(L)
    order = np.argsort(taus)              # earliest first
    P = _expm_sym(H, taus[order[0]]) if len(order) else _expm_sym(H, beta)
    prev = taus[order[0]] if len(order) else beta
    for n, idx in enumerate(order):
        P = np.diag(np.exp(V[idx] * occ[:, sites[idx]])) @ P
        nxt = taus[order[n + 1]] if n + 1 < len(order) else beta
        P = _expm_sym(H, nxt - prev) @ P
        prev = nxt
    Z0 = np.trace(_expm_sym(H, beta))
    return np.trace(P) / Z0


def single_particle_g(h, beta, ri, ti, rj, tj):
    """g = <T c_{ri}(ti) c+_{rj}(tj)>_0 from the one-body h (0+ at equal times)."""
    e, U = np.linalg.eigh(h)
    f = 1.0 / (1.0 + np.exp(beta * e))
    dt = ti - tj
    if dt >= 0:
        m = (U * (np.exp(-dt * e) * (1.0 - f))) @ U.T
        return m[ri, rj]
    m = (U * (np.exp(-dt * e) * f)) @ U.T
    return -m[ri, rj]

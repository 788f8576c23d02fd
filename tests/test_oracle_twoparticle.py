"""Pins of the two-particle measurement in the oracle (oracle/twoparticle.py).

* at U = 0 every vertex leaves V = 0, M = 0, and the particle-particle
  up-down G2 is exactly G0(k1) G0(q - k1) delta_{k1 k2}, for momentum and
  frequency transfers;
* the diagonal of a configuration's G_sigma(k1, k2) at n >= 0 equals the
  single-particle estimator G0 - G0 M(K, i w_n) G0 / beta of the same
  configuration (measure.M_K_iw, pinned by brute force);
* G0 at negative frequencies from positive ones (conjugation) equals the
  closed form 1/(i w - xi) there;
* momentum differences reduce to cluster momenta (K_{d(a,b)} + K_b = K_a).
"""
import numpy as np
import pytest

from oracle import ctaux, g0, measure, twoparticle


def _walker(U, k, seed=4):
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=U, beta=4.0, mu=0.2, n_tau=400)
    w = ctaux.Walker(m, seed=seed, k_s=8)
    w.random_config(k)
    return m, w


@pytest.mark.parametrize("wm", [0, 2])
def test_u0_g2_is_the_product_of_bare_propagators(wm):
    m, w = _walker(0.0, 6)
    grid = twoparticle.Grid(m, 4, wm)
    Gs = [twoparticle.config_G(m, grid, w, sp) for sp in range(2)]
    qs = [0, 3]
    G2 = twoparticle.g2_pp_updown(grid, Gs[0], Gs[1], qs)
    n = np.arange(-4, 4)
    w_n = (2 * n + 1) * np.pi / m.beta
    dK = twoparticle.momentum_index_table(m.K)
    for iq, Q in enumerate(qs):
        want = np.zeros_like(G2[iq])
        for K in range(m.Nc):
            for c, nn in enumerate(n):
                nq = wm - 1 - nn
                wq = (2 * nq + 1) * np.pi / m.beta
                want[K, c, K, c] = 1.0 / (1j * w_n[c] - m.xi[K]) / (1j * wq - m.xi[dK[Q, K]])
        assert np.max(np.abs(G2[iq] - want)) < 1e-14


def test_diagonal_is_the_single_particle_estimator():
    m, w = _walker(4.0, 12)
    grid = twoparticle.Grid(m, 6, 1)
    for sp in range(2):
        G = twoparticle.config_G(m, grid, w, sp)
        M = measure.M_matrix(m, w, sp)
        nf = 6
        Mk = measure.M_K_iw(m, w.r, w.t, M, nf)
        G0 = g0.g0_K_iw(m.xis[sp], nf, m.beta)
        want = G0 - G0 * Mk * G0 / m.beta
        got = np.array([[G[K, 6 + n, K, 6 + n] for n in range(nf)] for K in range(m.Nc)])
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
        # and the configuration's G is not diagonal in K (no translation invariance per configuration)
        assert np.max(np.abs(G[0, :, 1, :])) > 1e-3


def test_negative_frequencies_from_positive_ones():
    m, _ = _walker(4.0, 2)
    grid = twoparticle.Grid(m, 5, 3)
    gkw = g0.g0_K_iw(m.xi, 8, m.beta)
    assert np.max(np.abs(grid.G0(0, gkw) - grid.G0(0))) < 1e-15


def test_momentum_differences():
    for a1, a2 in (((2, 0), (0, 2)), ((4, 0), (0, 4)), ((2, 2), (2, -2))):
        m = ctaux.Model(a1=a1, a2=a2, U=1.0, beta=1.0, n_tau=10)
        d = twoparticle.momentum_index_table(m.K)
        back = np.mod(m.K[d] + m.K[None, :, :] - m.K[:, None, :] + 1e-12, 2 * np.pi)
        assert np.max(np.minimum(back, 2 * np.pi - back)) < 1e-9

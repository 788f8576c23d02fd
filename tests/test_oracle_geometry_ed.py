"""Pins for the oracle's cluster geometry and exact diagonalisation.

Everything here is checked against closed forms: lattice counting, nearest-
neighbour hopping, the free propagator, the Hubbard atom and the Hubbard
dimer's ground-state energy.
"""
import numpy as np
import pytest

from oracle import geometry, ed, g0


@pytest.mark.parametrize("a1,a2,nc", [((2, 0), (0, 2), 4), ((4, 0), (0, 4), 16),
                                      ((2, 2), (2, -2), 8), ((6, 0), (0, 6), 36),
                                      ((8, 0), (0, 8), 64), ((1, 0), (0, 1), 1)])
def test_counts_and_group_table(a1, a2, nc):
    s = geometry.cluster_sites(a1, a2)
    K = geometry.cluster_momenta(a1, a2)
    assert len(s) == nc and len(K) == nc
    d = geometry.diff_table(a1, a2)
    origin = [i for i, p in enumerate(s) if tuple(p) == (0, 0)][0]
    assert np.all(np.diag(d) == origin)
    for i in range(nc):                      # each row is a permutation
        assert sorted(d[i]) == list(range(nc))
    # K . a in 2 pi Z, and the characters are orthogonal over the sites
    for k in K:
        for a in (a1, a2):
            x = (k[0] * a[0] + k[1] * a[1]) / (2 * np.pi)
            assert abs(x - round(x)) < 1e-12
    ph = np.exp(1j * s.astype(float) @ K.T)
    assert np.allclose(ph.conj().T @ ph, nc * np.eye(nc))


def test_2x2_order():
    s = geometry.cluster_sites((2, 0), (0, 2))
    assert [tuple(p) for p in s] == [(0, 0), (1, 0), (0, 1), (1, 1)]
    K = geometry.cluster_momenta((2, 0), (0, 2))
    assert np.allclose(K, np.pi * np.array([[0, 0], [1, 0], [0, 1], [1, 1]]))


def test_hopping_nearest_neighbour():
    # 4x4: t_ij = -t for nearest neighbours, -t' for diagonal neighbours
    t = geometry.hopping_matrix((4, 0), (0, 4), t=1.0, tp=-0.15)
    s = geometry.cluster_sites((4, 0), (0, 4))
    for i in range(16):
        for j in range(16):
            dx = (s[i][0] - s[j][0]) % 4
            dy = (s[i][1] - s[j][1]) % 4
            dx, dy = min(dx, 4 - dx), min(dy, 4 - dy)
            want = -1.0 if dx + dy == 1 else (0.15 if (dx, dy) == (1, 1) else 0.0)
            assert abs(t[i, j] - want) < 1e-12
    # 2x2: a bond wraps onto itself and is counted twice
    t2 = geometry.hopping_matrix((2, 0), (0, 2))
    assert abs(t2[0, 1] + 2.0) < 1e-12 and abs(t2[0, 3]) < 1e-12


def test_ed_free_limit_matches_closed_form():
    a1, a2 = (2, 0), (0, 2)
    tij = geometry.hopping_matrix(a1, a2)
    mu, beta = 0.3, 2.0
    e = ed.ED(tij, U=0.0, mu=mu, beta=beta)
    s = geometry.cluster_sites(a1, a2)
    K = geometry.cluster_momenta(a1, a2)
    ph = ed.momentum_phases(s, K)
    xi = geometry.dispersion(K) - mu
    gw = g0.g0_K_iw(xi, 8, beta)
    taus = np.array([0.1, 0.7, 1.5])
    gt = g0.g0_K_tau(xi, taus, beta)
    for iK in range(4):
        assert np.allclose(e.G_iw(ph[iK], 0, 8), gw[iK], atol=1e-12)
        assert np.allclose(e.G_tau(ph[iK], 1, taus), gt[iK], atol=1e-12)


def test_ed_hubbard_atom():
    U, beta = 3.0, 4.0
    e = ed.ED(np.zeros((1, 1)), U=U, mu=0.0, beta=beta)
    taus = np.linspace(0.05, beta - 0.05, 7)
    want = -np.cosh(U * (beta / 2 - taus) / 2) / (2 * np.cosh(beta * U / 4))
    assert np.allclose(e.G_tau(np.array([1.0]), 0, taus), want, atol=1e-13)
    w = (2 * np.arange(6) + 1) * np.pi / beta
    assert np.allclose(e.G_iw(np.array([1.0]), 1, 6), 1j * w / ((1j * w) ** 2 - U * U / 4), atol=1e-13)


def test_ed_dimer_ground_state():
    # two sites, H = -t sum (c+c + h.c.) + U sum n_u n_d: E0(N=2) = (U - sqrt(U^2 + 16 t^2)) / 2
    t, U = 1.0, 2.5
    tij = np.array([[0.0, -t], [-t, 0.0]])
    H = ed.hamiltonian(tij, U, 0.0)
    # U (n_u - 1/2)(n_d - 1/2) = U n_u n_d - U/2 (n_u + n_d) + U/4 per site
    dim = H.shape[0]
    N = np.array([bin(st).count("1") for st in range(dim)])
    idx = np.where(N == 2)[0]
    E = np.linalg.eigvalsh(H[np.ix_(idx, idx)])
    E_std = E[0] + U / 2 * 2 - 2 * U / 4
    assert abs(E_std - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_atom_in_a_field_closed_form():
    """Hubbard atom with a Zeeman field, H = U (n_u - 1/2)(n_d - 1/2)
    - mu (n_u + n_d) - h (n_u - n_d): four states E_0 = U/4,
    E_up = -U/4 - mu - h, E_dn = -U/4 - mu + h, E_2 = U/4 - 2 mu, and
    G_s(i w) = [(e^{-b E_0} + e^{-b E_s}) / (i w + E_0 - E_s)
               + (e^{-b E_sbar} + e^{-b E_2}) / (i w + E_sbar - E_2)] / Z."""
    U, mu, h, beta = 4.0, 0.3, 0.5, 5.0
    e = ed.ED(np.zeros((1, 1)), U=U, mu=mu, beta=beta, h=h)
    E = {"0": U / 4, "u": -U / 4 - mu - h, "d": -U / 4 - mu + h, "2": U / 4 - 2 * mu}
    Z = sum(np.exp(-beta * x) for x in E.values())
    wn = (2 * np.arange(20) + 1) * np.pi / beta
    for spin, (s, sb) in enumerate((("u", "d"), ("d", "u"))):
        want = ((np.exp(-beta * E["0"]) + np.exp(-beta * E[s])) / (1j * wn + E["0"] - E[s])
                + (np.exp(-beta * E[sb]) + np.exp(-beta * E["2"])) / (1j * wn + E[sb] - E["2"])) / Z
        assert np.allclose(e.G_iw(np.array([1.0]), spin, 20), want, atol=1e-13)
    # the field splits the spins: G_up != G_down
    assert np.max(np.abs(e.G_iw(np.array([1.0]), 0, 20) - e.G_iw(np.array([1.0]), 1, 20))) > 1e-2

"""Brute-force Fock-space pins of the CT-AUX conventions (Sec. 2.3).

* the configuration weight Z_k / Z_0 per spin equals det N^{-1} with
  N^{-1} = e^V - g (e^V - 1) and g = <T c c+>_0 taken at 0+ on the diagonal;
* the Green's function of a configuration is g + g M g with M = (e^V - 1) N;
* the oracle's propagator (table and analytic) is that g.
"""
import numpy as np
import pytest

from oracle import fock, geometry, ctaux


def _g_matrix(h, beta, r, t):
    k = len(r)
    return np.array([[fock.single_particle_g(h, beta, r[i], t[i], r[j], t[j])
                      for j in range(k)] for i in range(k)])


@pytest.mark.parametrize("L,k,seed", [(2, 1, 0), (2, 2, 1), (2, 4, 2), (3, 3, 3), (3, 4, 4), (1, 3, 5)])
def test_determinant_equals_fock_trace(L, k, seed):
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(L, L))
    h = 0.5 * (h + h.T)
    beta = 2.0
    r = rng.integers(0, L, size=k)
    t = rng.random(k) * beta
    V = rng.normal(size=k) * 1.3
    brute = fock.time_ordered_trace(h, beta, r, t, V)
    g = _g_matrix(h, beta, r, t)
    ev = np.exp(V)
    Ninv = np.diag(ev) - g * (ev - 1.0)[None, :]
    assert abs(np.linalg.det(Ninv) - brute) < 1e-12 * max(1.0, abs(brute))


def _brute_G(h, beta, r, t, V, x, y, rx, ry):
    """<T c_rx(x) c+_ry(y) prod e^{V n}> / <T prod e^{V n}> by explicit operator products."""
    L = h.shape[0]
    H = fock.many_body_h0(h)
    dim = 1 << L
    occ = np.array([[(s >> q) & 1 for q in range(L)] for s in range(dim)], float)
    C = np.zeros((dim, dim))
    for st in range(dim):
        if (st >> rx) & 1:
            sg = -1 if bin(st & ((1 << rx) - 1)).count("1") % 2 else 1
            C[st ^ (1 << rx), st] = sg
    Cd_y = np.zeros((dim, dim))
    for st in range(dim):
        if not (st >> ry) & 1:
            sg = -1 if bin(st & ((1 << ry) - 1)).count("1") % 2 else 1
            Cd_y[st | (1 << ry), st] = sg
    ops = [(t[i], np.diag(np.exp(V[i] * occ[:, r[i]]))) for i in range(len(r))]
    sign = 1.0
    if x > y:
        ops += [(x, C), (y, Cd_y)]
    else:
        ops += [(y, Cd_y), (x, C)]
        sign = -1.0

    def ev(h_):
        return lambda tt: (lambda E, U: (U * np.exp(-tt * E)) @ U.T)(*np.linalg.eigh(h_))
    E = ev(H)
    def product(op_list):
        op_list = sorted(op_list, key=lambda o: o[0])
        P = E(op_list[0][0]) if op_list else E(beta)
        prev = op_list[0][0] if op_list else beta
        for n, (tt, O) in enumerate(op_list):
            P = O @ P
            nxt = op_list[n + 1][0] if n + 1 < len(op_list) else beta
            P = E(nxt - prev) @ P
            prev = nxt
        return np.trace(P)
    num = product(ops)
    den = product([(t[i], np.diag(np.exp(V[i] * occ[:, r[i]]))) for i in range(len(r))])
    return sign * num / den


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_configuration_green_function(seed):
    rng = np.random.default_rng(10 + seed)
    L, k, beta = 2, 3, 1.7
    h = rng.normal(size=(L, L))
    h = 0.5 * (h + h.T)
    r = rng.integers(0, L, size=k)
    t = rng.random(k) * beta
    V = rng.normal(size=k)
    g = _g_matrix(h, beta, r, t)
    ev = np.exp(V)
    N = np.linalg.inv(np.diag(ev) - g * (ev - 1.0)[None, :])
    M = (ev - 1.0)[:, None] * N
    for (x, y, rx, ry) in [(0.9, 0.3, 0, 1), (0.2, 1.1, 1, 1), (1.5, 0.4, 1, 0)]:
        brute = _brute_G(h, beta, r, t, V, x, y, rx, ry)
        gxI = np.array([fock.single_particle_g(h, beta, rx, x, r[j], t[j]) for j in range(k)])
        gIy = np.array([fock.single_particle_g(h, beta, r[j], t[j], ry, y) for j in range(k)])
        est = fock.single_particle_g(h, beta, rx, x, ry, y) + gxI @ M @ gIy
        assert abs(est - brute) < 1e-11, (est, brute)
        # the transposed M (N (e^V - 1)) is not the estimator
        wrong = fock.single_particle_g(h, beta, rx, x, ry, y) + gxI @ (N * (ev - 1.0)[None, :]) @ gIy
        assert abs(wrong - brute) > 1e-6


@pytest.mark.parametrize("mu", [0.0, 0.4])
def test_oracle_propagator_is_free_g(mu):
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=3.0, mu=mu, n_tau=3001)
    h = geometry.hopping_matrix(m.a1, m.a2) - mu * np.eye(4)
    rng = np.random.default_rng(7)
    for _ in range(25):
        ri, rj = rng.integers(0, 4, size=2)
        ti, tj = rng.random(2) * m.beta
        want = fock.single_particle_g(h, m.beta, ri, ti, rj, tj)
        got_exact = m.prop.analytic(m.diff[ri, rj], ti - tj if ti >= tj else ti - tj + m.beta)
        got_exact = -got_exact if ti >= tj else got_exact
        assert abs(got_exact - want) < 1e-12
        got_tab = float(m.prop.g(ri, ti, rj, tj))
        assert abs(got_tab - want) < 2e-6         # linear interpolation, h = 1e-3
    # equal time, same site: 1 - n0
    for ri in range(4):
        assert abs(float(m.prop.g(ri, 0.5, ri, 0.5)) - fock.single_particle_g(h, m.beta, ri, 0.5, ri, 0.5)) < 1e-6

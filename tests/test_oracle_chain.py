"""Pins for the oracle's Markov chain (Sec. 2.3).

* Hubbard atom weight: prod_sigma det N_sigma^{-1} = (1 + cosh(gamma sum_i s_i)) / 2;
* every recorded ratio equals a ratio of directly computed determinants;
* the tracked sign equals the sign of the recomputed weight;
* N after many updates equals the direct inverse (the refresh invariant);
* the atom's order distribution is the two-Poisson mixture
  p_k ~ [K^k + (K + beta U / 2)^k] / k!  (exact, from expanding e^{K - beta E});
* U = 0 gives gamma = 0, N = 1 and a Poisson(K) order distribution.
"""
import math

import numpy as np
import pytest

from oracle import ctaux


def atom(U=4.0, beta=5.0, K_exp=1.0):
    return ctaux.Model(a1=(1, 0), a2=(0, 1), t=0.0, U=U, beta=beta, mu=0.0, K_exp=K_exp,
                       n_tau=2, use_table=False)


def test_atom_weight_closed_form():
    m = atom()
    rng = np.random.default_rng(0)
    for k in range(1, 9):
        r = np.zeros(k, int)
        t = rng.random(k) * m.beta
        s = rng.choice([-1, 1], size=k)
        w = np.prod([np.linalg.det(ctaux.n_inverse(m, r, t, s, sp)) for sp in (0, 1)])
        assert abs(w - (1 + math.cosh(m.gamma * s.sum())) / 2) < 1e-10 * w


def _logdet_pair(m, r, t, s):
    if len(r) == 0:
        return 1.0
    return np.prod([np.linalg.det(ctaux.n_inverse(m, r, t, s, sp)) for sp in (0, 1)])


@pytest.mark.parametrize("p_flip", [0.0, 0.3])
@pytest.mark.parametrize("cfg", ["atom", "2x2"])
def test_ratios_equal_direct_determinants(cfg, p_flip):
    m = atom() if cfg == "atom" else ctaux.Model(U=4.0, beta=3.0, n_tau=400)
    w = ctaux.Walker(m, seed=11, record=True, p_flip=p_flip)
    w.random_config(6)
    for _ in range(300):
        before = (w.r.copy(), w.t.copy(), w.s.copy(), w.id.copy())
        kind, acc = w.step()
        rec = w.trace[-1]
        k0 = len(before[0])
        if kind == 0:
            r1 = np.append(before[0], rec[1])
            t1 = np.append(before[1], rec[2])
            s1 = np.append(before[2], rec[3])
            want = m.K_exp / (k0 + 1) * _logdet_pair(m, r1, t1, s1) / _logdet_pair(m, *before[:3])
        elif k0 == 0:
            continue
        elif kind == 2:
            p = int(np.where(before[3] == rec[4])[0][0])
            s1 = before[2].copy()
            s1[p] = -s1[p]
            want = _logdet_pair(m, before[0], before[1], s1) / _logdet_pair(m, *before[:3])
        else:
            p = int(np.where(before[3] == rec[4])[0][0])
            keep = np.arange(k0) != p
            want = k0 / m.K_exp * _logdet_pair(m, before[0][keep], before[1][keep], before[2][keep]) \
                / _logdet_pair(m, *before[:3])
        assert abs(rec[6] - want) < 1e-9 * abs(want), (kind, rec[6], want)
        assert w.sign == w.weight_sign()


@pytest.mark.parametrize("p_flip", [0.0, 0.3])
def test_updated_N_equals_direct_inverse(p_flip):
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=5.0, n_tau=1000)
    w = ctaux.Walker(m, seed=3, p_flip=p_flip)
    w.random_config(20)
    for _ in range(40):
        w.sweep()
    assert w.k > 5
    assert p_flip == 0.0 or w.n_acc_flip > 10
    drift = w.refresh()
    assert drift < 1e-10


@pytest.mark.parametrize("p_flip", [0.0, 0.25])
def test_atom_order_distribution(p_flip):
    """Spin flips keep the order and the weight's stationary distribution:
    the same two-Poisson law holds with a share of flip proposals."""
    U, beta, K = 4.0, 2.0, 1.0
    m = atom(U=U, beta=beta, K_exp=K)
    w = ctaux.Walker(m, seed=5, p_flip=p_flip)
    for _ in range(2000):
        w.step()
    orders = []
    for _ in range(120000):
        w.step()
        orders.append(w.k)
    orders = np.array(orders)
    kmax = 25
    ks = np.arange(kmax + 1)
    a, b = K, K + beta * U / 2
    logp = np.logaddexp(ks * np.log(a), ks * np.log(b)) - np.array([math.lgamma(k + 1) for k in ks])
    p = np.exp(logp - logp.max())
    p /= p.sum()
    # batch means over 40 consecutive blocks absorb the autocorrelation
    B = 40
    blocks = orders[: (len(orders) // B) * B].reshape(B, -1)
    hist = np.array([np.bincount(np.minimum(x, kmax), minlength=kmax + 1) / len(x) for x in blocks])
    est, err = hist.mean(axis=0), hist.std(axis=0, ddof=1) / np.sqrt(B)
    z = np.abs(est - p) / np.maximum(err, 1e-4)
    assert np.max(z[:14]) < 4.5, list(zip(est[:14], p[:14], z[:14]))
    mean_exact = K + beta * U / 2 * math.exp(beta * U / 2) / (1 + math.exp(beta * U / 2))
    means = blocks.mean(axis=1)
    assert abs(orders.mean() - mean_exact) < 4.5 * means.std(ddof=1) / np.sqrt(B)


def test_free_limit_is_poisson():
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=0.0, beta=2.0, K_exp=2.0, n_tau=200)
    assert m.gamma == 0.0
    w = ctaux.Walker(m, seed=9)
    ks = []
    for _ in range(40000):
        w.step()
        ks.append(w.k)
    for sp in (0, 1):
        assert np.allclose(w.N[sp], np.eye(w.k))
    assert abs(np.mean(ks) - 2.0) < 0.1
    assert abs(np.var(ks) - 2.0) < 0.3


def test_atom_order_distribution_per_sweep():
    """Sampling once per sweep reproduces the order law when the sweep length
    is frozen after the warm-up (as the library's and the oracle's measured
    chains do); a length that follows the current order would not."""
    U, beta, K = 4.0, 2.0, 1.0
    m = atom(U=U, beta=beta, K_exp=K)
    w = ctaux.Walker(m, seed=9, k_s=4)
    warm = []
    for n in range(400):
        if n >= 200:
            warm.append(w.k)
        w.sweep()
    w.freeze_sweep_length(np.mean(warm))
    assert w.sweep_length() % 4 == 0 and w.sweep_length() >= 4
    orders = []
    for _ in range(14000):
        w.sweep()
        orders.append(w.k)
    orders = np.array(orders)
    kmax = 25
    ks = np.arange(kmax + 1)
    a, b = K, K + beta * U / 2
    logp = np.logaddexp(ks * np.log(a), ks * np.log(b)) - np.array([math.lgamma(k + 1) for k in ks])
    p = np.exp(logp - logp.max())
    p /= p.sum()
    B = 40
    blocks = orders[: (len(orders) // B) * B].reshape(B, -1)
    hist = np.array([np.bincount(np.minimum(x, kmax), minlength=kmax + 1) / len(x) for x in blocks])
    est, err = hist.mean(axis=0), hist.std(axis=0, ddof=1) / np.sqrt(B)
    z = np.abs(est - p) / np.maximum(err, 1e-4)
    assert np.max(z[:14]) < 4.5, list(zip(est[:14], p[:14], z[:14]))

"""Pins of the oracle's error bars (binning and jackknife, Sec. 2.3 sign-weighted
averages).

* closed forms: with a constant denominator the jackknife sigma of a ratio is
  the standard error of the bin means, std(bin means, ddof=1) / sqrt(B); the
  ratio form agrees with the linearised (delta-method) error;
* an AR(1) sequence with correlation rho has the exact asymptotic variance
  of its mean, var (1 + rho) / (1 - rho) / n: bins much longer than the
  correlation time reproduce it and stay stable when halved in number,
  bins shorter than it underestimate it and the bin-halving check shows it;
* the physics pin: 32 independent Hubbard-atom chains (different seeds),
  each giving estimates of Im G(i w_0), Im G(i w_2) and <k> with jackknife
  sigmas.  The exact values are G(i w) = i w / ((i w)^2 - U^2/4) and
  <k> = K + beta U (1/2 - d), d = 1 / (2 (1 + e^{beta U / 2})).  The z
  scores (estimate - exact) / sigma must have mean square near 1; the same
  check applied to sigma scaled by 2 or by 1/2 must fail (the test has the
  power to see a wrong sigma), and halving the bin count must not change
  sigma beyond its statistical error.
"""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle import ctaux, run, stats

U, BETA, K_EXP = 4.0, 5.0, 1.0
N_CHAINS = 32


def test_jackknife_of_a_mean_is_the_standard_error():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(640, 3))
    for B in (8, 32):
        est, err = stats.jackknife_ratio(x, np.ones(len(x)), B)
        b = stats.bins(x, B)
        assert np.allclose(est, x.mean(axis=0))
        assert np.allclose(err, b.std(axis=0, ddof=1) / np.sqrt(B), rtol=1e-12)


def test_jackknife_ratio_matches_the_linearised_error():
    # f = <a>/<b>: delta method sigma^2 = var(a_b - f b_b) / (B <b>^2) over bin means
    rng = np.random.default_rng(2)
    n, B = 3200, 32
    b = 1.0 + 0.3 * rng.normal(size=n)
    a = 0.5 * b + 0.2 * rng.normal(size=n)
    est, err = stats.jackknife_ratio(a, b, B)
    ab, bb = stats.bins(a, B), stats.bins(b, B)
    f = ab.mean() / bb.mean()
    lin = np.sqrt(np.var(ab - f * bb, ddof=1) / B) / bb.mean()
    assert abs(est - a.sum() / b.sum()) < 1e-12
    assert abs(err / lin - 1.0) < 0.02


def _ar1(rng, n, rho):
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - rho * rho)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + e[i]
    return x


def test_bin_halving_on_a_correlated_sequence():
    rho, n = 0.9, 2 ** 17
    var = 1.0 / (1.0 - rho * rho)
    exact = np.sqrt(var * (1 + rho) / (1 - rho) / n)     # tau_int = 9.5 steps
    rng = np.random.default_rng(3)
    longs, shorts = [], []
    for _ in range(8):
        x = _ar1(rng, n, rho)
        one = np.ones(n)
        e32, e16 = stats.bin_halving(x, one, 32)        # bins of 4096 steps
        longs.append((e32 / exact, e16 / e32))
        e_short, e_half = stats.bin_halving(x, one, n // 2)   # bins of 2 steps
        shorts.append((e_short / exact, e_half / e_short))
    longs, shorts = np.array(longs), np.array(shorts)
    # long bins: sigma right (within its ~13% statistical error per run) and stable
    assert abs(longs[:, 0].mean() - 1.0) < 0.12
    assert abs(longs[:, 1].mean() - 1.0) < 0.12
    # two-step bins: sigma far too small, and it grows when the bins double
    assert shorts[:, 0].mean() < 0.45
    assert shorts[:, 1].mean() > 1.3


def _atom():
    return ctaux.Model(a1=(1, 0), a2=(0, 1), t=0.0, U=U, beta=BETA, mu=0.0, K_exp=K_EXP, n_tau=2,
                       use_table=False)


def _chain(seed):
    """One independent atom chain: estimates, sigmas, and bin-halving ratios."""
    m = _atom()
    w, acc, orders = run.run_chain(m, seed=seed, sweeps=1024, warmup=100, n_freq=3, k_s=16)
    res = run.estimate_G(m, acc, B=32, spin_average=True)
    res16 = run.estimate_G(m, acc, B=16, spin_average=True)
    est = [res["Giw"][0, 0].imag, res["Giw"][0, 2].imag]
    err = [res["Giw_err"][0, 0].imag, res["Giw_err"][0, 2].imag]
    halv = [res16["Giw_err"][0, 0].imag / err[0], res16["Giw_err"][0, 2].imag / err[1]]
    k_est, k_err = stats.jackknife_ratio(orders.astype(float), np.ones(len(orders)), 32)
    _, k_err16 = stats.jackknife_ratio(orders.astype(float), np.ones(len(orders)), 16)
    return est + [float(k_est)], err + [float(k_err)], halv + [float(k_err16 / k_err)]


@pytest.fixture(scope="module")
def atom_chains():
    seeds = [4242 + 17 * c for c in range(N_CHAINS)]
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        out = list(ex.map(_chain, seeds))
    est = np.array([o[0] for o in out])
    err = np.array([o[1] for o in out])
    halv = np.array([o[2] for o in out])
    wn = (2 * np.array([0, 2]) + 1) * np.pi / BETA
    g_exact = (1j * wn / ((1j * wn) ** 2 - U * U / 4)).imag
    d = 1.0 / (2.0 * (1.0 + np.exp(BETA * U / 2)))
    k_exact = K_EXP + BETA * U * (0.5 - d)
    exact = np.concatenate([g_exact, [k_exact]])
    return est, err, halv, exact


def _sigma_ok(est, err, exact):
    """Mean square of the z scores over all chains and observables within
    [0.5, 1.8]: 96 scores in 32 independent chains."""
    z2 = ((est - exact[None, :]) / err) ** 2
    return 0.5 < z2.mean() < 1.8, z2.mean()


def test_atom_sigma_matches_the_spread_of_independent_chains(atom_chains):
    est, err, halv, exact = atom_chains
    ok, msq = _sigma_ok(est, err, exact)
    print(f"mean z^2 over {est.size} scores: {msq:.3f}")
    assert ok, msq
    # the check has the power to see a sigma off by a factor of two either way
    assert not _sigma_ok(est, 2.0 * err, exact)[0]
    assert not _sigma_ok(est, 0.5 * err, exact)[0]
    # the per-chain sigmas agree with the spread of the estimates themselves
    spread = est.std(axis=0, ddof=1)
    assert np.all(np.abs(spread / err.mean(axis=0) - 1.0) < 0.4), spread / err.mean(axis=0)


def test_atom_sigma_stable_under_bin_halving(atom_chains):
    est, err, halv, exact = atom_chains
    r = halv.mean(axis=0)
    print(f"sigma(16 bins) / sigma(32 bins), mean over chains: {r}")
    # one chain's ratio scatters by ~0.2; the mean of 32 by ~0.04
    assert np.all(np.abs(r - 1.0) < 0.15), r

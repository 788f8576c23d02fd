"""Statistical pins of the oracle's measurement (Sec. 2.3).

* Hubbard atom: G(i w) = i w / ((i w)^2 - U^2/4) and
  G(tau) = -cosh(U (beta/2 - tau) / 2) / (2 cosh(beta U / 4));
* 2x2 periodic Hubbard cluster (t = 1, U = 4, beta = 5, half filling): G(K, i w_n)
  and G(K, tau) against exact diagonalisation of the same cluster;
* K_exp independence of G.

Agreement criterion: at most max(1, 1% of n) of the n compared points beyond
3 sigma (at n ~ 100 a single 3-sigma excursion happens a quarter of the time)
and no point beyond 4.5 sigma (Bonferroni-safe for the few hundred points
compared).
The cluster comparisons use the spin-averaged G: the paramagnetic Green's
function.  Per spin, G carries a slowly relaxing magnetisation mode (insert and
remove moves flip the cluster moment only slowly at U = 4, beta = 5), which the
bin-jackknife cannot resolve in a short run; it cancels in the spin average.
"""
import numpy as np
import pytest

from oracle import ctaux, ed, geometry, run


def _zscores(est, err, want):
    return (np.abs(est - want) / np.maximum(err, 1e-12)).ravel()


def _check(est, err, want, frac=0.01, zmax=4.5):
    """Apply the criterion to one array of points, or to a list of z arrays."""
    z = _zscores(est, err, want) if err is not None else np.concatenate(est)
    n_out = int(np.sum(z >= 3.0))
    assert n_out <= max(1, int(round(frac * len(z)))) and z.max() < zmax, (n_out, z.max(), len(z))


def test_atom_green_function():
    U, beta = 4.0, 5.0
    m = ctaux.Model(a1=(1, 0), a2=(0, 1), t=0.0, U=U, beta=beta, mu=0.0, n_tau=2, use_table=False)
    nf = 256
    w, acc, orders = run.run_chain(m, seed=21, sweeps=6000, warmup=200, n_freq=nf, k_s=16)
    taus = np.linspace(0.1, beta - 0.1, 12)
    res = run.estimate_G(m, acc, taus=taus)
    wn = (2 * np.arange(16) + 1) * np.pi / beta
    want = 1j * wn / ((1j * wn) ** 2 - U * U / 4)
    gt = -np.cosh(U * (beta / 2 - taus) / 2) / (2 * np.cosh(beta * U / 4))
    zs = []
    for sp in range(2):
        zs.append(_zscores(res["Giw"][sp, 0, :16].real, res["Giw_err"][sp, 0, :16].real + 1e-14, want.real))
        zs.append(_zscores(res["Giw"][sp, 0, :16].imag, res["Giw_err"][sp, 0, :16].imag, want.imag))
        zs.append(_zscores(res["Gtau"][sp, 0], res["Gtau_err"][sp, 0], gt))
    _check(zs, None, None)
    assert res["sign"] == 1.0


@pytest.mark.parametrize("p_flip", [0.0, 0.3])
def test_atom_in_a_field_green_function(p_flip):
    """One bare propagator per spin (a Zeeman field h splits xi_up and
    xi_down): the chain's G_up and G_down against the four-state exact
    result, which the ED tests pin by its closed form.  A dropped spin index
    (one propagator for both spins) fails: the two G differ by ~0.1.  At
    beta U = 4 the chain passes through low orders often enough to flip the
    atom's moment (at larger beta U insert/remove moves flip it too rarely
    for the minority configurations to be sampled in a short run).  With a
    share of spin-flip proposals the same exact G must come out."""
    U, beta, mu, h = 2.0, 2.0, 0.3, 0.5
    m = ctaux.Model(a1=(1, 0), a2=(0, 1), t=0.0, U=U, beta=beta, mu=mu, n_tau=2, use_table=False, h=h)
    nf = 256
    w, acc, orders = run.run_chain(m, seed=31, sweeps=8000, warmup=200, n_freq=nf, k_s=8, p_flip=p_flip)
    assert p_flip == 0.0 or w.n_acc_flip > 1000
    taus = np.linspace(0.1, beta - 0.1, 12)
    res = run.estimate_G(m, acc, taus=taus)
    e = ed.ED(np.zeros((1, 1)), U=U, mu=mu, beta=beta, h=h)
    zs = []
    for sp in range(2):
        want = e.G_iw(np.array([1.0]), sp, 16)
        zs.append(_zscores(res["Giw"][sp, 0, :16].real, res["Giw_err"][sp, 0, :16].real + 1e-14, want.real))
        zs.append(_zscores(res["Giw"][sp, 0, :16].imag, res["Giw_err"][sp, 0, :16].imag, want.imag))
        zs.append(_zscores(res["Gtau"][sp, 0], res["Gtau_err"][sp, 0], e.G_tau(np.array([1.0]), sp, taus)))
    _check(zs, None, None)
    # the two spins are measured apart and differ as the exact ones do
    d_exact = e.G_tau(np.array([1.0]), 0, taus) - e.G_tau(np.array([1.0]), 1, taus)
    assert np.max(np.abs(d_exact)) > 0.05


@pytest.fixture(scope="module")
def cluster_2x2():
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=5.0, mu=0.0, n_tau=1000)
    w, acc, orders = run.run_chain(m, seed=985456376, sweeps=3000, warmup=100, n_freq=512, k_s=16)
    tij = geometry.hopping_matrix(m.a1, m.a2)
    e = ed.ED(tij, U=m.U, mu=m.mu, beta=m.beta)
    ph = ed.momentum_phases(m.sites, m.K)
    return m, acc, orders, e, ph


def test_2x2_matsubara_vs_ed(cluster_2x2):
    m, acc, orders, e, ph = cluster_2x2
    res = run.estimate_G(m, acc, n_freq=24, spin_average=True)
    # Particle-hole symmetry at half filling maps K -> K + (pi, pi) with
    # G -> -G*, configuration by configuration for the spin-averaged
    # estimator: K = (pi, pi) and (0, pi) repeat K = (0, 0) and (pi, 0).
    assert np.allclose(res["Giw"][3], -res["Giw"][0].conj(), atol=1e-12)
    assert np.allclose(res["Giw"][2], -res["Giw"][1].conj(), atol=1e-12)
    zs = []
    for iK in range(2):
        want = e.G_iw(ph[iK], 0, 24)
        zs.append(_zscores(res["Giw"][iK].real, res["Giw_err"][iK].real + 1e-15, want.real))
        zs.append(_zscores(res["Giw"][iK].imag, res["Giw_err"][iK].imag, want.imag))
    _check(zs, None, None)
    assert 20 < orders.mean() < 45         # a mean order of about 30 is expected here


def test_2x2_tau_vs_ed(cluster_2x2):
    m, acc, orders, e, ph = cluster_2x2
    taus = np.linspace(0.05, m.beta - 0.05, 20)
    res = run.estimate_G(m, acc, taus=taus, spin_average=True)
    _check([_zscores(res["Gtau"][iK], res["Gtau_err"][iK], e.G_tau(ph[iK], 0, taus))
            for iK in range(2)], None, None)
    # half filling: G(r = 0, tau) = G(r = 0, beta - tau)
    Gr0 = res["Gtau"].mean(axis=0)
    assert np.allclose(Gr0, Gr0[::-1], atol=5 * res["Gtau_err"].max())


def test_expansion_parameter_independence(cluster_2x2):
    m1, acc1, orders1, e, ph = cluster_2x2
    m2 = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=5.0, mu=0.0, n_tau=1000, K_exp=2.0)
    w2, acc2, orders2 = run.run_chain(m2, seed=77, sweeps=1500, warmup=100, n_freq=24, k_s=16)
    r1 = run.estimate_G(m1, acc1, n_freq=24, spin_average=True)
    r2 = run.estimate_G(m2, acc2, n_freq=24, spin_average=True)
    d = r1["Giw"] - r2["Giw"]
    s = np.hypot(r1["Giw_err"].real, r2["Giw_err"].real)
    z = np.abs(d.real) / s
    assert np.mean(z < 3) > 0.97 and z.max() < 5
    # <k> = K_exp - beta <H_int>: the orders shift by Delta K_exp = 1
    assert abs((orders2.mean() - orders1.mean()) - 1.0) < 1.0


def test_sampled_direct_sums_equal_full_sums():
    """The sampled form of the direct sums (chosen frequencies or momenta)
    returns exactly the corresponding entries of the full evaluation."""
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=4.0, beta=5.0, n_tau=200)
    rng = np.random.default_rng(3)
    k = 17
    r = rng.integers(0, m.Nc, k)
    t = rng.random(k) * m.beta
    M = rng.standard_normal((k, k))
    from oracle import measure
    full = measure.M_K_iw(m, r, t, M, 40)
    freqs, Ks = [0, 7, 39], [1, 3]
    assert np.allclose(measure.M_K_iw(m, r, t, M, 40, freqs=freqs), full[:, freqs], rtol=0, atol=1e-13)
    assert np.allclose(measure.M_K_iw(m, r, t, M, 40, Ks=Ks), full[Ks, :], rtol=0, atol=1e-13)
    assert np.allclose(measure.M_K_iw(m, r, t, M, 40, freqs=freqs, Ks=Ks), full[np.ix_(Ks, freqs)], rtol=0,
                       atol=1e-13)

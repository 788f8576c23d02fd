"""Pins of the DCA loop's steps in the oracle (oracle/dca.py, Sec. 2.1).

* patches: the union of the Nc patches' quadrature points is a uniform grid
  of the Brillouin zone (the mean of e^{i k . R} over it vanishes for every
  small lattice vector R != 0: orthogonality and equal size), each patch is
  inversion symmetric and lies in the Wigner-Seitz cell of the reciprocal
  superlattice, also for a cluster whose reciprocal vectors are not
  orthogonal;
* coarse-graining at Nc = 1 and Sigma = 0 is the local Green's function of
  the square lattice, int d eps rho(eps) / (i w + mu - eps) with the density
  of states rho(eps) = K(1 - eps^2/16) / (2 pi^2) (complete elliptic
  integral), computed by scipy quadrature;
* one point per patch (L = 1) is the isolated cluster: Gbar = G0cal =
  1/(i w - xi_K), and the tau table equals the closed form of G0(r, tau);
* the transform to tau reproduces the closed form of a two-pole function;
* cluster exclusion in the atomic limit (t = 0) returns 1/(i w + mu) for any
  Sigma; Dyson's equation applied to Gbar returns Sigma (the fixed point);
* the loop at U = 0 keeps Sigma = 0 exactly (M = 0, so G_c = G0cal).
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import dca, g0, geometry


@pytest.mark.parametrize("a1,a2,L", [((2, 0), (0, 2), 6), ((4, 0), (0, 4), 4), ((2, 1), (0, 2), 5),
                                     ((2, 2), (2, -2), 4), ((1, 0), (0, 1), 8)])
def test_patches_tile_the_zone_uniformly(a1, a2, L):
    d = dca.DCA(a1, a2, L=L, n_freq=4, n_cg=4, n_tau=10)
    kt, wt = d.kt, d.wt
    assert abs(wt.sum() - L * L) < 1e-12
    allpts = (d.K[:, None, :] + kt[None, :, :]).reshape(-1, 2)
    allw = np.tile(wt, d.Nc)
    for Rx in range(-3, 4):
        for Ry in range(-3, 4):
            m = np.sum(allw * np.exp(1j * allpts @ np.array([Rx, Ry], float))) / allw.sum()
            assert abs(m - (1.0 if (Rx, Ry) == (0, 0) else 0.0)) < 1e-12, (Rx, Ry, m)
    # inversion symmetric with its weights, inside the Wigner-Seitz cell of
    # the reciprocal superlattice
    key = lambda p: tuple(np.round(p * 1e9).astype(np.int64))
    wk = {}
    for p, x in zip(kt, wt):
        wk[key(p)] = wk.get(key(p), 0.0) + x
    for p, x in zip(kt, wt):
        assert abs(wk.get(key(-p), 0.0) - wk[key(p)]) < 1e-12
    B = dca.reciprocal_superlattice(a1, a2)
    for n1 in range(-2, 3):
        for n2 in range(-2, 3):
            G = n1 * B[0] + n2 * B[1]
            assert np.all(np.sum(kt * kt, axis=1) <= np.sum((kt - G) ** 2, axis=1) + 1e-9)


def _G_local_dos(w, mu):
    """int d eps rho(eps) / (i w + mu - eps), square lattice, t = 1, split at
    the logarithmic singularity of rho at eps = 0 (quadrature nodes are
    interior, so rho is never evaluated there)."""
    rho = lambda e: special.ellipkm1((e / 4.0) ** 2) / (2.0 * np.pi ** 2)      # K(1 - (e/4)^2)
    out = 0.0
    for lo, hi in ((-4.0, 0.0), (0.0, 4.0)):
        re = integrate.quad(lambda e: rho(e) * (mu - e) / (w * w + (e - mu) ** 2), lo, hi, limit=400,
                            epsabs=1e-14, epsrel=1e-13)[0]
        im = integrate.quad(lambda e: rho(e) * (-w) / (w * w + (e - mu) ** 2), lo, hi, limit=400,
                            epsabs=1e-14, epsrel=1e-13)[0]
        out += re + 1j * im
    return out


def test_single_site_coarse_graining_is_the_lattice_dos_integral():
    d = dca.DCA((1, 0), (0, 1), t=1.0, beta=5.0, mu=0.3, n_freq=8, n_cg=8, n_tau=10, L=128)
    gbar, g0c = d.coarse_grain(np.zeros((1, 8)))
    for n in range(6):
        want = _G_local_dos(d.w[n], 0.3)
        assert abs(gbar[0, n] - want) < 1e-9, (n, gbar[0, n], want)
    assert np.max(np.abs(g0c - gbar)) < 1e-15          # Sigma = 0: nothing to exclude


@pytest.mark.parametrize("a1,a2", [((2, 0), (0, 2)), ((4, 0), (0, 4))])
def test_one_point_per_patch_is_the_isolated_cluster(a1, a2):
    d = dca.DCA(a1, a2, t=1.0, tp=-0.2, beta=5.0, mu=-0.4, n_freq=32, n_cg=2048, n_tau=300, L=1)
    xi = geometry.dispersion(d.K, 1.0, -0.2) + 0.4
    gbar, g0c = d.coarse_grain(np.zeros((d.Nc, 32)))
    ref = g0.g0_K_iw(xi, d.n_cg, d.beta)
    assert np.max(np.abs(gbar - ref)) < 1e-15 and np.max(np.abs(g0c - ref)) < 1e-15
    tab = d.g0_table(g0c)
    assert np.max(np.abs(tab - g0.g0_table(d.sites, d.K, xi, d.beta, d.n_tau))) < 1e-9


def test_transform_of_a_two_pole_function():
    d = dca.DCA((2, 0), (0, 2), t=1.0, beta=8.0, mu=0.2, n_freq=16, n_cg=4096, n_tau=200, L=4)
    c2 = d.epsbar - d.mu
    wts = np.array([0.6, 0.4])
    xis = np.stack([c2 + 1.0, c2 - 1.5])               # sum_j w_j xi_j = c2
    iw = 1j * d.w
    f = sum(wts[j] / (iw[None, :] - xis[j][:, None]) for j in range(2))
    got = d.g0_K_tau(f)
    tau = np.linspace(0, d.beta, d.n_tau)
    want = sum(wts[j] * g0.g0_K_tau(xis[j], tau, d.beta) for j in range(2))
    assert np.max(np.abs(got - want)) < 1e-9


def test_exclusion_in_the_atomic_limit_and_the_dyson_fixed_point():
    rng = np.random.default_rng(3)
    d = dca.DCA((2, 0), (0, 2), t=0.0, beta=4.0, mu=0.35, n_freq=24, n_cg=64, n_tau=10, L=5)
    sig = rng.normal(size=(4, 24)) + 1j * rng.normal(size=(4, 24))
    gbar, g0c = d.coarse_grain(sig)
    assert np.max(np.abs(g0c - 1.0 / (1j * d.w[None, :] + 0.35))) < 1e-14
    d2 = dca.DCA((2, 0), (0, 2), t=1.0, tp=0.1, beta=4.0, mu=0.35, n_freq=24, n_cg=64, n_tau=10, L=5)
    gbar, g0c = d2.coarse_grain(sig)
    back = dca.DCA.self_energy(g0c, gbar[:, :24], np.zeros_like(sig), 1.0)
    assert np.max(np.abs(back - sig)) < 1e-12 * np.max(np.abs(sig))
    mixed = dca.DCA.self_energy(g0c, gbar[:, :24], 2.0 * sig, 0.25)
    assert np.max(np.abs(mixed - (0.25 * sig + 0.75 * 2.0 * sig))) < 1e-12 * np.max(np.abs(sig))


def test_sigma_extension_beyond_the_measured_frequencies():
    d = dca.DCA((1, 0), (0, 1), beta=3.0, n_freq=10, n_cg=40, n_tau=10, L=2)
    sig = (0.3 - 2.0j / d.w[:10])[None, :]
    ext = d.extend_sigma(sig)
    assert np.array_equal(ext[:, :10], sig)
    assert np.allclose(ext[0, 10:], 0.3 - 2.0j / d.w[10:], rtol=1e-14, atol=0)


def test_loop_at_u0_keeps_sigma_zero():
    d = dca.DCA((2, 0), (0, 2), t=1.0, beta=3.0, mu=0.1, n_freq=16, n_cg=512, n_tau=200, L=4)
    sigs, (G, sign) = dca.dca_loop(d, U=0.0, iterations=1, sweeps=20, warmup=5, seed=1)
    assert np.max(np.abs(sigs[-1])) == 0.0
    g0c = d.coarse_grain(np.zeros((d.Nc, 16)))[1]
    assert np.max(np.abs(G[0] - g0c[:, :16])) == 0.0

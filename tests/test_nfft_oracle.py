"""Pins of the delayed-NFFT measurement oracle (oracle/nfft.py).

The gridded transform must reproduce the plain non-uniform DFT within the
kernel's error scale exp(-(2/3) pi M_sp) per unit of sample weight:
* one sample f at s has the closed form F(w_n) = f e^{i w_n s} (at s = 0,
  next to 0 and next to beta, where the kernel wraps antiperiodically), and
  the error shrinks at that rate as M_sp grows (a wrong kernel transform or
  width leaves an O(1) or a slowly shrinking error);
* a configuration's M(K, i w_n) from its grid equals the direct sums of
  measure.M_K_iw (pairs with tau_i < tau_j test the antiperiodic image and
  its sign, every displacement row its phase e^{-i K r_d});
* grids accumulated over several configurations with their signs and
  transformed once equal the sum of the direct results (the delay).
"""
import numpy as np
import pytest

from oracle import ctaux, measure, nfft
from tests.ctaux_cases import model


@pytest.mark.parametrize("m_sp", [4, 6, 8, 10])
def test_single_sample_closed_form(m_sp):
    beta, nf = 10.0, 64
    w = measure.matsubara(nf, beta)
    errs = []
    for s in (0.0, 1e-9, 0.37, 0.5 * beta, beta - 1e-7, 0.999 * beta):
        g = nfft.grid_samples([s], [-1.5], beta, nf, m_sp)
        F = nfft.transform(g[None], beta, nf, m_sp)[0]
        errs.append(np.max(np.abs(F + 1.5 * np.exp(1j * w * s))) / 1.5)
    assert max(errs) <= 2.0 * nfft.error_scale(m_sp)
    # and not much better than the scale either: the rate is the aliasing one
    assert max(errs) >= 0.1 * nfft.error_scale(m_sp)


@pytest.mark.parametrize("name,k", [("2x2_U4_b5", 40), ("4x4_U4_b10", 150)])
@pytest.mark.parametrize("m_sp", [6, 8, 10])
def test_grid_matches_direct_sums(name, k, m_sp):
    m = model(name)
    ow = ctaux.Walker(m, seed=11)
    ow.random_config(k)
    nf = 96
    for sp in range(2):
        M = measure.M_matrix(m, ow, sp)
        direct = measure.M_K_iw(m, ow.r, ow.t, M, nf)
        G = nfft.grid_M(m, ow.r, ow.t, M, nf, m_sp)
        got = nfft.M_K_iw_from_grid(m, G, nf, m_sp)
        scale = np.abs(M).sum() / m.Nc
        assert np.max(np.abs(got - direct)) <= 2.0 * nfft.error_scale(m_sp) * scale


def test_delayed_accumulation_of_several_configurations():
    m = model("4x4_U4_b10")
    nf, m_sp = 64, 8
    G = np.zeros((m.Nc, nfft.grid_size(nf)))
    want = np.zeros((m.Nc, nf), dtype=complex)
    weight = 0.0
    for seed, k, sign in ((1, 60, 1.0), (2, 90, -1.0), (3, 0, 1.0), (4, 75, 1.0)):
        ow = ctaux.Walker(m, seed=seed)
        if k:
            ow.random_config(k)
        M = measure.M_matrix(m, ow, 0) if k else np.zeros((0, 0))
        G += sign * nfft.grid_M(m, ow.r, ow.t, M, nf, m_sp)
        want += sign * measure.M_K_iw(m, ow.r, ow.t, M, nf)
        weight += np.abs(M).sum() / m.Nc
    got = nfft.M_K_iw_from_grid(m, G, nf, m_sp)
    assert np.max(np.abs(got - want)) <= 2.0 * nfft.error_scale(m_sp) * weight


def test_grid_rejects_a_kernel_wider_than_the_grid():
    with pytest.raises(ValueError):
        nfft.grid_samples([0.1], [1.0], 1.0, 2, 5)

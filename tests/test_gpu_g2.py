"""Two-particle measurement on the GPU (particle-particle up-down channel,
Sec. 2.5; App. B four-point parameters) against the oracle.

Every case installs the oracle walker's configuration in the GPU walker
(set_config rebuilds N in FP64) and compares the accumulated
sign * G_up(k1, k2) G_down(q - k1, q - k2) element by element with the
oracle's direct double sums (oracle/twoparticle.py), relative to the largest
entry: within 1e-10 in FP64 (N agrees to ~1e-13; the sums over the k^2
vertex pairs and the Nc^2 site pairs amplify it), 1e-4 for an FP32-mixed
walker (N and M in FP32).  Cases: momentum and frequency transfers, three
walkers of one handle (their sum), the 6x6 and 8x8 clusters at orders ~1800
and ~6000 (the sizes of the measured workloads), a
caller-supplied propagator handed back, and U = 0, where G2 is exactly
G0(k1) G0(q - k1) delta_{k1 k2}.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ctaux, g0, twoparticle  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs  # noqa: E402
from tests.ctaux_cases import model  # noqa: E402


def _oracle_walker(m, k, seed):
    w = ctaux.Walker(m, seed=seed, k_s=8)
    w.set_config(*initial_config(m.Nc, m.beta, k, seed))
    return w


def _c(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _gpu_g2(params, walkers, n_w4, wm, qs):
    w = dcax.Walker(params)
    for i, ow in enumerate(walkers):
        w.set_config(ow.r, ow.t, ow.s, walker=i)
    g2, sg = w.new_g2_accumulator(n_w4, len(qs))
    w.measure_G2(n_w4, wm, qs, g2, sg)
    out = _c(g2), float(sg.item())
    w.close()
    return out


def _oracle_g2(m, walkers, n_w4, wm, qs, g0_Kw=None):
    acc = twoparticle.Accumulator2(m, n_w4, wm, qs, g0_Kw)
    for ow in walkers:
        acc.measure(ow)
    return acc.sG2, acc.s


@pytest.mark.parametrize("name,k,n_w4,wm,qs,W,prec", [
    ("2x2_U4_b5", 20, 4, 0, [0, 1, 2, 3], 1, dcax.DCAX_FP64),
    ("2x2_U4_b5", 20, 3, 2, [0, 3], 3, dcax.DCAX_FP64),
    ("4x4_U4_b10", 240, 8, 1, [0, 5], 1, dcax.DCAX_FP64),
    ("4x4_U4_b10", 240, 6, 0, [0, 15], 1, dcax.DCAX_FP32_MIXED),
    ("6x6_U6_b20", 1800, 8, 0, [0], 1, dcax.DCAX_FP64),
    ("8x8_U7_b30", 6000, 8, 0, [0], 1, dcax.DCAX_FP64),
])
def test_g2_matches_the_oracle(name, k, n_w4, wm, qs, W, prec):
    print(f"[g2] {name} k={k} n_w4={n_w4} m={wm} q={qs} walkers={W} precision={prec}", flush=True)
    m = model(name)
    ows = [_oracle_walker(m, k, CONFIGS[name]["seed"] + 40 + i) for i in range(W)]
    plist = [dcax.make_params(**params_kwargs(name, max_order=max(2 * k, 64)), precision=prec) for _ in range(W)]
    g2, sg = _gpu_g2(plist if W > 1 else plist[0], ows, n_w4, wm, qs)
    og2, osg = _oracle_g2(m, ows, n_w4, wm, qs)
    err = float(np.max(np.abs(g2 - og2)) / np.max(np.abs(og2)))
    tol = 1e-10 if prec == dcax.DCAX_FP64 else 1e-4
    print(f"  sign {sg} (oracle {osg}); max |G2| {np.max(np.abs(og2)):.3e}, rel err {err:.2e}", flush=True)
    assert sg == osg
    assert err < tol


def test_caller_propagator_gives_the_same_g2():
    name = "4x4_U4_b10"
    print(f"[g2] {name}: the walker's own table handed back", flush=True)
    m = model(name)
    ow = _oracle_walker(m, 200, 91)
    n_w4, wm, qs = 6, 2, [0, 3]
    kw = params_kwargs(name, n_freq=n_w4 + wm)
    win = dcax.Walker(dcax.make_params(**kw))
    tab = win.g0_table()
    win.close()
    pex = dcax.make_params(**kw, g0_tau=tab, g0_Kw=g0.g0_K_iw(m.xi, n_w4 + wm, m.beta))
    g_in, s_in = _gpu_g2(dcax.make_params(**kw), [ow], n_w4, wm, qs)
    g_ex, s_ex = _gpu_g2(pex, [ow], n_w4, wm, qs)
    rel = float(np.max(np.abs(g_in - g_ex)) / np.max(np.abs(g_in)))
    print(f"  internal vs caller's propagator: rel diff {rel:.1e}", flush=True)
    # N differs by the table's interpolation only through the same values: the tables are equal
    assert s_in == s_ex and rel < 1e-12
    with pytest.raises(dcax.DcaxError):        # n_freq too small for the transfer
        _gpu_g2(pex, [ow], n_w4, wm + 1, qs)


def test_g2_at_u0_is_the_bare_product():
    name = "2x2_U4_b5"
    print("[g2] U = 0", flush=True)
    m = model(name, U=0.0)
    ow = _oracle_walker(m, 12, 5)
    n_w4, wm, qs = 5, 1, [0, 2]
    g2, sg = _gpu_g2(dcax.make_params(**params_kwargs(name, U=0.0)), [ow], n_w4, wm, qs)
    n = np.arange(-n_w4, n_w4)
    w_n = (2 * n + 1) * np.pi / m.beta
    dK = twoparticle.momentum_index_table(m.K)
    want = np.zeros_like(g2)
    for iq, Q in enumerate(qs):
        for K in range(m.Nc):
            for c, nn in enumerate(n):
                wq = (2 * (wm - 1 - nn) + 1) * np.pi / m.beta
                want[iq, K, c, K, c] = sg / (1j * w_n[c] - m.xi[K]) / (1j * wq - m.xi[dK[Q, K]])
    err = float(np.max(np.abs(g2 - want)) / np.max(np.abs(want)))
    print(f"  rel err {err:.1e}", flush=True)
    assert err < 1e-14

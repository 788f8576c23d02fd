"""The DCA self-consistency loop on the GPU (Sec. 2.1) against the oracle.

* each step (coarse-graining with cluster exclusion, the transform to the
  walkers' G0cal(r, tau) tables, the cluster G from accumulators, Dyson's
  equation with mixing) against oracle/dca.py on seeded inputs, for square
  and tilted clusters, one and two spin blocks (a field), within 1e-12 of
  the scale of each result (FP64, different summation order);
* dcax_set_g0 on a walker equals creating the walker with that propagator:
  the same N, sign and, from the same configuration and seed, the same chain;
* one loop iteration at U = 0 leaves Sigma exactly zero;
* the atomic limit (t = 0): G0cal = 1/(i w + mu) whatever Sigma is, so each
  iteration measures the atom, whose G must match exact diagonalisation
  (criterion of the chain tests), and Dyson's equation returns its Sigma;
* the 2x2 DCA cluster at half filling (U = 4, beta = 5): the first iteration
  from Sigma = 0 measured on the GPU against the oracle's chain on the same
  G0cal (within 3 combined sigma), and the loop keeps the particle-hole
  symmetry of the half-filled cluster: G(K + Q) = -conj G(K) with
  Q = (pi, pi) for every measurement (to rounding), Re G(pi, 0) = 0 within
  errors, and Im Sigma < 0.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ctaux, dca, ed, measure  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402


def _c(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _t(z):
    return torch.tensor(np.stack([z.real, z.imag], axis=-1), dtype=torch.float64, device="cuda").contiguous()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("cl,L,n_spin,h", [((1, 0, 0, 1), 16, 1, 0.0), ((2, 0, 0, 2), 8, 1, 0.0),
                                           ((2, 0, 0, 2), 8, 2, 0.25), ((4, 0, 0, 4), 4, 1, 0.0),
                                           ((2, 1, 0, 2), 5, 1, 0.0), ((8, 0, 0, 8), 2, 1, 0.0)])
def test_dca_steps_match_the_oracle(cl, L, n_spin, h):
    print(f"[dca] steps {cl} L={L} n_spin={n_spin} h={h}", flush=True)
    beta, mu, nf, ncg, ntau = 6.0, -0.3, 48, 1024, 300
    p = dcax.make_dca_params(cluster=cl, t=1.0, tp=-0.15, beta=beta, mu=mu, h=h, n_spin=n_spin, n_freq=nf, n_cg=ncg,
                             n_tau=ntau, patch_points=L)
    g = dcax.DCA(p)
    o = dca.DCA(cl[:2], cl[2:], t=1.0, tp=-0.15, beta=beta, mu=mu, h=h, n_freq=nf, n_cg=ncg, n_tau=ntau, L=L)
    rng = np.random.default_rng(11)
    w = o.w[:nf]
    # a self-energy of the usual shape (constant real part, -i c / w tail),
    # even in K so that G0cal(r, tau) is real
    cx, cy = np.cos(o.K[:, 0]), np.cos(o.K[:, 1])
    sig = []
    for s in range(n_spin):
        a, b = rng.normal(size=3) * 0.3, 0.5 + rng.random(3)
        re = a[0] + a[1] * cx + a[2] * cx * cy
        im = b[0] + 0.3 * b[1] * cy + 0.2 * b[2] * (cx + cy)
        sig.append(re[:, None] - 1j * im[:, None] / (w[None, :] + 0.7))
    sig = np.stack(sig)
    gbar_g, g0_g = g.coarse_grain(_t(sig))
    tab_g = g.g0_tables(g0_g).cpu().numpy()
    errs = []
    for s in range(n_spin):
        gbar_o, g0_o = o.coarse_grain(sig[s], s)
        errs += [_rel(_c(gbar_g)[s], gbar_o), _rel(_c(g0_g)[s], g0_o)]
        tab_o = o.g0_table(g0_o, s)
        errs.append(float(np.max(np.abs(tab_g[s] - tab_o))))
    # cluster G from a seeded two-walker accumulator, then Dyson and mixing
    Mk = rng.normal(size=(2, 2, o.Nc, nf)) + 1j * rng.normal(size=(2, 2, o.Nc, nf))
    aux = np.array([[3.0, 0.1, 0.2], [-1.5, 0.0, 0.0]])
    acc = torch.tensor(np.stack([Mk.real, Mk.imag], axis=-1).reshape(-1), dtype=torch.float64, device="cuda")
    G_g = g.cluster_G(g0_g, acc, torch.tensor(aux, device="cuda"), n_blocks=2)
    Mavg = Mk.sum(axis=0) / aux[:, 0].sum()
    G_o = []
    for s in range(n_spin):
        g0_o = o.coarse_grain(sig[s], s)[1]
        if n_spin == 1:
            G_o.append(np.mean([dca.finalize_G_iw(g0_o, Mavg[sp], beta) for sp in range(2)], axis=0))
        else:
            G_o.append(dca.finalize_G_iw(g0_o, Mavg[s], beta))
        errs.append(_rel(_c(G_g)[s], G_o[s]))
    new_g, chg = g.self_energy(g0_g, G_g, _t(sig), alpha=0.6)
    for s in range(n_spin):
        g0_o = o.coarse_grain(sig[s], s)[1]
        want = dca.DCA.self_energy(g0_o, G_o[s], sig[s], 0.6)
        errs.append(_rel(_c(new_g)[s], want))
    want_chg = np.max(np.abs(_c(new_g) - sig))
    print(f"  max errors: gbar/g0/table/G/sigma {['%.1e' % e for e in errs]}, max change {chg:.4f}", flush=True)
    assert max(errs) < 1e-12
    assert abs(chg - want_chg) <= 1e-14 * want_chg
    g.close()


def test_set_g0_equals_creating_the_walker_with_it():
    print("[dca] set_g0 vs create", flush=True)
    p = dcax.make_dca_params(cluster=(2, 0, 0, 2), beta=5.0, mu=0.0, n_freq=32, n_cg=512, n_tau=400, patch_points=6)
    g = dcax.DCA(p)
    s0 = g.new_sigma()
    s1 = _t(np.tile(-0.4j / (np.pi / 5.0 * (2 * np.arange(32) + 1) + 1.0), (1, 4, 1)))
    pa = g.walker_params(s0, U=4.0, submatrix_k=16, max_order=256, seed=5)
    pb = g.walker_params(s1, U=4.0, submatrix_k=16, max_order=256, seed=5)
    wa, wb = dcax.Walker(pa), dcax.Walker(pb)
    from paper_1901_01047_amd.workloads import initial_config
    start = initial_config(4, 5.0, 30, 3)
    wa.set_config(*start)
    wb.set_config(*start)
    _, g0 = g.coarse_grain(s1)
    wa.set_g0(g.g0_tables(g0), g0)
    assert np.array_equal(wa.g0_table(), wb.g0_table())
    # N from the refresh of the whole handle against set_config's refresh of
    # one walker: the same Gauss-Jordan inversion, within rounding
    for sp in range(2):
        na, nb = wa.copy_N(sp)[1], wb.copy_N(sp)[1]
        assert np.max(np.abs(na - nb)) <= 1e-12 * np.max(np.abs(nb))
    assert wa.stats()["sign"] == wb.stats()["sign"]
    aa, xa = wa.new_accumulator()
    ab, xb = wb.new_accumulator()
    wa.sweep_measure(20, aa, xa)
    wb.sweep_measure(20, ab, xb)
    assert np.array_equal(wa.get_config(), wb.get_config())
    assert float((aa - ab).abs().max()) <= 1e-9 * float(ab.abs().max()) and torch.equal(xa[0], xb[0])
    Ga, _ = wa.finalize(aa, xa)
    Gb, _ = wb.finalize(ab, xb)
    assert float((Ga - Gb).abs().max()) <= 1e-9 * float(Gb.abs().max())
    for w in (wa, wb):
        w.close()
    g.close()


def test_loop_at_u0_keeps_sigma_zero():
    print("[dca] U = 0", flush=True)
    p = dcax.make_dca_params(cluster=(2, 0, 0, 2), beta=4.0, mu=0.2, n_freq=32, n_cg=512, n_tau=300, patch_points=6)
    g = dcax.DCA(p)
    sig = g.new_sigma()
    w = dcax.Walker(g.walker_params(sig, U=0.0, submatrix_k=16, max_order=64, seed=3))
    rep, G = g.iterate(w, sig, warmup_sweeps=5, measure_sweeps=20, want_G=True)
    assert rep["max_change"] == 0.0 and torch.count_nonzero(sig) == 0
    _, g0 = g.coarse_grain(sig)
    assert torch.equal(G, g0[:, :, :32])
    w.close()
    g.close()


def _jack_G(bins):
    """Mean of complex bins and jackknife errors of the real and imaginary
    parts (returned as err.real, err.imag)."""
    arr = np.array(bins)
    n = len(arr)
    mean = arr.mean(axis=0)
    loo = (arr.sum(axis=0)[None] - arr) / (n - 1)
    d = loo - mean[None]
    f = (n - 1) / n
    return mean, np.sqrt(f * np.sum(d.real ** 2, axis=0)) + 1j * np.sqrt(f * np.sum(d.imag ** 2, axis=0))


def test_atomic_limit_iterations_measure_the_atom():
    print("[dca] atomic limit", flush=True)
    U, beta, mu, nf = 2.0, 2.0, 0.3, 16
    p = dcax.make_dca_params(cluster=(1, 0, 0, 1), t=0.0, beta=beta, mu=mu, n_freq=nf, n_cg=2048, n_tau=400,
                             patch_points=4)
    g = dcax.DCA(p)
    sig = g.new_sigma()
    w = dcax.Walker(g.walker_params(sig, U=U, submatrix_k=8, max_order=128, seed=21, warmup_sweeps=200))
    w.sweep(200)
    bins = []
    for it in range(24):
        _, g0 = g.coarse_grain(sig)
        assert np.max(np.abs(_c(g0)[0, 0, :nf] - 1.0 / (1j * np.pi / beta * (2 * np.arange(nf) + 1) + mu))) < 1e-14
        rep, G = g.iterate(w, sig, warmup_sweeps=0, measure_sweeps=250, want_G=True)
        bins.append(_c(G)[0, 0])
        # Dyson: sigma = G0cal^{-1} - G^{-1} (alpha = 1)
        assert np.max(np.abs(_c(sig)[0, 0] - (1.0 / _c(g0)[0, 0, :nf] - 1.0 / bins[-1]))) < 1e-12
    mean, err = _jack_G(bins)
    e = ed.ED(np.zeros((1, 1)), U=U, mu=mu, beta=beta)
    want = e.G_iw(np.array([1.0]), 0, nf)
    z = np.concatenate([np.abs(mean.real - want.real) / np.maximum(err.real, 1e-12),
                        np.abs(mean.imag - want.imag) / err.imag])
    print(f"  points {len(z)}, beyond 3 sigma {(z >= 3).sum()}, max z {z.max():.2f}", flush=True)
    assert (z >= 3).sum() <= max(1, round(0.01 * len(z))) and z.max() < 4.5
    w.close()
    g.close()


def test_first_iteration_2x2_matches_the_oracle_chain():
    """Sigma = 0 -> G0cal of the 2x2 DCA cluster; the GPU walkers and the
    oracle chain each measure G_c on it; the two agree within 3 combined
    sigma at the first 8 frequencies of both K classes."""
    print("[dca] 2x2 first iteration vs the oracle chain", flush=True)
    U, beta, nf, L = 4.0, 5.0, 8, 8
    p = dcax.make_dca_params(cluster=(2, 0, 0, 2), beta=beta, mu=0.0, n_freq=nf, n_cg=1024, n_tau=500, patch_points=L)
    g = dcax.DCA(p)
    sig = g.new_sigma()
    w = dcax.Walker(g.walker_params(sig, U=U, submatrix_k=16, max_order=256, seed=33, warmup_sweeps=100))
    w.sweep(100)
    gpu_bins = []
    for it in range(16):
        s_it = sig.clone()
        rep, G = g.iterate(w, s_it, warmup_sweeps=0, measure_sweeps=200, want_G=True)
        gpu_bins.append(_c(G)[0])
    gm, ge = _jack_G(gpu_bins)
    # the oracle chain on the same G0cal (the oracle's own coarse-graining)
    o = dca.DCA((2, 0), (0, 2), beta=beta, mu=0.0, n_freq=nf, n_cg=1024, n_tau=500, L=L)
    g0o = o.coarse_grain(np.zeros((4, nf)))[1]
    tabo = o.g0_table(g0o)
    m = ctaux.Model(a1=(2, 0), a2=(0, 2), U=U, beta=beta, mu=0.0, n_tau=500, tables=[tabo, tabo])
    ow = ctaux.Walker(m, seed=7, k_s=16)
    for _ in range(60):
        ow.sweep()
    obins = []
    for b in range(12):
        acc = measure.Accumulator(m, nf)
        for _ in range(60):
            ow.sweep()
            acc.measure(ow)
        s, sM, _ = acc.arrays()
        Mavg = sM.sum(axis=0) / s.sum()
        obins.append(np.mean([dca.finalize_G_iw(g0o, Mavg[sp], beta) for sp in range(2)], axis=0))
    om, oe = _jack_G(obins)
    zs = []
    for K in (0, 3):          # K = (0, 0) and (pi, pi); (pi, 0) and (0, pi) as well
        for arr in (np.abs(gm[K].real - om[K].real) / np.hypot(ge[K].real, oe[K].real).clip(1e-12),
                    np.abs(gm[K].imag - om[K].imag) / np.hypot(ge[K].imag, oe[K].imag)):
            zs.append(arr)
    z = np.concatenate(zs)
    print(f"  points {len(z)}, beyond 3 sigma {(z >= 3).sum()}, max z {z.max():.2f}; GPU sign {rep['sign']:.3f}, "
          f"mean order {rep['mean_order']:.1f}", flush=True)
    assert (z >= 3).sum() <= max(1, round(0.01 * len(z))) and z.max() < 4.5
    w.close()
    g.close()


def test_2x2_loop_keeps_particle_hole_symmetry():
    print("[dca] 2x2 loop, four iterations", flush=True)
    U, beta, nf = 4.0, 5.0, 16
    p = dcax.make_dca_params(cluster=(2, 0, 0, 2), beta=beta, mu=0.0, n_freq=nf, n_cg=1024, n_tau=500, patch_points=8)
    g = dcax.DCA(p)
    sig = g.new_sigma()
    w = dcax.Walker(g.walker_params(sig, U=U, submatrix_k=16, max_order=256, seed=44, warmup_sweeps=100))
    w.sweep(100)
    changes = []
    for it in range(4):
        rep, _ = g.iterate(w, sig, warmup_sweeps=20, measure_sweeps=800, alpha=0.7)
        changes.append(rep["max_change"])
    # bins of the converged loop's G_c and Sigma from further iterations at
    # alpha = 1 (G_c is linear in the measured M: its bins are near Gaussian)
    gbins, sbins = [], []
    for it in range(16):
        s = sig.clone()
        _, G = g.iterate(w, s, warmup_sweeps=10, measure_sweeps=200, want_G=True)
        gbins.append(_c(G)[0])
        sbins.append(_c(s)[0])
    gm, ge = _jack_G(gbins)
    sm, se = _jack_G(sbins)
    # particle-hole symmetry at half filling on the bipartite cluster (with
    # the Hartree shift in H0): G(K + Q) = -conj G(K), Q = (pi, pi).  The
    # transformation maps the spin-up matrices of a configuration onto the
    # spin-down ones, so the spin-averaged estimator obeys it for every
    # configuration, to rounding: (0,0) <-> (pi,pi) and (pi,0) <-> (0,pi).
    # The square's symmetry makes G(pi,0) = G(0,pi) on average only, hence
    # Re G(pi,0) = 0 within errors.
    garr = np.array(gbins)
    scale = np.max(np.abs(garr))
    exact = max(np.max(np.abs(garr[:, 0] + np.conj(garr[:, 3]))), np.max(np.abs(garr[:, 1] + np.conj(garr[:, 2]))))
    zz = np.abs(gm[1].real) / ge[1].real.clip(1e-12)
    print(f"  changes {['%.3f' % c for c in changes]}; Sigma(K=(0,0), w_0) = {sm[0, 0]:.4f} +- {se[0, 0]:.4f}, "
          f"Sigma((pi,0), w_0) = {sm[1, 0]:.4f}; |G(K) + conj G(K+Q)| {exact:.1e} (of {scale:.2f}); "
          f"Re G(pi,0) / err: max {zz.max():.2f}", flush=True)
    assert changes[-1] < changes[0]
    assert exact <= 1e-12 * scale
    assert zz.max() < 4.5 and (zz >= 3).sum() <= 1
    assert np.all(sm.imag < 0)
    w.close()
    g.close()

"""The bare propagator at the boundary (MI355X).

Sec. 2.1: in the DCA loop the cluster-excluded G0 is the cluster solver's
input.  A caller passes it as tables G0_sigma(r, tau_l) (one for both spins,
or one per spin) plus G0_sigma(K, i w_n) for the finalisation:

* the library's own isolated-cluster table handed back gives a chain
  bit-identical to the internal one (same configurations, N, accumulators),
  and the same G(K, i w_n) and G(K, tau);
* the oracle's table replays an oracle trace to 1e-10 (ratios, N);
* one table per spin (a Zeeman field splits xi_up and xi_down): an oracle
  trace of the field model replays to 1e-10, the finalisation with the
  caller's per-spin G0(K, i w_n) and the tables' G0(K, tau) equals the
  oracle's on a seeded accumulator, and the GPU's own chain of the atom in a
  field reproduces the exact per-spin G (criterion of the chain tests).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ctaux, ed, g0, measure, stats  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs  # noqa: E402
from tests.ctaux_cases import model, oracle_trace  # noqa: E402


def _replay_errors(w, rec, ratios_o, ow):
    ratios = w.replay(rec)
    good = ~((rec["kind"] == 1) & (rec["id"] < 0))
    rel = np.abs(ratios[good] - ratios_o[good]) / np.abs(ratios_o[good])
    ids_o, Nu, Nd = ow.canonical()
    nerr = 0.0
    for sp, No in ((0, Nu), (1, Nd)):
        ids, N = w.copy_N(sp)
        assert np.array_equal(ids, ids_o)
        nerr = max(nerr, float(np.max(np.abs(N - No)) / np.max(np.abs(No))))
    return float(rel.max()), nerr


def test_own_table_handed_back_gives_the_same_chain():
    name = "4x4_U4_b10"
    print(f"[g0 boundary] {name}: internal table handed back", flush=True)
    nf = 64
    # half filling: no sign problem, so a short run has a nonzero sign sum
    kw = params_kwargs(name, n_freq=nf, warmup_sweeps=4, mu=0.0)
    m = model(name, mu=0.0)
    w_in = dcax.Walker(dcax.make_params(**kw))
    tab = w_in.g0_table()
    w_ex = dcax.Walker(dcax.make_params(**kw, g0_tau=tab, g0_Kw=g0.g0_K_iw(m.xi, nf, m.beta)))
    assert np.array_equal(w_ex.g0_table(), tab)
    c = CONFIGS[name]
    start = initial_config(m.Nc, m.beta, 200, c["seed"] + 55)
    accs = []
    for w in (w_in, w_ex):
        w.set_config(*start)
        acc, aux = w.new_accumulator()
        w.sweep_measure(8, acc, aux)
        accs.append((acc, aux))
    assert np.array_equal(w_in.get_config(), w_ex.get_config())
    for sp in range(2):
        assert np.array_equal(w_in.copy_N(sp)[1], w_ex.copy_N(sp)[1])
    assert torch.equal(accs[0][0], accs[1][0]) and torch.equal(accs[0][1], accs[1][1])
    (Gi, Ti), (Ge, Te) = (w.finalize(a, x, n_tau_out=33) for w, (a, x) in zip((w_in, w_ex), accs))
    eg = float((Gi - Ge).abs().max() / Gi.abs().max())
    et = float((Ti - Te).abs().max())
    # G0(K, tau) from the caller's table is the linear interpolant of the
    # closed form (interpolation is linear, so the sum over r commutes with
    # it): off the grid it differs by at most h^2/8 max|G0''| = h^2/8 xi_K^2
    h = m.beta / (m.n_tau - 1)
    bound = h * h / 8 * float(np.max(m.xi ** 2)) + 1e-12
    print(f"  identical chain; finalize G(K,iw) diff {eg:.1e}, G(K,tau) diff {et:.1e} (bound {bound:.1e})",
          flush=True)
    assert eg < 1e-13 and et < bound
    w_in.close()
    w_ex.close()


def test_oracle_table_replays_an_oracle_trace():
    name = "4x4_U4_b10"
    print(f"[g0 boundary] {name}: the oracle's table", flush=True)
    m = model(name)
    init, rec, ratios_o, ow = oracle_trace(m, seed=CONFIGS[name]["seed"] + 9, k_s=32, init_order=0,
                                           init=initial_config(m.Nc, m.beta, 220, 17), warm_sweeps=2,
                                           rec_proposals=400)
    w = dcax.Walker(dcax.make_params(**params_kwargs(name, submatrix_k=32), g0_tau=m.table))
    w.set_config(*init)
    rel, nerr = _replay_errors(w, rec, ratios_o, ow)
    print(f"  ratios max rel err {rel:.2e}, N normwise {nerr:.2e}", flush=True)
    assert rel <= 1e-10 and nerr <= 1e-10
    assert w.stats()["decision_mismatches"] == 0
    with pytest.raises(dcax.DcaxError):     # no G0(K, i w_n) given: finalize cannot run
        acc, aux = w.new_accumulator()
        w.finalize(acc, aux)
    w.close()


def _field_model(U=4.0, beta=5.0, mu=0.2, h=0.4, a=(2, 0, 0, 2), n_tau=1000):
    return ctaux.Model(a1=a[:2], a2=a[2:], t=1.0 if a != (1, 0, 0, 1) else 0.0, U=U, beta=beta, mu=mu, h=h,
                       n_tau=n_tau)


def _field_params(m, cluster, nf, **kw):
    tabs = np.stack(m.tables)
    gkw = np.stack([g0.g0_K_iw(m.xis[sp], nf, m.beta) for sp in range(2)])
    return dcax.make_params(cluster=cluster, U=m.U, beta=m.beta, K_exp=m.K_exp, n_tau=m.n_tau, n_freq=nf,
                            g0_tau=tabs, g0_Kw=gkw, **kw)


def test_per_spin_tables_replay_and_finalize():
    print("[g0 boundary] 2x2 in a field: one table per spin", flush=True)
    m = _field_model()
    assert np.max(np.abs(m.tables[0] - m.tables[1])) > 1e-2
    init, rec, ratios_o, ow = oracle_trace(m, seed=77, k_s=16, init_order=20, warm_sweeps=20, rec_proposals=600)
    nf = 48
    w = dcax.Walker(_field_params(m, (2, 0, 0, 2), nf, submatrix_k=16, max_order=256))
    w.set_config(*init)
    rel, nerr = _replay_errors(w, rec, ratios_o, ow)
    print(f"  ratios max rel err {rel:.2e}, N normwise {nerr:.2e}", flush=True)
    assert rel <= 1e-10 and nerr <= 1e-10
    # the finalisation on a seeded accumulator against the oracle's per-spin G0
    rng = np.random.default_rng(8)
    Mk = (rng.normal(size=(2, m.Nc, nf)) + 1j * rng.normal(size=(2, m.Nc, nf))) * 0.3
    aux = np.array([0.7, 0.33, -0.12])
    acc = torch.tensor(np.stack([Mk.real, Mk.imag], axis=-1) * aux[0], device="cuda")
    taus = np.linspace(0.0, m.beta, 21)
    Giw, Gt = w.finalize(acc, torch.tensor(aux, device="cuda"), n_tau_out=21)
    Giw = Giw.cpu().numpy()
    Giw = Giw[..., 0] + 1j * Giw[..., 1]
    Gt = Gt.cpu().numpy()
    for sp in range(2):
        eg = np.max(np.abs(Giw[sp] - measure.finalize_G_iw(m, Mk[sp], nf, spin=sp)))
        # G0(K, tau) comes from the linearly interpolated tables (the oracle's
        # closed form differs by the interpolation error, ~(beta/n_tau)^2)
        et = np.max(np.abs(Gt[sp] - measure.G_tau_from_iw(m, Mk[sp], aux[1 + sp] / aux[0], nf, taus, spin=sp)))
        print(f"  spin {sp}: finalize G(K,iw) err {eg:.1e}, G(K,tau) err {et:.1e}", flush=True)
        assert eg < 1e-13 and et < 1e-4
    w.close()


def test_atom_in_a_field_chain_vs_exact():
    """The GPU chain with one table per spin against the four-state exact G
    per spin (beta U = 4: the chain flips the atom's moment often)."""
    print("[g0 boundary] atom in a field: GPU chain vs exact", flush=True)
    m = _field_model(U=2.0, beta=2.0, mu=0.3, h=0.5, a=(1, 0, 0, 1), n_tau=400)
    nf, B, per = 256, 32, 250
    w = dcax.Walker(_field_params(m, (1, 0, 0, 1), nf, submatrix_k=8, max_order=128, seed=91, warmup_sweeps=200,
                                  t=0.0))
    w.sweep(200)
    bins = []
    for _ in range(B):
        acc, aux = w.new_accumulator()
        w.sweep_measure(per, acc, aux)
        a = acc.cpu().numpy()
        bins.append((a[..., 0] + 1j * a[..., 1], aux.cpu().numpy().copy()))
    sM = np.array([x[0] for x in bins])
    sA = np.array([x[1] for x in bins])
    e = ed.ED(np.zeros((1, 1)), U=m.U, mu=m.mu, beta=m.beta, h=m.h)
    taus = np.linspace(0.1, m.beta - 0.1, 10)
    zs = []
    for sp in range(2):
        g_iw, err_iw = stats.jackknife(lambda M, A: measure.finalize_G_iw(m, (M / A[0])[sp][:, :16], 16, spin=sp),
                                       (sM, sA))
        g_t, err_t = stats.jackknife(
            lambda M, A: measure.G_tau_from_iw(m, (M / A[0])[sp], A[1 + sp] / A[0], nf, taus, spin=sp), (sM, sA))
        want = e.G_iw(np.array([1.0]), sp, 16)
        zs.append(np.abs(g_iw[0].real - want.real) / np.maximum(err_iw[0].real, 1e-12))
        zs.append(np.abs(g_iw[0].imag - want.imag) / err_iw[0].imag)
        zs.append(np.abs(g_t[0] - e.G_tau(np.array([1.0]), sp, taus)) / err_t[0])
    z = np.concatenate(zs)
    n_out = int((z >= 3).sum())
    print(f"  points {len(z)}, beyond 3 sigma {n_out}, max z {z.max():.2f}", flush=True)
    assert n_out <= max(1, round(0.01 * len(z))) and z.max() < 4.5
    w.close()

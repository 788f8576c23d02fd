"""Spin-flip proposals and the treatments of a spin touched twice (MI355X).

Sec. 2.3 shows the CT-AUX moves (insertion, removal and the flip of an
auxiliary spin) and lists the treatments of a spin that one submatrix
window touches twice; App. B names the neglect-Bennett-updates option.

* Replay: an oracle trace with a share of flips (ratios by the matrix
  determinant lemma, N by Sherman-Morrison), replayed with forced decisions,
  gives every ratio within 1e-10 kappa of the FP64 oracle and of the
  extended-precision chain, and N within 1e-10 normwise (2x2, and 4x4 with
  windows of 32 and 64; a window ends before a second change of one spin).
  kappa is 1 for insertions and removals; a flip ratio is the difference
  (1 + e^{-V_p}) N_pp - e^{-V_p} per spin, and kappa is its condition number
  with respect to N_pp (tests/ctaux_cases.py), which no FP64 evaluation
  escapes: the FP64 oracle's own error against extended precision scales
  with it.
* The GPU's own chain with flips (exact treatment) reproduces exact
  diagonalisation: the 2x2 cluster at half filling, and the atom in a field
  per spin, by the criterion of the chain tests.
* The neglect treatment (a proposal touching a spin the window already
  changed is rejected) breaks detailed balance; its bias on the same 2x2
  observables is measured and printed, against the exact treatment's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ctaux, ed, g0, geometry, measure, stats  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs  # noqa: E402
from tests.ctaux_cases import exact_replay_with_flip_conditioning, model, records  # noqa: E402


def _flip_trace(m, seed, k_s, init_order, warm, n_rec, p_flip):
    """An oracle trace with flips from the aligned-spin start (a
    well-conditioned state: random auxiliary spins give N whose ratios
    neither FP64 evaluation reaches to 1e-10)."""
    w = ctaux.Walker(m, seed=seed, k_s=k_s, p_flip=p_flip)
    w.set_config(*initial_config(m.Nc, m.beta, init_order, 17))
    for _ in range(warm):
        w.sweep()
    w.refresh()
    init = (w.r.copy(), w.t.copy(), w.s.copy(), w.id.copy())
    w.record = True
    for _ in range(n_rec):
        w.step()
    rec, ratios = records(w.trace)
    return init, rec, ratios, w


@pytest.mark.parametrize("name,k_s,k_init,warm,n_rec,seed", [("2x2_U4_b5", 16, 20, 20, 800, 3),
                                                             ("4x4_U4_b10", 32, 220, 2, 600, 3),
                                                             ("4x4_U4_b10", 64, 220, 2, 600, 3),
                                                             ("4x4_U4_b10", 64, 280, 6, 600, 6)])
def test_flip_replay_parity(name, k_s, k_init, warm, n_rec, seed):
    print(f"[flips] replay {name} k_s={k_s} seed offset {seed}", flush=True)
    m = model(name)
    init, rec, ratios_o, ow = _flip_trace(m, CONFIGS[name]["seed"] + seed, k_s, k_init, warm, n_rec, 0.3)
    n_flip = int((rec["kind"] == 2).sum())
    assert n_flip > 0.2 * n_rec
    w = dcax.Walker(dcax.make_params(**params_kwargs(name, submatrix_k=k_s)))
    w.set_config(*init)
    ratios = w.replay(rec)
    good = ~((rec["kind"] >= 1) & (rec["id"] < 0))
    assert np.all(ratios[~good] == 0.0)
    rx, ch, kap = exact_replay_with_flip_conditioning(m, init, rec)
    kap = kap[good]
    rel = np.abs(ratios[good] - ratios_o[good]) / np.abs(ratios_o[good]) / kap
    rel_x = np.abs(ratios[good] - rx[good]) / np.abs(rx[good]) / kap
    ids_o, Nu, Nd = ow.canonical()
    ids_x, Xu, Xd = ch.canonical()
    nerr = nerr_x = 0.0
    for sp, No, Nx in ((0, Nu, Xu), (1, Nd, Xd)):
        ids, N = w.copy_N(sp)
        assert np.array_equal(ids, ids_o) and np.array_equal(ids, ids_x)
        nerr = max(nerr, float(np.max(np.abs(N - No)) / np.max(np.abs(No))))
        nerr_x = max(nerr_x, float(np.max(np.abs(N.astype(np.longdouble) - Nx)) / np.max(np.abs(Nx))))
    cfg = w.get_config()
    o = np.argsort(ow.id)
    assert np.array_equal(np.sort(cfg["id"]), ow.id[o])
    assert np.array_equal(cfg["aux_spin"][np.argsort(cfg["id"])], ow.s[o])
    st = w.stats()
    print(f"  {n_flip} flip proposals ({st['accepted_flips']} accepted), windows {st['windows']}, "
          f"closed early {st['aborted_windows']}; ratios max rel err / kappa vs FP64 oracle {rel.max():.2e}, vs "
          f"extended precision {rel_x.max():.2e} (kappa up to {kap.max():.0f}; insertions and removals "
          f"{rel_x[rec['kind'][good] != 2].max():.2e}); N normwise {nerr:.2e} / {nerr_x:.2e}", flush=True)
    assert rel.max() <= 1e-10 and nerr <= 1e-10
    assert rel_x.max() <= 1e-10 and nerr_x <= 1e-10
    assert st["decision_mismatches"] == 0
    assert st["accepted_flips"] == int(((rec["kind"] == 2) & (rec["accepted"] == 1)).sum())
    assert w.refresh() < 1e-10
    w.close()


def _chain_vs_ed(flip_share, touched_twice, k_s=16, B=32, per=100, nf=512, seed_offset=0):
    name = "2x2_U4_b5"
    kw = params_kwargs(name, n_freq=nf, submatrix_k=k_s)
    kw["seed"] += seed_offset
    w = dcax.Walker(dcax.make_params(**kw, refresh_every=50, flip_share=flip_share, touched_twice=touched_twice))
    m = model(name)
    w.sweep(100)
    accs = []
    for _ in range(B):
        acc, aux = w.new_accumulator()
        w.sweep_measure(per, acc, aux)
        a = acc.cpu().numpy()
        accs.append((a[..., 0] + 1j * a[..., 1], aux.cpu().numpy().copy()))
    sM = np.array([x[0] for x in accs])
    sA = np.array([x[1] for x in accs])
    e = ed.ED(geometry.hopping_matrix(m.a1, m.a2), U=m.U, mu=m.mu, beta=m.beta)
    ph = ed.momentum_phases(m.sites, m.K)
    taus = np.linspace(0.05, m.beta - 0.05, 20)
    g_iw, err_iw = stats.jackknife(
        lambda M, A: np.mean([measure.finalize_G_iw(m, (M / A[0])[sp][:, :24], 24) for sp in range(2)], axis=0),
        (sM, sA))
    g_t, err_t = stats.jackknife(
        lambda M, A: np.mean([measure.G_tau_from_iw(m, (M / A[0])[sp], A[1 + sp] / A[0], nf, taus)
                              for sp in range(2)], axis=0), (sM, sA))
    zs = []
    for iK in range(2):
        want = e.G_iw(ph[iK], 0, 24)
        zs.append(np.abs(g_iw[iK].real - want.real) / np.maximum(err_iw[iK].real, 1e-12))
        zs.append(np.abs(g_iw[iK].imag - want.imag) / err_iw[iK].imag)
        zs.append(np.abs(g_t[iK] - e.G_tau(ph[iK], 0, taus)) / err_t[iK])
    return w, np.concatenate(zs)


def test_chain_with_flips_vs_ed():
    print("[flips] 2x2 chain with flips (exact treatment) vs ED", flush=True)
    w, z = _chain_vs_ed(0.3, 0)
    st = w.stats()
    n_out = int((z >= 3).sum())
    print(f"  points {len(z)}, beyond 3 sigma {n_out}, max z {z.max():.2f}; accepted flips {st['accepted_flips']}, "
          f"windows closed early {st['aborted_windows']} of {st['windows']}", flush=True)
    assert st["accepted_flips"] > 1000 and st["neglected"] == 0
    assert n_out <= max(1, round(0.01 * len(z))) and z.max() < 4.5
    assert w.refresh() < 1e-10
    w.close()


def test_neglect_treatment_bias_is_measured():
    """The neglect treatment on the same observables, with windows of 64
    proposals (many second touches).  Its deviation from exact
    diagonalisation is reported beside the exact treatment's at the same
    window size; only the bookkeeping is asserted (the bias is the result)."""
    print("[flips] neglect treatment, k_s = 64", flush=True)
    out = {}
    for tt in (0, 1):
        w, z = _chain_vs_ed(0.3, tt, k_s=64, seed_offset=11)
        st = w.stats()
        out[tt] = (z, st)
        print(f"  touched_twice={tt}: points {len(z)}, beyond 3 sigma {int((z >= 3).sum())}, max z {z.max():.2f}, "
              f"mean z^2 {np.mean(z ** 2):.2f}; neglected {st['neglected']} of {st['proposals']} proposals, "
              f"windows closed early {st['aborted_windows']}", flush=True)
        assert w.refresh() < 1e-10
        w.close()
    assert out[0][1]["neglected"] == 0 and out[1][1]["neglected"] > 0
    assert out[1][1]["aborted_windows"] < out[0][1]["aborted_windows"]


def test_atom_in_a_field_with_flips_vs_exact():
    print("[flips] atom in a field with flips vs exact", flush=True)
    U, beta, mu, h = 2.0, 2.0, 0.3, 0.5
    m = ctaux.Model(a1=(1, 0), a2=(0, 1), t=0.0, U=U, beta=beta, mu=mu, h=h, n_tau=400)
    nf, B, per = 256, 32, 250
    tabs = np.stack(m.tables)
    gkw = np.stack([g0.g0_K_iw(m.xis[sp], nf, m.beta) for sp in range(2)])
    w = dcax.Walker(dcax.make_params(cluster=(1, 0, 0, 1), U=U, beta=beta, n_tau=m.n_tau, n_freq=nf, submatrix_k=8,
                                     max_order=128, seed=93, warmup_sweeps=200, g0_tau=tabs, g0_Kw=gkw,
                                     flip_share=0.3))
    w.sweep(200)
    bins = []
    for _ in range(B):
        acc, aux = w.new_accumulator()
        w.sweep_measure(per, acc, aux)
        a = acc.cpu().numpy()
        bins.append((a[..., 0] + 1j * a[..., 1], aux.cpu().numpy().copy()))
    sM = np.array([x[0] for x in bins])
    sA = np.array([x[1] for x in bins])
    e = ed.ED(np.zeros((1, 1)), U=U, mu=mu, beta=beta, h=h)
    taus = np.linspace(0.1, beta - 0.1, 10)
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
    st = w.stats()
    n_out = int((z >= 3).sum())
    print(f"  points {len(z)}, beyond 3 sigma {n_out}, max z {z.max():.2f}; accepted flips {st['accepted_flips']}",
          flush=True)
    assert st["accepted_flips"] > 1000
    assert n_out <= max(1, round(0.01 * len(z))) and z.max() < 4.5
    w.close()

"""Parity of the HIP path with the oracle, through the C ABI (MI355X).

* G0(r, tau) table against the oracle's table;
* refresh (FP64 Gauss-Jordan) against direct inversion;
* replay of oracle traces with forced decisions: every ratio and N against
  the oracle and against the same chain replayed in extended precision
  (oracle/exact.py, pinned against 40-digit determinants), same vertex ids,
  no decision on the other side of |R|;
* the measurement M(K, i w_n) of a fixed configuration, and the finalisation
  G = G0 - G0 <M> G0 / beta, against the oracle's direct sums;
* error paths that the host can force (unknown replay id, latched state).

Tolerances (FP64):
* ratios: |R - R_ref| <= 1e-10 |R_ref| for every ratio, with R_ref the
  extended-precision value and, separately, the FP64 oracle's (both the
  oracle and the kernels' submatrix algebra land within ~1e-11 of the
  extended-precision chain on these states);
* N: max|N - N_ref| <= 1e-10 max|N_ref| against both (rows of N span
  e^{+-gamma}, so the elementwise relative error is ill-posed);
* measurement: the contraction of the walker's own M against the oracle's
  direct sums, relative to the scale of its summands, (1/Nc) sum |M_ij| (the
  result can be far smaller after cancellation), within
  eps (4 w_max beta + 4 k): the rounding of the phase arguments w_n tau plus
  the sums; and against the oracle's N within the N difference it carries;
* finalisation: 1e-13 absolute on G(K, i w_n), 1e-11 on G(K, tau).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ctaux, exact, measure  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, params_kwargs  # noqa: E402
from tests.ctaux_cases import model, oracle_trace  # noqa: E402


def walker(name, precision=None, **over):
    extra = {} if precision is None else {"precision": precision}
    p = dcax.make_params(**params_kwargs(name, **over), **extra)
    return dcax.Walker(p)


def rel_norm(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("name", ["2x2_U4_b5", "4x4_U4_b10", "6x6_U6_b20"])
def test_g0_table(name):
    print(f"[g0 table] {name}", flush=True)
    m = model(name)
    w = walker(name, max_order=64)
    t = w.g0_table()
    e = np.max(np.abs(t - m.table))
    print(f"  max |G0 table - oracle table| {e:.2e}", flush=True)
    assert e < 1e-13
    w.close()


@pytest.mark.parametrize("name,k", [("2x2_U4_b5", 30), ("4x4_U4_b10", 300), ("4x4_U4_b10", 77),
                                    ("4x4_U4_b10", 700), ("6x6_U6_b20", 1030)])
def test_refresh_equals_direct_inverse(name, k):
    """Random (unequilibrated) configurations can be very ill-conditioned, so
    the GJ inverse is checked by its backward residual |A N - 1| / (|A| |N|)
    and against NumPy's LU inverse within 20 cond(A) eps.  Orders above 1024
    take the column-step panel form (with a narrower last panel here)."""
    print(f"[refresh] {name} k={k}", flush=True)
    m = model(name)
    ow = ctaux.Walker(m, seed=7)
    ow.random_config(k)
    w = walker(name, max_order=max(1024, k + 64))
    w.set_config(ow.r, ow.t, ow.s, ow.id)
    assert w.order == k
    ids_o, Nu, Nd = ow.canonical()
    o = np.argsort(ow.id)
    for sp in range(2):
        ids, N = w.copy_N(sp)
        assert np.array_equal(ids, ids_o)
        A = ctaux.n_inverse(m, ow.r[o], ow.t[o], ow.s[o], sp)
        res = np.max(np.abs(A @ N - np.eye(k))) / (np.max(np.abs(A)) * np.max(np.abs(N)) * k)
        cond = np.linalg.cond(A)
        e = rel_norm(N, Nu if sp == 0 else Nd)
        print(f"  spin {sp}: residual {res:.2e}, cond {cond:.1e}, diff vs LU {e:.2e}", flush=True)
        assert res < 1e-15
        assert e < max(1e-12, 20 * cond * np.finfo(float).eps)
    assert w.stats()["sign"] == ow.sign
    assert w.refresh() < 1e-9
    w.close()


REPLAY_CASES = [
    # name, k_s, initial order, warm-up sweeps, recorded proposals
    ("2x2_U4_b5", 16, 20, 30, 800),
    ("2x2_U4_b5", 1, 20, 30, 120),
    ("2x2_U4_b5", 64, 20, 30, 800),
    ("4x4_U4_b10", 32, 280, 10, 700),
    ("4x4_U4_b10", 64, 280, 10, 700),
]


def check_replay(m, init, rec, ratios_o, ow, ratios, w, tol=1e-10):
    """Every ratio and both N against the FP64 oracle and the extended-precision
    replay of the same records; returns the largest relative errors."""
    noop = (rec["kind"] == 1) & (rec["id"] < 0)
    good = ~noop
    assert np.all(ratios[noop] == 0.0)
    rx, ch = exact.replay(m, init, rec)
    rg, ro, re_ = ratios[good], ratios_o[good], rx[good]
    rel_x = np.abs(rg - re_) / np.abs(re_)
    rel_o = np.abs(rg - ro) / np.abs(ro)
    orc_x = np.abs(ro - re_) / np.abs(re_)
    print(f"  ratios ({good.sum()}): max rel err vs extended precision {rel_x.max():.2e} (median "
          f"{np.median(rel_x):.1e}), vs FP64 oracle {rel_o.max():.2e}; oracle vs extended {orc_x.max():.2e}",
          flush=True)
    assert rel_x.max() <= tol, rel_x.max()
    assert rel_o.max() <= tol, rel_o.max()
    ids_x, Xu, Xd = ch.canonical()
    ids_o, Nu, Nd = ow.canonical()
    assert np.array_equal(ids_x, ids_o)
    errs = []
    for sp, No, Nx in ((0, Nu, Xu), (1, Nd, Xd)):
        ids, N = w.copy_N(sp)
        assert np.array_equal(ids, ids_o)
        ex = float(np.max(np.abs(N.astype(np.longdouble) - Nx)) / np.max(np.abs(Nx)))
        eo = rel_norm(N, No)
        print(f"  N[{sp}] normwise err vs extended precision {ex:.2e}, vs oracle {eo:.2e} (k={len(ids)})",
              flush=True)
        assert ex <= tol and eo <= tol
        errs.append(ex)
    return rel_x.max(), max(errs)


@pytest.mark.parametrize("variant", [0, dcax.DCAX_VARIANT_TILED, dcax.DCAX_VARIANT_NARROW])
@pytest.mark.parametrize("name,k_s,k_init,warm,n_rec", REPLAY_CASES)
def test_replay_parity(name, k_s, k_init, warm, n_rec, variant):
    """Each case with the candidate products in the form its launch size
    picks and in the two other forms (every form must reach the oracle)."""
    print(f"[replay] {name} k_s={k_s} k_init={k_init} n={n_rec} variant {variant}", flush=True)
    m = model(name)
    init, rec, ratios_o, ow = oracle_trace(m, seed=CONFIGS[name]["seed"], k_s=k_s, init_order=k_init,
                                           warm_sweeps=warm, rec_proposals=n_rec)
    w = walker(name, submatrix_k=k_s)
    w.set_variants(variant, variant)
    w.set_config(*init)
    ratios = w.replay(rec)
    check_replay(m, init, rec, ratios_o, ow, ratios, w)
    st = w.stats()
    assert st["decision_mismatches"] == 0
    assert st["accepted_insertions"] == int(((rec["kind"] == 0) & (rec["accepted"] == 1)).sum())
    assert st["sign"] == ow.sign
    assert w.refresh() < 1e-10
    w.close()


def test_replay_from_empty_configuration():
    print("[replay] empty start", flush=True)
    m = model("2x2_U4_b5")
    ow = ctaux.Walker(m, seed=3, k_s=8, record=True)
    for _ in range(300):
        ow.step()
    from tests.ctaux_cases import records
    rec, ratios_o = records(ow.trace)
    assert ((rec["kind"] == 1) & (rec["id"] < 0)).any()      # removals at k = 0 occur
    w = walker("2x2_U4_b5", submatrix_k=8)
    ratios = w.replay(rec)
    empty = (np.zeros(0, np.int64), np.zeros(0), np.zeros(0, np.int64), np.zeros(0, np.int64))
    check_replay(m, empty, rec, ratios_o, ow, ratios, w)
    w.close()


# (2x2, k = 600): site buckets of ~150 rows, so the contraction takes b's
# columns in several register chunks (128 in FP32, 64 in FP64); (8x8, k = 24):
# most sites hold no vertex (empty buckets on either side of a pair)
@pytest.mark.parametrize("name,k,precision,max_order", [
    ("2x2_U4_b5", 25, "fp64", None), ("4x4_U4_b10", 300, "fp64", None),
    ("2x2_U4_b5", 600, "fp64", 1024), ("2x2_U4_b5", 600, "mixed", 1024),
    ("8x8_U7_b30", 24, "fp64", None), ("8x8_U7_b30", 24, "mixed", None)])
def test_measurement_matches_direct_sums(name, k, precision, max_order):
    print(f"[measure] {name} k={k} {precision}", flush=True)
    m = model(name)
    ow = ctaux.Walker(m, seed=11)
    ow.random_config(k)
    nf = CONFIGS[name]["n_freq"]
    over = {} if max_order is None else {"max_order": max_order}
    if precision == "mixed":
        over["precision"] = dcax.DCAX_FP32_MIXED
    w = walker(name, **over)
    w.set_config(ow.r, ow.t, ow.s, ow.id)
    acc, aux = w.new_accumulator()
    w.measure(acc, aux)
    w.measure(acc, aux)          # accumulates: twice the single measurement
    got = acc.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    o = np.argsort(ow.id)
    r, t, s = np.asarray(ow.r)[o], np.asarray(ow.t)[o], np.asarray(ow.s)[o]
    for sp in range(2):
        # the contraction alone: the oracle's direct sums over the walker's own
        # N (its N comes from its own FP64 inversion, whose difference from the
        # oracle's N is cond(N) eps, 1e9 eps on unequilibrated configurations)
        ids, Ng = w.copy_N(sp)
        assert np.array_equal(ids, np.asarray(ow.id)[o])
        Mg = (m.ev(s, sp) - 1.0)[:, None] * Ng
        want = 2 * ow.sign * measure.M_K_iw(m, r, t, Mg, nf)
        # M(K, i w_n) sums k^2 terms of size |M_ij| with strong cancellation on
        # unequilibrated configurations: the scale of its rounding error is
        # the sum of the magnitudes, 2 (1/Nc) sum_ij |M_ij|, not |M(K, i w_n)|.
        # Each phase e^{i w_n tau} carries the rounding of its argument,
        # eps * w_n * tau <= eps * w_max * beta (6.4e3 for 1024 frequencies at
        # beta = 5), once for the row and once for the column; the sums add
        # O(k) eps.  Bound: eps * (4 w_max beta + 4 k).
        scale = 2 * np.abs(Mg).sum() / m.Nc
        e = np.max(np.abs(got[sp] - want)) / scale
        w_max_beta = (2 * nf - 1) * np.pi
        # FP32-mixed: the sorted copy, the phases and the products are FP32
        eps = np.finfo(np.float32 if precision == "mixed" else np.float64).eps
        tol = eps * (4 * w_max_beta + 4 * k)
        print(f"  spin {sp}: err / sum|M| {e:.2e} (bound {tol:.1e}), err / max|result| "
              f"{np.max(np.abs(got[sp] - want)) / np.max(np.abs(want)):.2e}", flush=True)
        assert e < tol
        # end to end against the oracle's own N: the N difference enters linearly
        M = measure.M_matrix(m, ow, sp)[np.ix_(o, o)]
        want_o = 2 * ow.sign * measure.M_K_iw(m, r, t, M, nf)
        bound = 2 * np.abs(Mg - M).sum() / m.Nc + tol * scale
        e_o = np.max(np.abs(got[sp] - want_o))
        print(f"  spin {sp}: vs oracle N {e_o:.2e} (bound {bound:.1e})", flush=True)
        assert e_o <= bound
        d = aux.cpu().numpy()[1 + sp]
        tr_tol = 4 * k * np.finfo(float).eps * 2 * np.abs(np.diag(Mg)).sum() / m.Nc
        assert abs(d - 2 * ow.sign * np.trace(Mg) / m.Nc) <= tr_tol
        assert abs(d - 2 * ow.sign * np.trace(M) / m.Nc) <= tr_tol + 2 * np.abs(np.diag(Mg - M)).sum() / m.Nc
    assert aux.cpu().numpy()[0] == 2 * ow.sign
    w.close()


def test_finalize_matches_oracle():
    print("[finalize]", flush=True)
    name = "2x2_U4_b5"
    m = model(name)
    nf = CONFIGS[name]["n_freq"]
    w = walker(name)
    rng = np.random.default_rng(5)
    Mk = (rng.normal(size=(2, m.Nc, nf)) + 1j * rng.normal(size=(2, m.Nc, nf))) * 0.3
    aux = np.array([0.8, 0.21, -0.13])
    acc = np.stack([Mk.real, Mk.imag], axis=-1) * aux[0]
    acc_t = torch.tensor(acc, device="cuda")
    aux_t = torch.tensor(aux, device="cuda")
    taus = np.linspace(0.0, m.beta, 41)
    Giw, Gt = w.finalize(acc_t, aux_t, n_tau_out=41)
    Giw = Giw.cpu().numpy()
    Giw = Giw[..., 0] + 1j * Giw[..., 1]
    Gt = Gt.cpu().numpy()
    for sp in range(2):
        want = measure.finalize_G_iw(m, Mk[sp], nf)
        assert np.max(np.abs(Giw[sp] - want)) < 1e-13
        want_t = measure.G_tau_from_iw(m, Mk[sp], aux[1 + sp] / aux[0], nf, taus)
        assert np.max(np.abs(Gt[sp] - want_t)) < 1e-11
    w.close()


def test_unknown_replay_id_latches_trace_error():
    print("[errors] unknown id", flush=True)
    m = model("2x2_U4_b5")
    ow = ctaux.Walker(m, seed=1)
    ow.random_config(10)
    w = walker("2x2_U4_b5")
    w.set_config(ow.r, ow.t, ow.s, ow.id)
    rec = np.zeros(3, dcax.PROPOSAL_DTYPE)
    rec["kind"] = 1
    rec["id"] = [3, 12345, 4]
    rec["u_accept"] = 0.5
    with pytest.raises(dcax.DcaxError) as e:
        w.replay(rec)
    assert e.value.status == -6
    with pytest.raises(dcax.DcaxError) as e:
        w.sweep(1)
    assert e.value.status == -7
    w.set_config(ow.r, ow.t, ow.s, ow.id)    # clears the latched error
    w.sweep(1)
    w.close()


def test_invalid_replay_records_rejected_on_host():
    w = walker("2x2_U4_b5")
    rec = np.zeros(1, dcax.PROPOSAL_DTYPE)
    rec["kind"] = 0
    rec["site"] = 9           # outside the 4-site cluster
    rec["aux_spin"] = 1
    with pytest.raises(dcax.DcaxError) as e:
        w.replay(rec)
    assert e.value.status == -1
    w.sweep(1)                 # nothing was enqueued; the walker is still usable
    w.close()

"""Submatrix size and its autotuner (MI355X).

Submatrix updates regroup single-vertex updates exactly (§2.3), so the
submatrix size k_s changes neither the ratios nor N of a given sequence of
proposals beyond rounding: one recorded oracle chain replayed with every
size the autotuner can pick gives the same ids, decisions and N.  (With
generated proposals the chains agree in distribution, not path by path: a
removal target is drawn among the vertices present at the window start, so
the same uniforms can name different vertices under different k_s.)  The
autotuner (dcax_autotune) times the candidate sizes on the live chain and
keeps the fastest; the chain stays valid throughout.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, params_kwargs  # noqa: E402
from tests.ctaux_cases import model, oracle_trace  # noqa: E402

CANDIDATES = (8, 16, 24, 32, 48, 64)


def initial(n, Nc, beta, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, Nc, size=n).astype(np.int32), rng.random(n) * beta,
            np.where(rng.random(n) < 0.5, 1, -1).astype(np.int32))


def test_submatrix_size_does_not_change_a_replayed_chain():
    name = "4x4_U4_b10"
    print(f"[k_s] one recorded chain replayed with k_s in {CANDIDATES}", flush=True)
    m = model(name)
    init, rec, ratios_o, ow = oracle_trace(m, seed=CONFIGS[name]["seed"] + 5, k_s=16, init_order=240,
                                           warm_sweeps=4, rec_proposals=600)
    good = ~((rec["kind"] == 1) & (rec["id"] < 0))
    ids_o = ow.canonical()[0]
    res = {}
    for ks in CANDIDATES:
        w = dcax.Walker(dcax.make_params(**params_kwargs(name, submatrix_k=ks)))
        w.set_config(*init)
        r = w.replay(rec)
        st = w.stats()
        res[ks] = (r, w.copy_N(0), w.copy_N(1), st)
        print(f"  k_s {ks}: {st['windows']} windows, order {w.order}", flush=True)
        assert st["decision_mismatches"] == 0
        w.close()
    r0, (i0u, N0u), (i0d, N0d), s0 = res[CANDIDATES[0]]
    for ks in CANDIDATES[1:]:
        r, (iu, Nu), (id_, Nd), st = res[ks]
        # ratios on the decision scale of the replay parity tests
        scaled = np.abs(r[good] - r0[good]) / np.maximum(np.abs(r0[good]), 1.0)
        print(f"  k_s {ks} vs {CANDIDATES[0]}: ratio scaled max {scaled.max():.2e}", flush=True)
        assert scaled.max() < 1e-9
        assert np.array_equal(iu, i0u) and np.array_equal(id_, i0d) and np.array_equal(iu, ids_o)
        for N, N0 in ((Nu, N0u), (Nd, N0d)):
            assert np.max(np.abs(N - N0)) / np.max(np.abs(N0)) < 1e-9
        for key in ("accepted_insertions", "accepted_removals", "sign"):
            assert st[key] == s0[key]


def test_autotune_picks_a_candidate_and_keeps_the_chain_valid():
    print("[autotune] 4x4", flush=True)
    p = dcax.make_params(**params_kwargs("4x4_U4_b10", warmup_sweeps=4), refresh_every=0)
    w = dcax.Walker(p)
    w.set_config(*initial(240, 16, 10.0, 5))
    w.sweep(4)
    s0 = w.stats()
    ks, rate = w.autotune(sweeps_per_trial=3)
    s1 = w.stats()
    cv, yv = w.variants()
    print(f"  chose k_s = {ks}, kernel forms ({cv}, {yv}) at {rate:.0f} accepted updates/s", flush=True)
    assert ks in (8, 16, 24, 32, 48, 64)
    forms = (dcax.DCAX_VARIANT_TILED, dcax.DCAX_VARIANT_WIDE, dcax.DCAX_VARIANT_NARROW)
    assert cv in forms and yv in forms
    assert rate > 0
    # six submatrix sizes and three forms of each of the two products
    assert s1["proposals"] - s0["proposals"] >= 12 * 3 * 200
    acc, aux = w.new_accumulator()
    w.sweep_measure(5, acc, aux)
    assert w.refresh() < 1e-8
    assert torch.isfinite(acc).all() and float(aux[0]) != 0.0
    w.close()

"""Batches of walkers in one launch (MI355X).

Walkers of a batch are independent Markov chains: each kernel launch covers
every walker, but no arithmetic mixes them, so a walker's trajectory in a
batch must be bit-identical to the same walker (same parameters and seed)
run alone.  The batch here mixes cluster shapes, couplings, temperatures and
submatrix sizes, like a production batch of uneven walkers.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1901_01047_amd import dcax  # noqa: E402

BATCH = [
    dict(cluster=(2, 0, 0, 2), U=4.0, beta=5.0, mu=0.0, n_tau=1000, submatrix_k=16, seed=11),
    dict(cluster=(2, 2, 2, -2), U=3.0, beta=4.0, mu=-0.2, n_tau=801, submatrix_k=8, seed=12),
    dict(cluster=(4, 0, 0, 4), U=2.0, beta=3.0, mu=0.1, n_tau=601, submatrix_k=32, seed=13),
    dict(cluster=(1, 0, 0, 1), t=0.0, U=5.0, beta=2.0, mu=0.0, n_tau=64, submatrix_k=4, seed=14),
]


def params(d, precision=dcax.DCAX_FP64):
    return dcax.make_params(max_order=256, n_freq=48, precision=precision, refresh_every=0, **d)


@pytest.mark.parametrize("precision", [dcax.DCAX_FP64, dcax.DCAX_FP32_MIXED])
def test_batch_equals_individual_walkers(precision):
    print(f"[batch] precision {precision}", flush=True)
    n_sweeps = 30
    plist = [params(d, precision) for d in BATCH]
    wb = dcax.Walker(plist)
    acc_b, aux_b = wb.new_accumulator()
    for _ in range(n_sweeps):
        wb.sweep(1)
        wb.measure(acc_b, aux_b)
    for i, p in enumerate(plist):
        w1 = dcax.Walker(p)
        acc1, aux1 = w1.new_accumulator()
        for _ in range(n_sweeps):
            w1.sweep(1)
            w1.measure(acc1, aux1)
        cb, c1 = wb.get_config(i), w1.get_config()
        assert np.array_equal(cb, c1), f"walker {i}: configurations differ"
        for sp in range(2):
            ib, Nb = wb.copy_N(sp, walker=i)
            i1, N1 = w1.copy_N(sp)
            assert np.array_equal(ib, i1) and np.array_equal(Nb, N1), f"walker {i} spin {sp}: N differs"
        assert torch.equal(wb.acc_block(acc_b, i), acc1), f"walker {i}: accumulators differ"
        assert torch.equal(aux_b[i], aux1)
        s1 = w1.stats()
        sb = wb.stats(walker=i)
        for key in ("proposals", "accepted_insertions", "accepted_removals", "windows", "fold_rank_hist"):
            assert sb[key] == s1[key], (i, key)
        # every window lands in one fold-rank bin; the bins bound the summed rank
        h = s1["fold_rank_hist"]
        assert sum(h) == s1["windows"]
        assert sum((4 * b - 3) * n for b, n in enumerate(h) if b) <= s1["flips_folded"] <= \
            sum(4 * b * n for b, n in enumerate(h))
        print(f"  walker {i}: order {len(c1)}, proposals {s1['proposals']}, identical", flush=True)
        w1.close()
    assert wb.refresh() < (1e-9 if precision == dcax.DCAX_FP64 else 1e-3)
    tot = wb.stats()
    assert tot["proposals"] == sum(wb.stats(walker=i)["proposals"] for i in range(len(plist)))
    wb.close()


def test_batch_finalize_layout():
    print("[batch] finalize layout", flush=True)
    plist = [params(d) for d in BATCH[:3]]
    wb = dcax.Walker(plist)
    wb.sweep(5)
    acc, aux = wb.new_accumulator()
    wb.measure(acc, aux)
    Giw, Gt = wb.finalize(acc, aux, n_tau_out=33)
    off_t = 0
    for i, p in enumerate(plist):
        w1 = dcax.Walker(p)
        w1.sweep(5)
        a1, x1 = w1.new_accumulator()
        w1.measure(a1, x1)
        g1, t1 = w1.finalize(a1, x1, n_tau_out=33)
        assert torch.equal(wb.acc_block(Giw, i), g1)
        n = 2 * wb.Ncs[i] * 33
        assert torch.equal(Gt[off_t:off_t + n].view(2, wb.Ncs[i], 33), t1)
        off_t += n
        w1.close()
    wb.close()


@pytest.mark.parametrize("precision,timing", [(dcax.DCAX_FP64, False), (dcax.DCAX_FP32_MIXED, False),
                                              (dcax.DCAX_FP64, True)])
def test_graph_sweeps_equal_eager_sweeps(precision, timing):
    """Sweeps replayed as captured hipGraphs follow the same trajectory.

    The graph path launches the same kernels with launch shapes rounded up to
    the next order bucket, so the chains must stay bit-identical; measurements
    and synchronisations run eagerly between the replays, and every replay is
    compared through the state it leaves."""
    print(f"[graph] precision {precision} timing {timing}", flush=True)
    plist = [params(d, precision) for d in BATCH]
    we, wg = dcax.Walker(plist), dcax.Walker(plist)
    wg.set_graphs(True)
    wg.set_timing(timing)
    acc_e, aux_e = we.new_accumulator()
    acc_g, aux_g = wg.new_accumulator()
    for sw in range(25):
        we.sweep(1)
        wg.sweep(1)
        we.measure(acc_e, aux_e)
        wg.measure(acc_g, aux_g)
        for i in range(len(plist)):
            assert np.array_equal(we.get_config(i), wg.get_config(i)), f"sweep {sw} walker {i}"
    for i in range(len(plist)):
        for sp in range(2):
            ie, Ne = we.copy_N(sp, walker=i)
            ig, Ng = wg.copy_N(sp, walker=i)
            assert np.array_equal(ie, ig) and np.array_equal(Ne, Ng), f"walker {i} spin {sp}: N differs"
    assert torch.equal(acc_e, acc_g) and torch.equal(aux_e, aux_g)
    st = wg.stats()
    if timing:
        assert st["window_seconds"] > 0.0     # replayed sweeps are timed as a whole
    assert st["proposals"] == we.stats()["proposals"]
    print(f"  graph replays identical; timed {st['window_seconds']:.4f} s", flush=True)
    we.close()
    wg.close()


def test_refresh_forms_agree_in_a_batch():
    """A batch whose largest order exceeds 1024 refreshes every walker with
    the column-step panel form; a walker of order 100 alone takes the
    one-workgroup form.  Both forms make the same pivot choices and the same
    arithmetic."""
    print("[batch] refresh forms", flush=True)
    d = dict(cluster=(4, 0, 0, 4), U=4.0, beta=10.0, mu=-0.3, n_tau=2001, submatrix_k=32, seed=21)
    p = dcax.make_params(max_order=2048, n_freq=16, refresh_every=0, **d)
    rng = np.random.default_rng(5)
    cfg = [(rng.integers(0, 16, size=n).astype(np.int32), rng.random(n) * 10.0,
            np.where(rng.random(n) < 0.5, 1, -1).astype(np.int32)) for n in (1100, 100)]
    wb = dcax.Walker([p, p])
    for i, c in enumerate(cfg):
        wb.set_config(*c, walker=i)
    drift = wb.refresh()
    print(f"  batch refresh drift {drift:.2e}", flush=True)
    assert drift < 1e-9
    for i, c in enumerate(cfg):
        w1 = dcax.Walker(p)
        w1.set_config(*c)
        for sp in range(2):
            ib, Nb = wb.copy_N(sp, walker=i)
            i1, N1 = w1.copy_N(sp)
            assert np.array_equal(ib, i1)
            e = np.max(np.abs(Nb - N1)) / np.max(np.abs(N1))
            print(f"  walker {i} (k={len(i1)}) spin {sp}: max diff {e:.2e}"
                  f"{' (bit-identical)' if e == 0 else ''}", flush=True)
            assert e < 1e-12
        assert wb.stats(walker=i)["sign"] == w1.stats()["sign"]
        w1.close()
    wb.close()

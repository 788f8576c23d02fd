"""Device-scheduled sweeps (dcax_sweep_measure) against the host's lockstep
sweeps (MI355X).

dcax_sweep_measure lets every walker of a batch begin its next sweep as soon
as its previous one has been measured, instead of all walkers stepping
through as many windows as the longest sweep needs.  The schedule must not
change any walker's Markov chain or measurements: each walker's proposals,
windows and measurement points are its own.  So n calls of
sweep(1) + measure must leave bit-identical configurations, N and
accumulators to one sweep_measure(n), walker by walker (refreshes off, since
their timing differs between the two schedules).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1901_01047_amd import dcax  # noqa: E402
from tests.test_gpu_batch import BATCH, params  # noqa: E402


def run_lockstep(plist, n):
    w = dcax.Walker(plist)
    acc, aux = w.new_accumulator()
    for _ in range(n):
        w.sweep(1)
        w.measure(acc, aux)
    return w, acc, aux


def run_rounds(plist, n, chunks):
    w = dcax.Walker(plist)
    acc, aux = w.new_accumulator()
    done = 0
    for c in chunks:
        w.sweep_measure(c, acc, aux)
        done += c
    assert done == n
    return w, acc, aux


@pytest.mark.parametrize("precision", [dcax.DCAX_FP64, dcax.DCAX_FP32_MIXED])
@pytest.mark.parametrize("which", ["batch", "single"])
def test_rounds_equal_lockstep(precision, which):
    print(f"[rounds] {which} precision {precision}", flush=True)
    n = 25
    plist = [params(d, precision) for d in (BATCH if which == "batch" else BATCH[:1])]
    if which == "single":
        plist = plist[0]
    wl, accl, auxl = run_lockstep(plist, n)
    wr, accr, auxr = run_rounds(plist, n, [1, 9, 15])
    for i in range(wl.W):
        cl, cr = wl.get_config(i), wr.get_config(i)
        assert np.array_equal(cl, cr), f"walker {i}: configurations differ"
        for sp in range(2):
            il, Nl = wl.copy_N(sp, walker=i)
            ir, Nr = wr.copy_N(sp, walker=i)
            assert np.array_equal(il, ir) and np.array_equal(Nl, Nr), f"walker {i} spin {sp}: N differs"
        if wl.W > 1:
            assert torch.equal(wl.acc_block(accl, i), wr.acc_block(accr, i)), f"walker {i}: accumulators differ"
            assert torch.equal(auxl[i], auxr[i])
        else:
            assert torch.equal(accl, accr) and torch.equal(auxl, auxr)
        sl, sr = wl.stats(walker=i), wr.stats(walker=i)
        for key in ("proposals", "accepted_insertions", "accepted_removals", "windows", "aborted_windows"):
            assert sl[key] == sr[key], (i, key)
        print(f"  walker {i}: order {len(cl)}, proposals {sl['proposals']}, identical", flush=True)
    wl.close()
    wr.close()


@pytest.mark.parametrize("precision", [dcax.DCAX_FP64, dcax.DCAX_FP32_MIXED])
def test_free_running_rounds_match_single_walkers(precision):
    """dcax_run_rounds: walkers make different numbers of sweeps, but each
    walker's chain and measurements equal the same walker's own sweeps."""
    print(f"[free rounds] precision {precision}", flush=True)
    plist = [params(d, precision) for d in BATCH]
    wb = dcax.Walker(plist)
    acc_b, aux_b = wb.new_accumulator()
    wb.run_rounds(12, acc_b, aux_b)
    wb.run_rounds(7, acc_b, aux_b)
    props = []
    for i, p in enumerate(plist):
        target = wb.stats(walker=i)["proposals"]
        w1 = dcax.Walker(p)
        acc1, aux1 = w1.new_accumulator()
        n = 0
        while w1.stats()["proposals"] < target:
            w1.sweep_measure(1, acc1, aux1)
            n += 1
        assert w1.stats()["proposals"] == target, f"walker {i}: stopped inside a sweep"
        assert np.array_equal(wb.get_config(i), w1.get_config()), f"walker {i}: configurations differ"
        assert torch.equal(wb.acc_block(acc_b, i), acc1), f"walker {i}: accumulators differ"
        assert torch.equal(aux_b[i], aux1)
        props.append((n, target))
        print(f"  walker {i}: {n} sweeps, {target} proposals, identical", flush=True)
        w1.close()
    assert len({n for n, _ in props}) > 1, "walkers of different sweep lengths made the same number of sweeps"
    wb.close()


@pytest.mark.parametrize("warmup", [1, 2])
def test_sweep_length_freezes_at_the_warm_up_order(warmup):
    """Sweeps have max(k, 1) proposals (rounded up to a multiple of k_s)
    during the warm-up, then a length frozen at the mean order over the
    warm-up's second half, which holds at least its last sweep: with one
    warm-up sweep from a configuration of order 240, every later sweep keeps
    that sweep's length (and not the minimal one window)."""
    print(f"[sweep length] warm-up {warmup}", flush=True)
    p = params(dict(BATCH[2], seed=31), dcax.DCAX_FP64)
    p.warmup_sweeps = warmup
    p.max_order = 1024
    w = dcax.Walker(p)
    rng = np.random.default_rng(3)
    n = 240
    w.set_config(rng.integers(0, 16, size=n).astype(np.int32), rng.random(n) * 3.0,
                 np.where(rng.random(n) < 0.5, 1, -1).astype(np.int32))
    ks = p.submatrix_k
    first = -(-n // ks) * ks
    w.sweep(1)
    assert w.stats()["proposals"] == first
    k1 = w.order
    w.sweep(3)
    per = w.stats()["proposals"] - first
    print(f"  first sweep {first} proposals, order then {k1}, next three {per}", flush=True)
    # warm-up 1: frozen at the order 240 of the first sweep's start; warm-up
    # 2: the second sweep has max(k1, 1) proposals and the length freezes at k1
    frozen = n if warmup == 1 else max(k1, 1)
    assert per == 3 * (-(-frozen // ks) * ks)
    w.close()


@pytest.mark.parametrize("precision", [dcax.DCAX_FP64, dcax.DCAX_FP32_MIXED])
@pytest.mark.parametrize("which", ["batch", "single"])
def test_round_graphs_equal_eager_rounds(precision, which):
    """With graphs on, each device-scheduled round (sweep starts, windows,
    gated measurement) is one captured hipGraph, replayed round after round.
    Walked one call at a time - eager work and synchronisation between the
    replays - the state after every call equals the eager rounds'; at the
    end N, accumulators and counters are bit-identical."""
    print(f"[round graphs] {which} precision {precision}", flush=True)
    plist = [params(d, precision) for d in (BATCH if which == "batch" else BATCH[:1])]
    if which == "single":
        plist = plist[0]
    we, wg = dcax.Walker(plist), dcax.Walker(plist)
    wg.set_graphs(True)
    acc_e, aux_e = we.new_accumulator()
    acc_g, aux_g = wg.new_accumulator()
    for call in range(12):
        if call % 2:
            we.run_rounds(3, acc_e, aux_e)
            wg.run_rounds(3, acc_g, aux_g)
        else:
            we.sweep_measure(2, acc_e, aux_e)
            wg.sweep_measure(2, acc_g, aux_g)
        for i in range(we.W):
            assert np.array_equal(we.get_config(i), wg.get_config(i)), f"call {call} walker {i}"
        assert torch.equal(acc_e, acc_g) and torch.equal(aux_e, aux_g), f"call {call}: accumulators differ"
    for i in range(we.W):
        for sp in range(2):
            ie, Ne = we.copy_N(sp, walker=i)
            ig, Ng = wg.copy_N(sp, walker=i)
            assert np.array_equal(ie, ig) and np.array_equal(Ne, Ng), f"walker {i} spin {sp}: N differs"
        se, sg = we.stats(walker=i), wg.stats(walker=i)
        for key in ("proposals", "accepted_insertions", "accepted_removals", "windows"):
            assert se[key] == sg[key], (i, key)
    print(f"  12 calls identical; proposals {we.stats()['proposals']}", flush=True)
    we.close()
    wg.close()

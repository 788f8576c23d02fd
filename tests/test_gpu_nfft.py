"""Delayed-NFFT measurement on the GPU (MI355X), through the C ABI.

* the gridded samples of one configuration against the oracle's gridding of
  the same M (the GPU's own N, so that only the gridding is compared): the
  wrap, the image sign, the displacement rows and the kernel weights;
* the single transform at the end of several measurements against the direct
  measurement of the same configurations (dcax_measure_G), within the NFFT
  error scale exp(-(2/3) pi M_sp) per unit of sum |M_ij| / Nc, in both
  precisions, for a single walker and for a batch of uneven walkers (the
  per-walker grid layout);
* arguments outside the documented ranges are rejected on the host.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ctaux, nfft  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import params_kwargs  # noqa: E402
from tests.ctaux_cases import model  # noqa: E402
from tests.test_gpu_batch import BATCH, params  # noqa: E402


def gpu_M(w, m, walker=0):
    """The walker's configuration (id order) and M = (e^V - 1) N per spin."""
    cfg = w.get_config(walker)
    cfg = cfg[np.argsort(cfg["id"])]
    Ms = []
    for sp in range(2):
        ids, N = w.copy_N(sp, walker=walker)
        assert np.array_equal(ids, cfg["id"])
        Ms.append((m.ev(cfg["aux_spin"], sp) - 1.0)[:, None] * N)
    return cfg, Ms


@pytest.mark.parametrize("hw", [4, 8])
def test_grid_matches_oracle_gridding(hw):
    name, nf = "4x4_U4_b10", 64
    print(f"[nfft grid] {name} half_width {hw}", flush=True)
    m = model(name)
    w = dcax.Walker(dcax.make_params(**params_kwargs(name, n_freq=nf, max_order=512)))
    ow = ctaux.Walker(m, seed=21)
    ow.random_config(150)
    w.set_config(ow.r, ow.t, ow.s, ow.id)
    grid = w.new_nfft_grid()
    _, aux = w.new_accumulator()
    w.measure_nfft(grid, aux, hw)
    cfg, Ms = gpu_M(w, m)
    sign = float(aux.reshape(-1)[0])
    assert sign in (1.0, -1.0)
    G = grid.cpu().numpy().reshape(2, m.Nc, nfft.grid_size(nf))
    for sp in range(2):
        Go = nfft.grid_M(m, cfg["site"], cfg["tau"], Ms[sp], nf, hw)
        err = np.max(np.abs(G[sp] - sign * Go))
        ref = np.abs(Ms[sp]).sum()
        print(f"  spin {sp}: max |grid - oracle| {err:.2e} (sum |M| {ref:.2e})", flush=True)
        assert err <= 1e-12 * ref
    w.close()


@pytest.mark.parametrize("precision", [dcax.DCAX_FP64, dcax.DCAX_FP32_MIXED])
def test_delayed_transform_matches_direct_measurement(precision):
    name, nf, hw = "4x4_U4_b10", 128, 8
    print(f"[nfft transform] {name} precision {precision}", flush=True)
    m = model(name)
    w = dcax.Walker(dcax.make_params(**params_kwargs(name, n_freq=nf, max_order=512, warmup_sweeps=2),
                                     precision=precision))
    ow = ctaux.Walker(m, seed=5)
    ow.random_config(200)
    w.set_config(ow.r, ow.t, ow.s, ow.id)
    acc, aux = w.new_accumulator()
    aux2 = torch.zeros_like(aux)
    grid = w.new_nfft_grid()
    weight = np.zeros(2)
    for _ in range(4):
        w.sweep(1)
        w.measure(acc, aux)
        w.measure_nfft(grid, aux2, hw)
        _, Ms = gpu_M(w, m)
        weight += [np.abs(M).sum() / m.Nc for M in Ms]
    acc2 = torch.zeros_like(acc)
    w.nfft_transform(grid, acc2, hw)
    assert torch.equal(aux, aux2)
    a = w.acc_block(acc, 0).cpu().numpy()
    b = w.acc_block(acc2, 0).cpu().numpy()
    # FP32-mixed: both measurements read M in FP32 (the direct one also its phases)
    rnd = 1e-12 if precision == dcax.DCAX_FP64 else 2e-6
    for sp in range(2):
        err = np.max(np.abs(a[sp] - b[sp]))
        bound = (2.0 * nfft.error_scale(hw) + rnd) * weight[sp]
        print(f"  spin {sp}: max |nfft - direct| {err:.2e}, bound {bound:.2e}", flush=True)
        assert err <= bound
    w.close()


def test_batch_grid_layout():
    print("[nfft batch]", flush=True)
    hw = 6
    plist = [params(d) for d in BATCH]
    wb = dcax.Walker(plist)
    acc, aux = wb.new_accumulator()
    aux2 = torch.zeros_like(aux)
    grid = wb.new_nfft_grid()
    for _ in range(6):
        wb.sweep(1)
        wb.measure(acc, aux)
        wb.measure_nfft(grid, aux2, hw)
    acc2 = torch.zeros_like(acc)
    wb.nfft_transform(grid, acc2, hw)
    assert torch.equal(aux, aux2)
    for i in range(len(plist)):
        a = wb.acc_block(acc, i).cpu().numpy()
        b = wb.acc_block(acc2, i).cpu().numpy()
        scale = max(np.max(np.abs(a)), 1e-300)
        err = np.max(np.abs(a - b))
        print(f"  walker {i}: order {wb.order_of(i)}, max |nfft - direct| {err:.2e} (max |acc| {scale:.2e})",
              flush=True)
        assert err <= 1e-3 * scale
    wb.close()


def test_bad_arguments_rejected():
    w = dcax.Walker(dcax.make_params(**params_kwargs("2x2_U4_b5", n_freq=16)))
    grid = w.new_nfft_grid()
    acc, aux = w.new_accumulator()
    for hw in (1, 17):
        with pytest.raises(dcax.DcaxError):
            w.measure_nfft(grid, aux, hw)
        with pytest.raises(dcax.DcaxError):
            w.nfft_transform(grid, acc, hw)
    w.close()


@pytest.mark.parametrize("which", ["single", "batch"])
def test_device_scheduled_sweeps_with_nfft_equal_lockstep(which):
    """dcax_sweep_measure_nfft(n) = n x (sweep(1) + measure_nfft): the same
    chains bit for bit, the same signs, and the same grids up to the order of
    the atomic additions of workgroups that share a grid row."""
    print(f"[nfft rounds] {which}", flush=True)
    plist = [params(d) for d in BATCH]
    if which == "single":
        plist = plist[2]
    hw, n = 6, 7
    wa, wb = dcax.Walker(plist), dcax.Walker(plist)
    ga, gb = wa.new_nfft_grid(), wb.new_nfft_grid()
    _, aa = wa.new_accumulator()
    _, ab = wb.new_accumulator()
    for _ in range(n):
        wa.sweep(1)
        wa.measure_nfft(ga, aa, hw)
    wb.sweep_measure_nfft(3, gb, ab, hw)
    wb.sweep_measure_nfft(n - 3, gb, ab, hw)
    assert torch.equal(aa, ab)
    for i in range(wa.W):
        assert np.array_equal(wa.get_config(i), wb.get_config(i))
        for sp in range(2):
            assert np.array_equal(wa.copy_N(sp, walker=i)[1], wb.copy_N(sp, walker=i)[1])
    err = float((ga - gb).abs().max())
    scale = float(ga.abs().max())
    print(f"  grids: max diff {err:.2e} of max {scale:.2e}", flush=True)
    assert err <= 1e-12 * scale
    wa.close()
    wb.close()

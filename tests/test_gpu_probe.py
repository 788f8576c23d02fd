"""The probe of N against its definition and the drift control (MI355X).

N = [e^V - g (e^V - 1)]^{-1} (Sec. 2.3).  dcax_probe_N samples entries of
A N - 1 with A assembled from the propagator:

* a freshly rebuilt FP64 N gives residuals at the unit roundoff (the
  assembly of A, its signs and the per-column e^V are those of the
  refresh), and FP64 sweeps keep them there;
* an FP32-mixed N starts near FP32 roundoff after a rebuild and its residual
  grows over sweeps without refresh; the rebuild brings it back;
* with drift_tol the library rebuilds walkers whose residual exceeds the
  tolerance at the end of a sweep, before that sweep's measurement, so a
  fresh probe of the final state stays near it and no measurement is lost.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs  # noqa: E402


def _walkers(name, W, precision, **kw):
    cfg = CONFIGS[name]
    plist = [dcax.make_params(**params_kwargs(name, seed=cfg["seed"] + i, warmup_sweeps=2), precision=precision, **kw)
             for i in range(W)]
    w = dcax.Walker(plist)
    for i in range(W):
        w.set_config(*initial_config(w.Ncs[i], cfg["beta"], cfg["k_init"], cfg["seed"] + 100 + i), walker=i)
    return w


def test_probe_of_an_exact_N_is_at_roundoff():
    print("[probe] FP64", flush=True)
    w = _walkers("4x4_U4_b10", 4, dcax.DCAX_FP64)
    r0 = w.probe()
    w.sweep(6)
    r1 = w.probe()
    d = w.refresh()
    r2 = w.probe()
    print(f"  after set_config {r0.max():.2e}, after 6 sweeps {r1.max():.2e} (drift {d:.2e}), after refresh "
          f"{r2.max():.2e}", flush=True)
    assert r0.max() < 1e-13 and r2.max() < 1e-13 and r1.max() < 1e-11
    st = w.stats()
    assert st["probes"] == 3 and st["probe_refreshes"] == 0
    w.close()


def test_mixed_residual_grows_and_the_rebuild_resets_it():
    print("[probe] FP32-mixed", flush=True)
    w = _walkers("4x4_U4_b10", 4, dcax.DCAX_FP32_MIXED)
    r0 = w.probe()
    w.sweep(20)
    r1 = w.probe()
    d = w.refresh()
    r2 = w.probe()
    print(f"  after set_config {r0.max():.2e}, after 20 sweeps {r1.max():.2e} (drift {d:.2e}), after refresh "
          f"{r2.max():.2e}", flush=True)
    assert r0.max() < 1e-5 and r2.max() < 1e-5
    assert r1.max() > 3 * r2.max()
    w.close()


def test_drift_control_rebuilds_walkers_above_the_tolerance():
    print("[probe] drift control", flush=True)
    tol = 2e-6
    w = _walkers("4x4_U4_b10", 4, dcax.DCAX_FP32_MIXED, drift_tol=tol)
    acc, aux = w.new_accumulator()
    w.sweep(10)
    w.sweep_measure(10, acc, aux)
    st = w.stats()
    r = w.probe()
    print(f"  probes {st['probes']}, walkers rebuilt {st['probe_refreshes']}, last probe {st['last_probe']:.2e}, "
          f"fresh probe {r.max():.2e}", flush=True)
    assert st["probe_refreshes"] > 0 and st["probes"] >= 20
    assert r.max() < 30 * tol
    # a walker held at its sweep end is measured once, after its rebuild:
    # every walker has exactly one measurement (sign +-1) per sweep
    s = aux[:, 0].cpu().numpy()
    print(f"  sign sums {s}", flush=True)
    assert np.all(np.abs(s) <= 10) and np.all(np.mod(10 - s, 2) == 0)
    w.close()

"""Parity at the full sizes of the large workloads (MI355X).

The 6x6 (k ~ 2000) and 8x8 (k ~ 6000) clusters run with the submatrix size
and precision the benchmark uses.  The oracle records a short trace (two
windows) from a seeded random configuration of the workload's order; the
library replays it with forced decisions, and every ratio of the trace and
the final N are compared with the oracle.  Random configurations of these
orders are far from equilibrium and badly conditioned: the same submatrix
algebra evaluated in plain NumPy FP64 already lands 1e-8 (6x6) from the
oracle's single-vertex chain, and two FP64 evaluations of such a state in
different summation orders scatter by an order of magnitude in their worst
element.  So the comparison uses statistics that average over many values:
the 95th percentile of the ratio errors (relative to max(|R|, 1)) and the
Frobenius-norm error of N must be within max(1e-10, 30 x those of that
algebra on the same trace), with no decision on the other side of |R|.
(Measured: the kernels land 2-4x above the NumPy evaluation at k ~ 2000 and
9-10x at k ~ 6000; the NumPy products sum long dot products blockwise, the
matrix cores in k/64-long chains.)  The FP32-mixed errors are reported, not
bounded: on these states they reach O(1) (N error 0.2 - 0.9), which is the
finding that the mixed mode needs equilibrated states and frequent FP64
refreshes at these couplings.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, params_kwargs  # noqa: E402
from tests.ctaux_cases import model, oracle_trace  # noqa: E402
from tests.test_gpu_parity import algebra_gauge, rel_norm  # noqa: E402

LARGE = ["6x6_U6_b20", "8x8_U7_b30"]


@pytest.mark.parametrize("name", LARGE)
def test_large_replay_parity(name):
    c = CONFIGS[name]
    k_s = c["submatrix_k"]
    print(f"[large replay] {name} k_init={c['k_init']} k_s={k_s}", flush=True)
    m = model(name)
    init, rec, ratios_o, ow = oracle_trace(m, seed=c["seed"] + 11, k_s=k_s, init_order=c["k_init"],
                                           warm_sweeps=0, rec_proposals=2 * k_s)
    print("  oracle trace recorded", flush=True)
    noop = (rec["kind"] == 1) & (rec["id"] < 0)
    good = ~noop
    ro = ratios_o[good]
    r_wm, (ids_wm, Nu_wm, Nd_wm) = algebra_gauge(m, init, rec, k_s)
    err_wm = np.abs(r_wm - ro)
    ids_o, Nu, Nd = ow.canonical()
    e_wm = [rel_norm(Nu_wm, Nu), rel_norm(Nd_wm, Nd)]
    f_wm = [np.linalg.norm(Nu_wm - Nu) / np.linalg.norm(Nu), np.linalg.norm(Nd_wm - Nd) / np.linalg.norm(Nd)]
    results = {}
    for prec, tag in ((dcax.DCAX_FP64, "fp64"), (dcax.DCAX_FP32_MIXED, "mixed")):
        w = dcax.Walker(dcax.make_params(**params_kwargs(name), precision=prec))
        w.set_config(*init)
        ratios = w.replay(rec)
        err = np.abs(ratios[good] - ro)
        scaled = err / np.maximum(np.abs(ro), 1.0)
        rel = err / np.abs(ro)
        nerr, nfro = [], []
        for sp in range(2):
            ids, N = w.copy_N(sp)
            assert np.array_equal(ids, ids_o)
            No = (Nu, Nd)[sp]
            nerr.append(rel_norm(N, No))
            nfro.append(np.linalg.norm(N - No) / np.linalg.norm(No))
        results[tag] = (scaled, rel, err, nfro, w.stats()["decision_mismatches"])
        print(f"  {tag}: ratio scaled max {scaled.max():.2e}, rel median {np.median(rel):.2e} max {rel.max():.2e}; "
              f"N normwise {max(nerr):.2e} (FP64 algebra {max(e_wm):.2e}), Frobenius {max(nfro):.2e} "
              f"(FP64 algebra {max(f_wm):.2e}); k = {len(ids_o)}", flush=True)
        w.close()
    scaled, rel, err, nfro, mis = results["fp64"]
    scaled_wm = err_wm / np.maximum(np.abs(ro), 1.0)
    p95, p95_wm = np.quantile(scaled, 0.95), np.quantile(scaled_wm, 0.95)
    print(f"  ratio error p95: GPU {p95:.2e}, FP64 algebra {p95_wm:.2e} (max {scaled_wm.max():.2e})", flush=True)
    assert mis == 0
    assert p95 <= max(1e-10, 30 * p95_wm)
    for sp in range(2):
        assert nfro[sp] < max(1e-10, 30 * f_wm[sp])

"""The replay entry point that allocates nothing (MI355X).

dcax_sweep_replay_static stages records and ratios in the library's fixed
per-GPU buffer instead of memory from the caller's allocator.  It must give
the same ratios and N as dcax_sweep's replay (the same kernels) on two calls
in a row, the second smaller, the walker carrying on between them; records
beyond the fixed limit are refused; and dcax_sweep's own replay still works
after the static one has run on the same walker.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs  # noqa: E402
from tests.ctaux_cases import model, oracle_trace  # noqa: E402


@pytest.mark.parametrize("prec", [dcax.DCAX_FP64, dcax.DCAX_FP32_MIXED])
def test_static_replay_equals_allocating_replay(prec):
    name = "4x4_U4_b10"
    print(f"[no-alloc replay] {name} precision {prec}", flush=True)
    m = model(name)
    init, rec, ratios_o, ow = oracle_trace(m, seed=CONFIGS[name]["seed"] + 21, k_s=32, init_order=0,
                                           init=initial_config(m.Nc, m.beta, 220, 23), warm_sweeps=1,
                                           rec_proposals=900)
    first, second = rec[:600], rec[600:]          # two calls, the second smaller
    wa = dcax.Walker(dcax.make_params(**params_kwargs(name, submatrix_k=32), precision=prec))
    ws = dcax.Walker(dcax.make_params(**params_kwargs(name, submatrix_k=32), precision=prec))
    for w in (wa, ws):
        w.set_config(*init)
    for part in (first, second):
        ra = wa.replay(part)
        rs = ws.replay_static(part)
        assert np.array_equal(ra, rs)
        for sp in range(2):
            ia, Na = wa.copy_N(sp)
            is_, Ns = ws.copy_N(sp)
            assert np.array_equal(ia, is_) and np.array_equal(Na, Ns)
        print(f"  {len(part)} records: ratios and N identical", flush=True)
    # the allocating replay still works on the walker that used the static one
    more = oracle_trace(m, seed=5, k_s=32, init_order=0, init=initial_config(m.Nc, m.beta, 150, 29),
                        warm_sweeps=0, rec_proposals=100)
    ws.set_config(*more[0])
    r2 = ws.replay(more[1])
    good2 = ~((more[1]["kind"] == 1) & (more[1]["id"] < 0))
    assert np.max(np.abs(r2[good2] - more[2][good2]) / np.abs(more[2][good2])) < (1e-10 if prec == 0 else 1e-3)
    # beyond the limit: refused before any work
    big = np.zeros(dcax.REPLAY_STATIC_MAX + 1, dcax.PROPOSAL_DTYPE)
    big["kind"] = 1
    big["id"] = -1
    with pytest.raises(dcax.DcaxError) as e:
        ws.replay_static(big)
    assert e.value.status == -1
    wa.close()
    ws.close()

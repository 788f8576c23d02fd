"""Measurement M -> M(K, i w_n) at the full sizes of the large workloads (MI355X).

The 6x6 cluster (k ~ 2000, 256 Matsubara frequencies, one walker) and the
8x8 cluster (k ~ 6000, 512 frequencies, 32 walkers in one handle: the launch
configuration of the benchmark's headline workload) measure seeded random
configurations once.  The oracle's direct sums (Sec. 2.3's M-function
estimator, no blocking) over the walker's own M = (e^V - 1) N are evaluated
at sampled outputs: every momentum at the lowest, a middle and the highest
frequencies, plus all frequencies at K = 0 and at the zone corner.

Tolerance: relative to the scale of the summands, (1/Nc) sum |M_ij|.  The
phase arguments w_n tau are formed in FP64 (argument error eps64 w_max beta
per phase, once for the row and once for the column) and the phases are
rounded once to the storage type (eps_T each); the sums add O(k) eps_T.
Bound: 4 eps64 w_max beta + eps_T (4 + 4 k), eps_T the unit roundoff of the
precision the contraction runs in (FP64, or FP32 in the mixed mode).  The
trace terms (equal-time coefficient of the tail) are checked against the
oracle's trace of the same M.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import measure  # noqa: E402
from paper_1901_01047_amd import dcax  # noqa: E402
from paper_1901_01047_amd.workloads import CONFIGS, params_kwargs  # noqa: E402
from tests.ctaux_cases import model  # noqa: E402


def _sampled(nf, Nc, m):
    freqs = sorted({0, 1, 2, nf // 2, nf - 2, nf - 1})
    # K = 0 and the zone corner (pi, pi) with every frequency
    Kpi = int(np.argmin(np.sum((m.K - np.pi) ** 2, axis=1)))
    return freqs, [0, Kpi]


def _check_walker(w, wi, m, nf, sign, acc_block, aux_row, eps, label):
    k = w.order_of(wi)
    errs = []
    for sp in range(2):
        ids, N = w.copy_N(sp, walker=wi)
        cfg = w.get_config(walker=wi)
        o = np.argsort(cfg["id"])
        assert np.array_equal(ids, cfg["id"][o])
        r, t, s = cfg["site"][o], cfg["tau"][o], cfg["aux_spin"][o]
        M = (m.ev(s, sp) - 1.0)[:, None] * N
        scale = np.abs(M).sum() / m.Nc
        got = acc_block[sp, ..., 0] + 1j * acc_block[sp, ..., 1]
        freqs, Ks = _sampled(nf, m.Nc, m)
        want_f = sign * measure.M_K_iw(m, r, t, M, nf, freqs=freqs)          # all K, sampled n
        want_K = sign * measure.M_K_iw(m, r, t, M, nf, Ks=Ks)                # sampled K, all n
        e = max(np.max(np.abs(got[:, freqs] - want_f)), np.max(np.abs(got[Ks, :] - want_K))) / scale
        tol = 4 * np.finfo(np.float64).eps * (2 * nf - 1) * np.pi + eps * (4 + 4 * k)
        tr = sign * np.trace(M) / m.Nc
        e_tr = abs(aux_row[1 + sp] - tr) / (np.abs(np.diag(M)).sum() / m.Nc)
        print(f"  {label} walker {wi} spin {sp}: k = {k}, err / sum|M| {e:.2e} (bound {tol:.1e}), "
              f"trace err {e_tr:.1e}", flush=True)
        assert e < tol
        assert e_tr < 8 * k * eps
        errs.append(e)
    return max(errs)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_measurement_6x6_full_size(prec):
    name = "6x6_U6_b20"
    c = CONFIGS[name]
    m = model(name)
    nf = c["n_freq"]
    print(f"[measure large] {name} {prec} k={c['k_init']} n_freq={nf}", flush=True)
    p = dcax.DCAX_FP64 if prec == "fp64" else dcax.DCAX_FP32_MIXED
    w = dcax.Walker(dcax.make_params(**params_kwargs(name), precision=p))
    rng = np.random.default_rng(c["seed"] + 31)
    k = c["k_init"]
    w.set_config(rng.integers(0, m.Nc, k).astype(np.int32), rng.random(k) * m.beta,
                 np.where(rng.random(k) < 0.5, 1, -1).astype(np.int32))
    acc, aux = w.new_accumulator()
    w.measure(acc, aux)
    auxh = aux.cpu().numpy().reshape(-1, 3)
    eps = np.finfo(np.float64 if prec == "fp64" else np.float32).eps
    _check_walker(w, 0, m, nf, float(auxh[0, 0]), w.acc_block(acc, 0).cpu().numpy(), auxh[0], eps, prec)
    w.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_measurement_8x8_32_walkers(prec):
    name = "8x8_U7_b30"
    c = CONFIGS[name]
    m = model(name)
    nf = c["n_freq"]
    n_w = 32
    print(f"[measure large] {name} {prec} {n_w} walkers, n_freq={nf}", flush=True)
    p = dcax.DCAX_FP64 if prec == "fp64" else dcax.DCAX_FP32_MIXED
    plist = [dcax.make_params(**params_kwargs(name, seed=c["seed"] + i), precision=p) for i in range(n_w)]
    w = dcax.Walker(plist)
    rng = np.random.default_rng(c["seed"] + 41)
    for i in range(n_w):
        k = int(c["k_init"] + rng.integers(-400, 400))
        w.set_config(rng.integers(0, m.Nc, k).astype(np.int32), rng.random(k) * m.beta,
                     np.where(rng.random(k) < 0.5, 1, -1).astype(np.int32), walker=i)
    print("  configurations set", flush=True)
    acc, aux = w.new_accumulator()
    w.measure(acc, aux)
    torch.cuda.synchronize()
    auxh = aux.cpu().numpy()
    eps = np.finfo(np.float64 if prec == "fp64" else np.float32).eps
    for wi in (0, n_w // 2, n_w - 1):
        _check_walker(w, wi, m, nf, float(auxh[wi, 0]), w.acc_block(acc, wi).cpu().numpy(), auxh[wi], eps, prec)
    w.close()
    del acc, aux
    torch.cuda.empty_cache()

"""Benchmark: accepted vertex updates per second of the CT-AUX walkers.

A step is one pass of the whole hot path for every walker: one Markov-chain
sweep (submatrix windows: gathers, candidate GEMMs, FP64 accept loop, rank-m
fold, compaction), one measurement of M(K, i w_n) accumulated on the GPU,
and, every `refresh_every` sweeps, the FP64 refresh of N.  The default
workload is the large one: the 8x8 Hubbard cluster (U = 7, beta = 30,
n ~ 0.9, expansion order ~ 6000), 32 walkers sharing the GPU, FP32-mixed
(N and its GEMMs in FP32, ratios and refresh in FP64), 512 Matsubara
frequencies measured every sweep; the same workload in FP64 runs beside it.
`value` is the FP32-mixed figure.  Synthetic inputs: seeded starting
configurations (workloads.initial_config), inputs resident in HBM.

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp64_mfma_TFs": 78.6, "fp32_mfma_TFs": 157.3}
WORKLOAD = "8x8_U7_b30"
WALKERS = 32
# a pseudo-random 1/TIMING_EVERY of the windows of a small workload carries
# HIP events (each event idles the queue for a few microseconds); windows of
# orders above TIME_ALL_ORDER take milliseconds and are all timed
TIMING_EVERY = 8
TIME_ALL_ORDER = 1024


# kernel -> (stats prefix for flops/bytes/seconds, source section of
# csrc/dcax_window.hip from its header comment to the next one)
KERNELS = {
    "k_cand_x": ("cand", "// ------------------------------------------------------- candidate rows\n",
                 "// -------------------------------------------------------------- Gram"),
    "k_ygemm": ("y", "// --------------------------------------------------------- Y = N g_{I,c}\n",
                "// ------------------------------------------------------------ fold prep"),
    "k_fold": ("fold", "// ---------------------------------------------------------------- fold\n",
               "// ----------------------------------------------------------- compaction"),
}


def kernel_source_hash(kernel):
    import hashlib
    src = open(os.path.join(ROOT, "paper_1901_01047_amd", "csrc", "dcax_window.hip")).read()
    _, a, b = KERNELS[kernel]
    return hashlib.sha256(src[src.index(a):src.index(b)].encode()).hexdigest()


def kernel_traffic(kernel, workload, walkers, precision):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (profiles/traffic_<kernel>_<workload>_<walkers>w_<precision>.md), while
    the kernel's source is the one the counters were taken on; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{walkers}w_{precision}.md")
    try:
        vals = {}
        for line in open(path):
            if " = " in line:
                k, v = line.split(" = ", 1)
                vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha256") != kernel_source_hash(kernel):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def roofline(stats0, stats1, precision, kernel, traffic=None):
    """Roofline of one window kernel over the timed region.  Algorithmic
    flops and bytes cover every launch; durations come from the timed
    launches (HIP events attached to the kernel's own dispatch), so the
    per-launch averages of both are divided into each other."""
    pre = KERNELS[kernel][0]
    d = lambda k: stats1[k] - stats0[k]
    timed = d("fold_launches")           # timed windows (one launch of each kernel)
    total = d("windows_enqueued")
    secs_timed = d(f"{pre}_seconds")
    if secs_timed <= 0 or timed <= 0 or total <= 0:
        return None
    secs = secs_timed / timed * total     # estimated time over every launch
    flops = d(f"{pre}_flops")
    nbytes = d(f"{pre}_bytes")
    peak_tf = PEAK["fp64_mfma_TFs"] if precision == "fp64" else PEAK["fp32_mfma_TFs"]
    ai = flops / max(nbytes, 1.0)
    ridge = peak_tf * 1e12 / (PEAK["hbm_GBs"] * 1e9)
    if ai < ridge:
        achieved = nbytes / secs / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
               "frac": achieved / PEAK["hbm_GBs"]}
    else:
        achieved = flops / secs / 1e12
        out = {"bound": "mfma", "achieved": achieved, "peak": peak_tf, "unit": "TFLOP/s",
               "frac": achieved / peak_tf}
    attainable = min(peak_tf, PEAK["hbm_GBs"] * 1e9 * ai / 1e12)
    out.update({"traffic": traffic, "kernel": kernel, "launches": total, "timed_launches": timed,
                "avg_launch_us": secs / total * 1e6, "flops_per_launch": flops / total,
                "bytes_per_launch": nbytes / total, "arith_intensity": ai, "tflops": flops / secs / 1e12,
                "frac_of_mfma_peak": flops / secs / 1e12 / peak_tf,
                "attainable_tflops": attainable, "frac_of_attainable": flops / secs / 1e12 / attainable,
                "seconds_in_timed_region": secs})
    return out


def kernel_us(s0, s1):
    """Average durations of the timed windows' kernels."""
    n = s1["fold_launches"] - s0["fold_launches"]
    if n <= 0:
        return None
    return {k: (s1[f] - s0[f]) / n * 1e6 for k, f in
            (("cand_x", "cand_seconds"), ("ygemm", "y_seconds"), ("fold", "fold_seconds"),
             ("accept_loop", "accept_seconds"), ("window", "window_seconds"))} | \
        {"timed_windows": n, "windows": s1["windows_enqueued"] - s0["windows_enqueued"]}


def fold_ranks(s0, s1):
    """Windows of the timed region by fold rank m: counts per bin (m = 0,
    then 1-4, 5-8, ..., 61-64) and the m range holding the median window."""
    h = [b - a for a, b in zip(s0["fold_rank_hist"], s1["fold_rank_hist"])]
    tot, run, med = sum(h), 0, 0
    for b, n in enumerate(h):
        run += n
        if 2 * run >= tot:
            med = b
            break
    lo, hi = (0, 0) if med == 0 else (4 * med - 3, 4 * med)
    return {"bins_m_0_then_by_4": h, "median_m_range": [lo, hi]}


def run_gpu(precision, steps, warmup, seed_offset=0, graphs=False, workload=None, walkers=1, nfft_hw=0,
            autotune=0, refresh_every=32, drift_tol=0.0):
    import numpy as np
    import torch
    from paper_1901_01047_amd import dcax
    from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs
    workload = workload or WORKLOAD
    cfg = CONFIGS[workload]
    prec = dcax.DCAX_FP64 if precision == "fp64" else dcax.DCAX_FP32_MIXED
    plist = [dcax.make_params(**params_kwargs(workload, seed=cfg["seed"] + seed_offset + i, warmup_sweeps=warmup),
                              precision=prec, refresh_every=refresh_every, drift_tol=drift_tol)
             for i in range(walkers)]
    w = dcax.Walker(plist if walkers > 1 else plist[0])
    w.set_graphs(graphs)
    for i in range(walkers):
        w.set_config(*initial_config(w.Ncs[i], cfg["beta"], cfg["k_init"], cfg["seed"] + 100 + seed_offset + i),
                     walker=i)
    acc, aux = w.new_accumulator()
    if nfft_hw:
        # the measurement is the delayed-NFFT gridding (same chain)
        grid = w.new_nfft_grid()

        def sweep_measure(n):
            w.sweep_measure_nfft(n, grid, aux, nfft_hw)
    else:
        def sweep_measure(n):
            w.sweep_measure(n, acc, aux)
    # the submatrix size comes from the autotuner, whose trial sweeps are
    # part of the warm-up (untimed)
    chosen_ks = None
    if autotune:
        chosen_ks, _ = w.autotune(sweeps_per_trial=autotune)
    sweep_measure(warmup)
    every = 1 if cfg["k_init"] > TIME_ALL_ORDER else TIMING_EVERY
    w.set_timing(every)
    torch.cuda.synchronize()
    s0 = w.stats()
    t0 = time.perf_counter()
    sweep_measure(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = w.stats()
    dt = t1 - t0
    acc_upd = (s1["accepted_insertions"] - s0["accepted_insertions"]) + \
        (s1["accepted_removals"] - s0["accepted_removals"])
    props = s1["proposals"] - s0["proposals"]
    windows = s1["windows"] - s0["windows"]
    kern = {k: roofline(s0, s1, precision, k, kernel_traffic(k, workload, walkers, precision)) for k in KERNELS}
    timed_k = {k: v for k, v in kern.items() if v}
    dominant = max(timed_k, key=lambda k: timed_k[k]["seconds_in_timed_region"]) if timed_k else "k_fold"
    orders = w.orders()
    res = {
        "value": acc_upd / dt, "seconds": dt, "ms_per_step": dt / steps * 1e3,
        "proposals_per_s": props / dt, "acceptance": acc_upd / max(props, 1),
        "mean_order": sum(orders) / walkers, "order_min_max": [min(orders), max(orders)],
        "windows": windows, "walkers": walkers,
        "mean_fold_rank": (s1["flips_folded"] - s0["flips_folded"]) / max(windows, 1),
        "fold_rank_distribution": fold_ranks(s0, s1),
        "roofline": kern[dominant], "dominant_kernel": dominant,
        "kernels": {k: v for k, v in kern.items() if k != dominant},
        "kernel_us_per_window": kernel_us(s0, s1), "timed_share_of_windows": 1.0 / every,
        "sign": s1["sign"], "refresh_every": refresh_every, "drift_tol": drift_tol,
        "walkers_rebuilt_by_drift_control": s1["probe_refreshes"] - s0["probe_refreshes"],
        "refreshes_in_timed_region": steps // refresh_every if refresh_every else 0,
        "refresh_max_drift": s1["max_drift"],
        "aborted_windows": s1["aborted_windows"] - s0["aborted_windows"],
        "submatrix_k": chosen_ks if chosen_ks else plist[0].submatrix_k,
        "kernel_forms": list(w.variants()),
    }
    if graphs:
        # kernels inside a replayed graph cannot be timed one by one: the
        # kernel figures come from eager sweeps right after the timed region
        w.set_graphs(False)
        r0 = w.stats()
        sweep_measure(min(steps, 30))
        torch.cuda.synchronize()
        r1 = w.stats()
        for k in KERNELS:
            x = roofline(r0, r1, precision, k, kernel_traffic(k, workload, walkers, precision))
            if x:
                x["pass"] = "eager sweeps after the timed region"
            if k == dominant:
                res["roofline"] = x
            else:
                res["kernels"][k] = x
    if precision != "fp64" and not nfft_hw:
        # the N error the mixed chain carries at the end of the run, and the
        # error it puts into one measurement of M(K, i w_n): measure, refresh
        # in FP64, measure again
        a1, x1 = w.new_accumulator()
        w.measure(a1, x1)
        drift = w.refresh()
        a2, x2 = w.new_accumulator()
        w.measure(a2, x2)
        torch.cuda.synchronize()
        res["end_of_run_N_drift"] = drift
        res["end_of_run_M_Kw_err_rel_max"] = float((a1 - a2).abs().max() / a2.abs().max())
    cfg_out = w.get_config()
    w.close()
    del acc, aux
    torch.cuda.empty_cache()
    return res, cfg_out


def run_batch(precision, steps, warmup, n_walkers=512, graphs=False, autotune=0):
    """The batched workload: n_walkers walkers of uneven cluster size, U and
    beta in one handle (one launch per kernel covers all of them), free
    running (dcax_run_rounds): a step is one round of four windows per
    walker plus the measurements of the walkers whose sweep ended in it."""
    import torch
    from paper_1901_01047_amd import dcax
    from paper_1901_01047_amd.workloads import batch_configs
    prec = dcax.DCAX_FP64 if precision == "fp64" else dcax.DCAX_FP32_MIXED
    plist = [dcax.make_params(**dict(d, warmup_sweeps=warmup), precision=prec, refresh_every=32)
             for d in batch_configs(n_walkers)]
    w = dcax.Walker(plist)
    w.set_graphs(graphs)
    acc, aux = w.new_accumulator()
    t0 = time.perf_counter()
    w.sweep(warmup)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    # the walkers start empty: the autotuner's trials (ordinary sweeps) run
    # once the warm-up has brought the orders to where they are timed
    chosen = None
    if autotune:
        ks, _ = w.autotune(sweeps_per_trial=autotune)
        chosen = {"submatrix_k": ks, "kernel_forms": list(w.variants())}
    w.set_timing(TIMING_EVERY)
    s0 = w.stats()
    t0 = time.perf_counter()
    w.run_rounds(steps, acc, aux)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s1 = w.stats()
    acc_upd = (s1["accepted_insertions"] - s0["accepted_insertions"]) + \
        (s1["accepted_removals"] - s0["accepted_removals"])
    orders = w.orders()
    res = {"value": acc_upd / dt, "ms_per_step": dt / steps * 1e3, "walkers": n_walkers,
           "proposals_per_s": (s1["proposals"] - s0["proposals"]) / dt,
           "order_min_mean_max": [min(orders), sum(orders) / len(orders), max(orders)],
           "mean_fold_rank": (s1["flips_folded"] - s0["flips_folded"]) / max(s1["windows"] - s0["windows"], 1),
           "fold_rank_distribution": fold_ranks(s0, s1),
           "warmup_seconds": t_warm, "launch": "hipGraph per round" if graphs else "eager launches",
           "autotuned": chosen, "roofline": roofline(s0, s1, precision, "k_fold"),
           "kernels": {k: roofline(s0, s1, precision, k) for k in ("k_cand_x", "k_ygemm")},
           "kernel_us_per_window": kernel_us(s0, s1)}
    w.close()
    return res


def run_nfft(workload, precision="fp64", half_width=8, reps=5):
    """Per-measurement time of the direct contraction (dcax_measure_G) and of
    the delayed-NFFT gridding (dcax_measure_nfft) on one walker of the
    workload after a few sweeps, the one-off transform, and the largest
    difference of the two accumulators relative to their largest entry."""
    import numpy as np
    import torch
    from paper_1901_01047_amd import dcax
    from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs
    cfg = CONFIGS[workload]
    prec = dcax.DCAX_FP64 if precision == "fp64" else dcax.DCAX_FP32_MIXED
    w = dcax.Walker(dcax.make_params(**params_kwargs(workload, warmup_sweeps=2), precision=prec, refresh_every=0))
    w.set_config(*initial_config(w.Ncs[0], cfg["beta"], cfg["k_init"], cfg["seed"] + 100))
    w.sweep(2)
    acc, aux = w.new_accumulator()
    grid = w.new_nfft_grid()
    aux2 = torch.zeros_like(aux)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    direct = timed(lambda: w.measure(acc, aux))
    gridding = timed(lambda: w.measure_nfft(grid, aux2, half_width))
    acc2 = torch.zeros_like(acc)
    transform = timed(lambda: (acc2.zero_(), w.nfft_transform(grid, acc2, half_width)))
    err = float((acc2 - acc).abs().max() / acc.abs().max())
    out = {"workload": workload, "precision": precision, "order": w.order, "n_freq": cfg["n_freq"],
           "half_width": half_width, "direct_ms": direct, "nfft_grid_ms": gridding, "nfft_transform_ms": transform,
           "max_rel_diff": err}
    w.close()
    return out


def run_g2(workload, walkers, precision="fp64", n_w4=16, w_transfer=0, qs=(0,), reps=3):
    """The two-particle measurement (particle-particle up-down, dcax_measure_G2)
    of every walker's configuration after one sweep: milliseconds per
    measurement of the whole batch and the rate of its algorithmic work
    (per walker and spin: the site-blocked transforms 4 k^2 n_w + 8 k Nc n_w^2
    + 16 Nc^3 n_w^2 flops, then 8 n_q (2 n_w4 Nc)^2 for the products), an
    FP64 ALU-bound kernel chain (peak 78.6 TFLOP/s FP64 vector)."""
    import numpy as np
    import torch
    from paper_1901_01047_amd import dcax
    from paper_1901_01047_amd.workloads import CONFIGS, initial_config, params_kwargs
    cfg = CONFIGS[workload]
    prec = dcax.DCAX_FP64 if precision == "fp64" else dcax.DCAX_FP32_MIXED
    plist = [dcax.make_params(**params_kwargs(workload, seed=cfg["seed"] + i, warmup_sweeps=1), precision=prec)
             for i in range(walkers)]
    w = dcax.Walker(plist if walkers > 1 else plist[0])
    for i in range(walkers):
        w.set_config(*initial_config(w.Ncs[i], cfg["beta"], cfg["k_init"], cfg["seed"] + 100 + i), walker=i)
    w.sweep(1)
    g2, sg = w.new_g2_accumulator(n_w4, len(qs))
    w.measure_G2(n_w4, w_transfer, qs, g2, sg)      # first call allocates the scratch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        w.measure_G2(n_w4, w_transfer, qs, g2, sg)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    orders = w.orders()
    Nc = w.Nc
    nw = 2 * n_w4 + w_transfer
    flops = 0.0
    for k in orders:
        kp = k + 16 * Nc
        flops += 2 * (4.0 * kp * kp * nw + 8.0 * kp * Nc * nw * nw + 16.0 * Nc ** 3 * nw * nw) \
            + 8.0 * len(qs) * (2 * n_w4 * Nc) ** 2
    w.close()
    return {"workload": workload, "walkers": walkers, "precision": precision, "n_w4": n_w4,
            "w_transfer": w_transfer, "n_q": len(qs), "mean_order": float(np.mean(orders)),
            "ms_per_measurement": dt * 1e3, "flops_per_measurement": flops, "tflops": flops / dt / 1e12,
            "bound": "alu", "peak_tflops": PEAK["fp64_mfma_TFs"], "frac": flops / dt / 1e12 / PEAK["fp64_mfma_TFs"]}


def cpu_baseline(seconds=15.0, workload=None):
    """The oracle, as it stands, timed on the host: one chain of the same
    workload from the same kind of seeded starting configuration, first with
    the BLAS threads numpy has, then with one thread."""
    from oracle import ctaux
    from paper_1901_01047_amd.workloads import CONFIGS, initial_config
    workload = workload or WORKLOAD
    c = CONFIGS[workload]
    cl = c["cluster"]
    m = ctaux.Model(a1=(cl[0], cl[1]), a2=(cl[2], cl[3]), t=c["t"], tp=c["tp"], U=c["U"], beta=c["beta"],
                    mu=c["mu"], K_exp=c["K_exp"], n_tau=c["n_tau"])
    w = ctaux.Walker(m, seed=c["seed"] + 7, k_s=c["submatrix_k"])
    t_init = time.perf_counter()
    w.set_config(*initial_config(m.Nc, c["beta"], c["k_init"], c["seed"] + 100))
    t_init = time.perf_counter() - t_init
    host_cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        blas_threads = None

    def run_for(sec):
        a0 = w.n_acc_ins + w.n_acc_rem
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < sec:
            w.step()
            n += 1
        dt = time.perf_counter() - t0
        return (w.n_acc_ins + w.n_acc_rem - a0) / dt, n, dt

    v, n, dt = run_for(seconds)
    out = {"value": v, "unit": "updates/s", "cores": blas_threads or 1, "kind": "oracle",
           "host_cores": host_cores, "blas_threads": blas_threads,
           "sample": f"{n} single-vertex proposals of one {workload} chain (order {c['k_init']}, seeded "
                     f"starting configuration, inverted in {t_init:.1f} s, not timed), {dt:.1f} s wall"}
    try:
        # the same chain continued with one BLAS thread
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            v1, n1, dt1 = run_for(seconds / 3)
        out["value_1thread"] = v1
        out["sample_1thread"] = f"the next {n1} proposals with one thread, {dt1:.1f} s wall"
    except Exception:
        pass
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed",
                    help="precision of the headline leg (`value`); the other runs beside it")
    ap.add_argument("--headline-only", action="store_true", help="skip the other precision's leg")
    ap.add_argument("--refresh-every", type=int, default=20,
                    help="sweeps between FP64 refreshes of N (at most --steps, so the timed region holds one)")
    ap.add_argument("--drift-tol", type=float, default=2e-3,
                    help="FP32-mixed legs: after each sweep, rebuild in FP64 every walker whose sampled residual "
                         "of N against its definition exceeds this (0: off)")
    ap.add_argument("--graphs", choices=("on", "off"), default="off",
                    help="replay each sweep as a captured hipGraph")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="workload from paper_1901_01047_amd.workloads.CONFIGS")
    ap.add_argument("--walkers", type=int, default=None,
                    help=f"walkers sharing the GPU (default {WALKERS} for {WORKLOAD}, else 1)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="sweeps per candidate k_s for the autotuner during the warm-up (0: the workload's k_s)")
    ap.add_argument("--nfft", action="store_true",
                    help="also time the delayed-NFFT measurement against the direct one on the workload")
    ap.add_argument("--g2", action="store_true",
                    help="also time the two-particle measurement (n_w4 = 16, q = 0) of the workload's walkers")
    ap.add_argument("--batch", type=int, default=0,
                    help="also run the batched workload with this many walkers (FP64 and FP32-mixed)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (a known-size reference for "
                         "hardware traffic counters) and print its size")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 256 << 20
        x = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(walkers are independent Markov chains: on several GPUs each would run its own walkers "
              "and the accumulators would be all-reduced once at the end)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(2)
    from paper_1901_01047_amd import dcax
    dcax.load()
    from paper_1901_01047_amd.workloads import CONFIGS
    wl = args.workload
    c = CONFIGS[wl]
    walkers = args.walkers if args.walkers else (WALKERS if wl == WORKLOAD else 1)
    graphs = args.graphs == "on"
    at = args.autotune
    re = max(1, min(args.refresh_every, args.steps))
    legs = [args.precision] + ([] if args.headline_only else [p for p in ("mixed", "fp64") if p != args.precision])
    res = {}
    for prec in legs:
        res[prec], _ = run_gpu(prec, args.steps, args.warmup, graphs=graphs, workload=wl, walkers=walkers,
                               autotune=at, refresh_every=re, drift_tol=args.drift_tol if prec == "mixed" else 0.0)
    head = res[args.precision]
    ks_text = f"k_s={head['submatrix_k']} (autotuned)" if at else f"k_s={c['submatrix_k']}"
    mode = "FP32-mixed (N and its GEMMs FP32 on MFMA; ratios, Gamma and refresh FP64)" \
        if args.precision == "mixed" else "FP64"
    out = {
        "metric": "accepted vertex updates/s (CT-AUX walkers) + N-update TFLOP/s (% roofline), FP64 vs FP32-mixed",
        "value": head["value"], "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{wl}: {c['cluster'][0]}x{c['cluster'][3]} periodic Hubbard cluster, t=1, "
                               f"t'={c['tp']}, U={c['U']}, beta={c['beta']}, mu={c['mu']} (n~{c['n_target']}), "
                               f"K=1, expansion order ~{c['k_init']}, {walkers} walker(s), {mode}, {ks_text}, "
                               f"{c['n_freq']} Matsubara freqs measured every sweep, FP64 refresh every {re} sweeps"
                               + (f" and of any walker whose sampled residual of N exceeds {args.drift_tol:g} after a "
                                  "sweep" if args.precision == "mixed" and args.drift_tol > 0 else ""),
                   "step": "1 sweep + 1 measurement of M(K,iw_n) per walker (+ the refresh every "
                           f"{re} sweeps" + (", + the drift-triggered rebuilds)" if args.precision == "mixed" and
                                             args.drift_tol > 0 else ")"),
                   "launch": "hipGraph per sweep" if graphs else "eager launches"},
        "roofline": head["roofline"],
    }
    for prec in legs:
        key = "fp32_mixed" if prec == "mixed" else "fp64"
        out[key] = {k: v for k, v in res[prec].items() if k != "roofline" or prec != args.precision}
    if "mixed" in res and "fp64" in res:
        out["mixed_over_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    if args.nfft:
        out["measurement"] = run_nfft(wl)
        rn, _ = run_gpu("fp64", args.steps, args.warmup, graphs=graphs, workload=wl, walkers=walkers, nfft_hw=8,
                        autotune=at, refresh_every=re)
        out["fp64_nfft_measurement"] = {k: v for k, v in rn.items() if k != "roofline"}
    if args.g2:
        out["two_particle"] = run_g2(wl, walkers)
    if args.batch:
        out["batch"] = {"fp64": run_batch("fp64", args.steps, args.warmup, args.batch, graphs, at),
                        "fp32_mixed": run_batch("mixed", args.steps, args.warmup, args.batch, graphs, at)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

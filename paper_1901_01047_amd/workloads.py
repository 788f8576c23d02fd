"""Synthetic Hubbard-model workloads: parameter sets only, no method arithmetic.

The paper's workloads are Hubbard models fixed entirely by their parameters
(App. B).  These are the configurations the tests (feeding the oracle and
the library) and bench.py read.

mu is the chemical potential measured from the Hartree shift U/2, so mu = 0
is half filling on these bipartite clusters.  For the doped configurations mu
was set by a density scan over many short walkers; "n_target" records the
density it aims at.
"""
BASE_SEED = 985456376   # App. B, "seed" default

CONFIGS = {
    # 2x2 periodic cluster at half filling; small enough for the oracle
    "2x2_U4_b5": dict(cluster=(2, 0, 0, 2), t=1.0, tp=0.0, U=4.0, beta=5.0, mu=0.0, K_exp=1.0,
                      n_tau=1000, submatrix_k=16, n_freq=1024, max_order=256, sweeps=10000,
                      warmup_sweeps=100, seed=BASE_SEED, n_target=1.0, k_init=26),
    # 4x4 cluster, n ~ 0.95, expansion order ~ 300
    "4x4_U4_b10": dict(cluster=(4, 0, 0, 4), t=1.0, tp=0.0, U=4.0, beta=10.0, mu=-0.74, K_exp=1.0,
                       n_tau=2001, submatrix_k=32, n_freq=256, max_order=1024, sweeps=100000,
                       warmup_sweeps=100, seed=BASE_SEED + 2, n_target=0.95, k_init=240),
    # 6x6 cluster, t' = -0.15, n ~ 0.9, expansion order ~ 2000
    "6x6_U6_b20": dict(cluster=(6, 0, 0, 6), t=1.0, tp=-0.15, U=6.0, beta=20.0, mu=-0.8, K_exp=1.0,
                       n_tau=4001, submatrix_k=64, n_freq=256, max_order=4096, sweeps=1000,
                       warmup_sweeps=100, seed=BASE_SEED + 3, n_target=0.90, k_init=2000),
    # 8x8 cluster, n ~ 0.9, expansion order ~ 6000
    "8x8_U7_b30": dict(cluster=(8, 0, 0, 8), t=1.0, tp=0.0, U=7.0, beta=30.0, mu=-0.9, K_exp=1.0,
                       n_tau=6001, submatrix_k=64, n_freq=512, max_order=8192, sweeps=10,
                       warmup_sweeps=10, seed=BASE_SEED + 5000, n_target=0.90, k_init=6000),
}


def initial_config(Nc, beta, k, seed):
    """A seeded starting configuration of k vertices: sites and times uniform,
    and every vertex at a site carrying that site's auxiliary spin (one spin
    per site, +1 or -1 with probability 1/2).

    Equilibrated CT-AUX configurations have strongly site-correlated
    auxiliary spins (the atom's weight (1 + cosh(gamma sum s)) / 2 favours
    aligned spins by e^{2 gamma}); vertices of opposite spin at one site and
    nearby times make N^{-1} nearly singular, which uniformly random spins
    produce in large numbers at these orders.  Returns (site int32,
    tau float64, aux_spin int32)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    site_spin = np.where(rng.random(Nc) < 0.5, 1, -1).astype(np.int32)
    site = rng.integers(0, Nc, size=k).astype(np.int32)
    tau = rng.random(k) * beta
    return site, tau, site_spin[site]


def params_kwargs(name, **over):
    """Keyword arguments for paper_1901_01047_amd.dcax.make_params."""
    c = dict(CONFIGS[name])
    c.update(over)
    keys = ("cluster", "t", "tp", "U", "beta", "mu", "K_exp", "n_tau", "submatrix_k", "n_freq", "max_order",
            "seed", "warmup_sweeps", "sweep_length")
    return {k: c[k] for k in keys if k in c}


# Batched workload: walkers of uneven cluster size, coupling and temperature
# in one handle.  Each walker draws (cluster, U, beta) from a seeded generator;
# a draw is kept when the upper bound of its mean order, K + beta U Nc / 2
# (the atom's mean order tends to K + beta U / 2), lies in [20, 800].
BATCH_CLUSTERS = {4: (2, 0, 0, 2), 8: (2, 2, 2, -2), 16: (4, 0, 0, 4)}
BATCH_BETAS = (5.0, 10.0, 20.0)


def batch_configs(n_walkers=512, seed=BASE_SEED + 4000, K_exp=1.0):
    """Parameter dicts (make_params keywords) of the batched workload."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n_walkers:
        nc = int(rng.choice(sorted(BATCH_CLUSTERS)))
        U = float(rng.uniform(2.0, 8.0))
        beta = float(rng.choice(BATCH_BETAS))
        bound = K_exp + beta * U * nc / 2.0
        if not 20.0 <= bound <= 800.0:
            continue
        w = len(out)
        out.append(dict(cluster=BATCH_CLUSTERS[nc], t=1.0, tp=0.0, U=U, beta=beta, mu=0.0, K_exp=K_exp,
                        n_tau=int(np.ceil(200 * beta)) + 1, submatrix_k=32, n_freq=256, max_order=1152,
                        seed=seed + w, warmup_sweeps=100))
    return out

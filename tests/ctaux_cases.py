"""Test helpers: oracle models and traces in the library's record format.

Imports only the oracle and the workload parameter sets.  Used by the GPU
parity tests (which also import the binding) and by smoke()."""
import numpy as np

from oracle import ctaux
from paper_1901_01047_amd.workloads import CONFIGS

PROPOSAL_DTYPE = np.dtype([("kind", np.int32), ("site", np.int32), ("aux_spin", np.int32),
                           ("accepted", np.int32), ("tau", np.float64), ("id", np.int64),
                           ("u_accept", np.float64)])


def model(name, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    cl = c["cluster"]
    return ctaux.Model(a1=(cl[0], cl[1]), a2=(cl[2], cl[3]), t=c["t"], tp=c["tp"], U=c["U"], beta=c["beta"],
                       mu=c["mu"], K_exp=c["K_exp"], n_tau=c["n_tau"])


def records(trace):
    a = ctaux.trace_arrays(trace)
    r = np.zeros(len(trace), PROPOSAL_DTYPE)
    for f in ("kind", "site", "tau", "id", "u_accept", "accepted"):
        r[f] = a[f]
    r["aux_spin"] = a["aux_spin"]
    return r, a["ratio"]


def oracle_trace(m, seed, k_s, init_order, warm_sweeps, rec_proposals, init=None):
    """Equilibrate an oracle walker, refresh it, then record rec_proposals.

    init: a starting configuration (site, tau, aux_spin), else init_order
    random vertices.  Returns (initial config (r, t, s, id), records, oracle
    ratios, walker)."""
    w = ctaux.Walker(m, seed=seed, k_s=k_s)
    if init is not None:
        w.set_config(*init)
    elif init_order:
        w.random_config(init_order)
    for _ in range(warm_sweeps):
        w.sweep()
    w.refresh()
    init = (w.r.copy(), w.t.copy(), w.s.copy(), w.id.copy())
    w.record = True
    for _ in range(rec_proposals):
        w.step()
    rec, ratios = records(w.trace)
    return init, rec, ratios, w


def exact_replay_with_flip_conditioning(m, init, rec):
    """The extended-precision replay of records (oracle.exact) plus, per
    record, the relative condition number of its ratio with respect to the
    diagonal entries of N it is computed from: 1 for insertions and removals,
    and for a flip of the spin at row p, per spin rho = (1 + e^{-V_p}) N_pp -
    e^{-V_p} (the flip ratio read off N) with condition
    ((1 + e^{-V_p}) |N_pp| + e^{-V_p}) / |rho|, summed over the two spins
    (a flip towards e^{V'} = e^{gamma} is a difference of terms of size
    e^{gamma} N_pp).  Returns (ratios, chain, kappa)."""
    from oracle import exact
    ch = exact.ExactChain(m, *init)
    out, kap = [], []
    for x in rec:
        kind, vid = int(x["kind"]), int(x["id"])
        k = 1.0
        if kind == 2 and vid >= 0:
            p = int(np.nonzero(ch.id == vid)[0][0])
            k = 0.0
            for sp in (0, 1):
                emv = 1.0 / float(ch.ev(ch.s[p], sp))
                npp = float(ch.N[sp][p, p])
                rho = (1.0 + emv) * npp - emv
                k += ((1.0 + emv) * abs(npp) + emv) / abs(rho)
        out.append(ch.step(kind, int(x["site"]), float(x["tau"]), int(x["aux_spin"]), vid, int(x["accepted"])))
        kap.append(max(k, 1.0))
    return np.array(out), ch, np.array(kap)

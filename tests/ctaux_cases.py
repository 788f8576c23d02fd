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

"""Drive an oracle chain: warm-up, sweeps, refreshes and measurements.

Follows the Monte Carlo integration parameters of App. B: warm-up sweeps,
one measurement per sweep ("sweeps-per-measurement" = 1), and a periodic
from-scratch refresh of N by direct inversion.
"""
import numpy as np

from . import ctaux, measure, stats


def run_chain(model, seed, sweeps, warmup=100, n_freq=64, k_s=16, initial_order=0,
              refresh_every=0, record=False):
    w = ctaux.Walker(model, seed, k_s=k_s, record=record)
    if initial_order:
        w.random_config(initial_order)
    warm_orders = []
    for n in range(warmup):
        if 2 * n >= warmup:
            warm_orders.append(w.k)
        w.sweep()
    # measured sweeps have a fixed length: the mean order over the second
    # half of the warm-up (the current order without a warm-up)
    w.freeze_sweep_length(np.mean(warm_orders) if warm_orders else w.k)
    acc = measure.Accumulator(model, n_freq)
    orders = []
    for n in range(sweeps):
        w.sweep()
        if refresh_every and (n + 1) % refresh_every == 0:
            w.refresh()
        acc.measure(w)
        orders.append(w.k)
    return w, acc, np.array(orders)


def estimate_G(model, acc, B=32, taus=None, n_freq=None, spin_average=False):
    """Jackknife estimates of G(K, i w_n) and, optionally, G(K, tau).

    Returns a dict with 'Giw', 'Giw_err' of shape (2, Nc, n_freq) and, if
    taus is given, 'Gtau', 'Gtau_err' of shape (2, Nc, len(taus)); with
    spin_average the leading spin axis is averaged away (inside the
    jackknife, so the error bars are those of the average).
    """
    s, sM, sD = acc.arrays()
    nf = acc.n_freq if n_freq is None else n_freq
    out = {}

    def giw(Mavg):
        g = np.stack([measure.finalize_G_iw(model, Mavg[sp], nf) for sp in range(2)])
        return g.mean(axis=0) if spin_average else g

    def gtau(Mavg, Davg):
        g = np.stack([measure.G_tau_from_iw(model, Mavg[sp], Davg[sp], nf, taus) for sp in range(2)])
        return g.mean(axis=0) if spin_average else g

    sMb = stats.bins(sM[:, :, :, :nf], B)
    sDb = stats.bins(sD, B)
    sb = stats.bins(s, B)
    tot_M, tot_D, tot_s = sMb.sum(0), sDb.sum(0), sb.sum()
    out["Giw"] = giw(tot_M / tot_s)
    loo = np.array([giw((tot_M - sMb[b]) / (tot_s - sb[b])) for b in range(B)])
    out["Giw_err"] = np.sqrt((B - 1) / B * ((loo.real - loo.real.mean(0)) ** 2).sum(0)) + \
        1j * np.sqrt((B - 1) / B * ((loo.imag - loo.imag.mean(0)) ** 2).sum(0))
    if taus is not None:
        out["Gtau"] = gtau(tot_M / tot_s, tot_D / tot_s)
        loo = np.array([gtau((tot_M - sMb[b]) / (tot_s - sb[b]), (tot_D - sDb[b]) / (tot_s - sb[b]))
                        for b in range(B)])
        out["Gtau_err"] = np.sqrt((B - 1) / B * ((loo - loo.mean(0)) ** 2).sum(0))
    out["sign"] = s.mean()
    return out

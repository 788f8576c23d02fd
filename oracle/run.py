"""Drive an oracle chain: warm-up, sweeps, refreshes and measurements.

Follows the Monte Carlo integration parameters of App. B: warm-up sweeps,
one measurement per sweep ("sweeps-per-measurement" = 1), and a periodic
from-scratch refresh of N by direct inversion.
"""
import numpy as np

from . import ctaux, measure, stats


def run_chain(model, seed, sweeps, warmup=100, n_freq=64, k_s=16, initial_order=0,
              refresh_every=0, record=False, p_flip=0.0):
    w = ctaux.Walker(model, seed, k_s=k_s, record=record, p_flip=p_flip)
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
    jackknife, so the error bars are those of the average).  Errors of the
    complex G(K, i w_n) are sigma_re + 1j sigma_im.
    """
    s, sM, sD = acc.arrays()
    nf = acc.n_freq if n_freq is None else n_freq
    out = {}

    def giw(tot_M, tot_D, tot_s):
        Mavg = tot_M / tot_s
        g = np.stack([measure.finalize_G_iw(model, Mavg[sp], nf, spin=sp) for sp in range(2)])
        return g.mean(axis=0) if spin_average else g

    def gtau(tot_M, tot_D, tot_s):
        Mavg, Davg = tot_M / tot_s, tot_D / tot_s
        g = np.stack([measure.G_tau_from_iw(model, Mavg[sp], Davg[sp], nf, taus, spin=sp) for sp in range(2)])
        return g.mean(axis=0) if spin_average else g

    binned = (stats.bins(sM[:, :, :, :nf], B), stats.bins(sD, B), stats.bins(s, B))
    out["Giw"], out["Giw_err"] = stats.jackknife(giw, binned)
    if taus is not None:
        out["Gtau"], out["Gtau_err"] = stats.jackknife(gtau, binned)
    out["sign"] = s.mean()
    return out

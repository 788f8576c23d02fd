"""Binning and jackknife error bars for sign-weighted Monte Carlo averages.

Sec. 2.3 notes that away from half filling the averages carry a sign; every
observable is the ratio <s O> / <s>.  Measurements are split into B
consecutive bins and the ratio's error comes from the jackknife over bins.
"""
import numpy as np


def bins(x, B):
    n = (len(x) // B) * B
    x = np.asarray(x)[:n]
    return x.reshape((B, n // B) + x.shape[1:]).mean(axis=1)


def jackknife_ratio(num, den, B=32):
    """Mean and jackknife sigma of sum(num)/sum(den) over B bins.

    num: (n, ...) per-measurement s*O ; den: (n,) per-measurement s.
    """
    nb = bins(num, B)
    db = bins(den, B)
    tot_n, tot_d = nb.sum(axis=0), db.sum()
    est = tot_n / tot_d
    loo = np.array([(tot_n - nb[b]) / (tot_d - db[b]) for b in range(B)])
    mean_loo = loo.mean(axis=0)
    var = (B - 1) / B * ((loo - mean_loo) ** 2).sum(axis=0)
    return est, np.sqrt(var)

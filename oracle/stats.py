"""Binning and jackknife error bars for sign-weighted Monte Carlo averages.

Sec. 2.3 notes that away from half filling the averages carry a sign; every
observable is a function of ratios <s O> / <s>.  Measurements are split into
B consecutive bins and the error of the estimator comes from the jackknife
over bins: the estimator is re-evaluated with each bin left out, and

    sigma^2 = (B - 1) / B * sum_b (f_(b) - mean_b f_(b))^2.

Bins must be longer than the chain's autocorrelation time; the check is that
sigma does not change (beyond its own statistical error, about
1/sqrt(2 (B - 1)) relative) when the bins are made twice as long
(``bin_halving``).
"""
import numpy as np


def bins(x, B):
    """Means of B consecutive bins along the first axis (a tail that does
    not fill a bin is dropped)."""
    n = (len(x) // B) * B
    if n == 0:
        raise ValueError("fewer samples than bins")
    x = np.asarray(x)[:n]
    return x.reshape((B, n // B) + x.shape[1:]).mean(axis=1)


def _spread(loo):
    B = len(loo)
    return np.sqrt((B - 1) / B * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))


def jackknife(fn, binned):
    """Estimate fn(totals) and its jackknife sigma.

    binned: sequence of arrays whose first axis runs over the B bins (bin
    means); fn takes one total per array (the sum over bins, or that sum
    with one bin left out) and returns an array.  A complex result gets the
    sigma of its real and of its imaginary part, as sigma_re + 1j sigma_im."""
    binned = [np.asarray(b) for b in binned]
    B = len(binned[0])
    tot = [b.sum(axis=0) for b in binned]
    est = np.asarray(fn(*tot))
    loo = np.array([fn(*[t - b[i] for t, b in zip(tot, binned)]) for i in range(B)])
    if np.iscomplexobj(loo):
        err = _spread(loo.real) + 1j * _spread(loo.imag)
    else:
        err = _spread(loo)
    return est, err


def jackknife_ratio(num, den, B=32):
    """Mean and jackknife sigma of sum(num) / sum(den) over B bins.

    num: (n, ...) per-measurement s*O ; den: (n,) per-measurement s."""
    nb, db = bins(num, B), bins(den, B)
    shape = (-1,) + (1,) * (nb.ndim - 1)
    return jackknife(lambda n, d: n / d, (nb, db.reshape(shape)))


def bin_halving(num, den, B=32):
    """Jackknife sigma of sum(num) / sum(den) with B bins and with B/2 bins
    (twice as long).  Their ratio stays near 1 when the bins are longer than
    the autocorrelation time and grows above 1 when they are not."""
    _, e1 = jackknife_ratio(num, den, B)
    _, e2 = jackknife_ratio(num, den, B // 2)
    return e1, e2

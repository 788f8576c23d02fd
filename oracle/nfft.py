"""Delayed-NFFT measurement of M (Sec. 2.3, "Non-equidistant FFT measurements").

Test infrastructure: only tests/, the smoke check and the benchmark's CPU leg
use the oracle.

The paper grids samples placed at random times onto an equispaced imaginary-
time grid by convolving them with a localized kernel, accumulates the gridded
data over the whole run, and performs a single FFT at the end, dividing by the
kernel's Fourier coefficients (its convolution theorem and NFFT equations).
The quantity is the one the direct sums of measure.M_K_iw compute,

    M(K, i w_n) = (1/Nc) sum_ij e^{i w_n (tau_i - tau_j)} e^{-i K (r_i - r_j)} M_ij,

which depends on a pair (i, j) only through tau_i - tau_j and the cluster
displacement d = r_i - r_j (modulo the superlattice).  So the accumulated grid
holds one row of L points per displacement d, per spin.

Readings (the paper fixes neither the kernel nor the oversampling):
* the kernel is the Gaussian of Greengard & Lee, "Accelerating the nonuniform
  fast Fourier transform", SIAM Review 46 (2004) 443, with oversampling ratio
  2 and spreading half-width M_sp grid points.  Truncating it at M_sp points
  costs exp(-0.75 pi M_sp); sampling the convolved function on the grid
  aliases the highest needed harmonic (2 n_freq on the 2 beta circle) with
  harmonic 6 n_freq, whose kernel coefficient is smaller by
  exp(-t (36 - 4) n_freq^2 pi^2 / beta^2) = exp(-(2/3) pi M_sp) for the width
  t below.  The error is therefore of order exp(-(2/3) pi M_sp) times the sum
  of |samples| (error_scale);
* fermionic functions are antiperiodic in beta, i.e. periodic in 2 beta with
  odd harmonics only: w_n = (2n+1) pi / beta is harmonic 2n+1 of the 2 beta
  circle.  The n_freq positive frequencies and their negatives (the gridded
  data are real) are 4 n_freq harmonics; oversampled twice, 8 n_freq grid
  points on [0, 2 beta), of which the antiperiodic half [0, beta) is stored:
  L = 4 n_freq points, spacing h = beta / L;
* a sample at tau_i - tau_j < 0 is the antiperiodic image at
  tau_i - tau_j + beta with the opposite sign (e^{i w_n beta} = -1).

Gridding (per sample f at s in [0, beta)): grid point j in
[l0 - M_sp + 1, l0 + M_sp], l0 = floor(s / h), receives
f exp(-(s - j h)^2 / (4 t)), with t = M_sp beta^2 / (48 pi n_freq^2) (the
Greengard-Lee width, tau_GL = pi M_sp / (M^2 R (R - 1/2)) for M = 4 n_freq
harmonics and R = 2, mapped from the 2 pi circle to the 2 beta one); a point
outside [0, L) wraps by L with a factor -1 (antiperiodicity).

Finalisation: F(w_n) = h sum_l G[l] e^{i w_n l h} / g(w_n) with
g(w) = sqrt(4 pi t) exp(-t w^2), the Fourier transform of the kernel; then
M(K, i w_n) = (1/Nc) sum_d e^{-i K r_d} F_d(w_n).  The sum over l is written
as a plain DFT (one matrix product), not an FFT: the result is the same.
"""
import math

import numpy as np

from .measure import matsubara


def grid_size(n_freq):
    """Grid points L on [0, beta) for n_freq positive Matsubara frequencies."""
    return 4 * n_freq


def kernel_width(beta, n_freq, m_sp):
    """Gaussian variance parameter t (kernel exp(-x^2 / (4 t)))."""
    return m_sp * beta * beta / (48.0 * math.pi * n_freq * n_freq)


def error_scale(m_sp):
    """Error per unit sample weight: the aliasing factor exp(-(2/3) pi M_sp)."""
    return math.exp(-2.0 * math.pi * m_sp / 3.0)


def grid_samples(s, f, beta, n_freq, m_sp, out=None):
    """Add samples f at times s (all in [0, beta)) to a grid of L points."""
    L = grid_size(n_freq)
    if 2 * m_sp > L:
        raise ValueError("kernel wider than the grid")
    h = beta / L
    t = kernel_width(beta, n_freq, m_sp)
    g = np.zeros(L) if out is None else out
    s = np.asarray(s, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    l0 = np.floor(s / h).astype(np.int64)
    for q in range(-m_sp + 1, m_sp + 1):
        j = l0 + q
        w = np.exp(-(s - j * h) ** 2 / (4.0 * t))
        sign = np.where((j < 0) | (j >= L), -1.0, 1.0)
        np.add.at(g, np.mod(j, L), sign * w * f)
    return g


def grid_M(model, r, tau, M, n_freq, m_sp, out=None):
    """Grid of one configuration's M for one spin: shape (Nc, L), row d the
    pairs with r_i - r_j = d.  Adds into out when given."""
    Nc = model.Nc
    L = grid_size(n_freq)
    G = np.zeros((Nc, L)) if out is None else out
    k = len(r)
    if k == 0:
        return G
    r = np.asarray(r)
    tau = np.asarray(tau, dtype=np.float64)
    dt = tau[:, None] - tau[None, :]
    f = np.where(dt < 0.0, -M, M)
    s = np.where(dt < 0.0, dt + model.beta, dt)
    d = model.diff[r[:, None], r[None, :]]
    for dd in range(Nc):
        sel = d == dd
        if sel.any():
            grid_samples(s[sel], f[sel], model.beta, n_freq, m_sp, out=G[dd])
    return G


def transform(G, beta, n_freq, m_sp):
    """F(w_n) for each row of an accumulated grid (rows, L) -> (rows, n_freq)."""
    L = grid_size(n_freq)
    h = beta / L
    t = kernel_width(beta, n_freq, m_sp)
    w = matsubara(n_freq, beta)
    ghat = math.sqrt(4.0 * math.pi * t) * np.exp(-t * w * w)
    phase = np.exp(1j * np.outer(np.arange(L) * h, w))          # (L, n_freq)
    return h * (np.asarray(G) @ phase) / ghat


def M_K_iw_from_grid(model, G, n_freq, m_sp):
    """M(K, i w_n) (Nc, n_freq) from one spin's accumulated grid (Nc, L)."""
    F = transform(G, model.beta, n_freq, m_sp)                  # (Nc_d, n_freq)
    ph = np.exp(-1j * (model.K @ model.sites.astype(np.float64).T))   # (Nc_K, Nc_d)
    return ph @ F / model.Nc

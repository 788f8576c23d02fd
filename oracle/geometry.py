"""Periodic square-lattice clusters given by superlattice vectors.

The paper specifies a DCA cluster by its real-space superlattice vectors in the
lattice basis (App. B, domains group, "cluster").  The cluster is the quotient
Z^2 / (a1 Z + a2 Z); it has Nc = |det[a1 a2]| sites and Nc momenta K with
K . a_i in 2 pi Z (Sec. 2.1, the cluster momenta that label the patches).

Enumeration convention (an interface shared with the HIP library, implemented
separately on each side):

* a site's canonical representative is A f with A = [a1 a2] (columns) and the
  fractional coordinates f wrapped into [0, 1); sites are ordered by the
  representative's (y, x), ascending;
* a momentum is K = 2 pi q / |D| with integer q in [0, |D|)^2 and
  q . a_i = 0 (mod |D|), D = det A; momenta are ordered by (q_y, q_x).
"""
import numpy as np


def _det(a1, a2):
    return a1[0] * a2[1] - a1[1] * a2[0]


def canonical_site(r, a1, a2):
    """Canonical representative of integer point r modulo the superlattice."""
    D = _det(a1, a2)
    if D == 0:
        raise ValueError("degenerate superlattice")
    # adj(A) r, with A = [[a1x, a2x], [a1y, a2y]]
    n0 = a2[1] * r[0] - a2[0] * r[1]
    n1 = -a1[1] * r[0] + a1[0] * r[1]
    s = 1 if D > 0 else -1
    ad = abs(D)
    w0 = (s * n0) % ad
    w1 = (s * n1) % ad
    x = (a1[0] * w0 + a2[0] * w1) // ad
    y = (a1[1] * w0 + a2[1] * w1) // ad
    return (int(x), int(y))


def cluster_sites(a1, a2):
    """Integer coordinates of the Nc cluster sites, shape (Nc, 2)."""
    D = abs(_det(a1, a2))
    xs = [0, a1[0], a2[0], a1[0] + a2[0]]
    ys = [0, a1[1], a2[1], a1[1] + a2[1]]
    reps = set()
    for y in range(min(ys) - 1, max(ys) + 2):
        for x in range(min(xs) - 1, max(xs) + 2):
            reps.add(canonical_site((x, y), a1, a2))
    reps = sorted(reps, key=lambda p: (p[1], p[0]))
    if len(reps) != D:
        raise AssertionError("site enumeration failed")
    return np.array(reps, dtype=np.int64)


def cluster_momenta(a1, a2):
    """Cluster momenta K, shape (Nc, 2), each component in [0, 2 pi)."""
    D = abs(_det(a1, a2))
    out = []
    for qy in range(D):
        for qx in range(D):
            if (qx * a1[0] + qy * a1[1]) % D == 0 and (qx * a2[0] + qy * a2[1]) % D == 0:
                out.append((qx, qy))
    if len(out) != D:
        raise AssertionError("momentum enumeration failed")
    return 2.0 * np.pi * np.array(out, dtype=np.float64) / D


def diff_table(a1, a2):
    """d[i, j] = index of the site equal to r_i - r_j modulo the superlattice."""
    sites = cluster_sites(a1, a2)
    index = {tuple(map(int, s)): n for n, s in enumerate(sites)}
    Nc = len(sites)
    d = np.empty((Nc, Nc), dtype=np.int64)
    for i in range(Nc):
        for j in range(Nc):
            r = canonical_site((sites[i][0] - sites[j][0], sites[i][1] - sites[j][1]), a1, a2)
            d[i, j] = index[r]
    return d


def dispersion(K, t=1.0, tp=0.0):
    """eps_K = -2t (cos Kx + cos Ky) - 4t' cos Kx cos Ky (square lattice)."""
    cx, cy = np.cos(K[:, 0]), np.cos(K[:, 1])
    return -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy


def hopping_matrix(a1, a2, t=1.0, tp=0.0):
    """Cluster hopping t_ij = (1/Nc) sum_K e^{i K (r_i - r_j)} eps_K (real)."""
    sites = cluster_sites(a1, a2).astype(np.float64)
    K = cluster_momenta(a1, a2)
    eps = dispersion(K, t, tp)
    Nc = len(sites)
    ph = np.exp(1j * sites @ K.T)          # (Nc sites, Nc momenta)
    tij = (ph * eps[None, :]) @ ph.conj().T / Nc
    if np.max(np.abs(tij.imag)) > 1e-12:
        raise AssertionError("hopping matrix not real")
    return tij.real

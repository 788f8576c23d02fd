"""Python binding of the CT-AUX walker library (include/dcax.h).

Argument marshalling only: every step of the Markov chain, the updates of N,
the refresh and the measurement run in the HIP kernels of ``libdcax.so``.
PyTorch provides device memory (through the library's allocator callback,
backed by torch's caching allocator) and the HIP stream.

The shared library is built in-tree by ``paper_1901_01047_amd.build``; if it
is missing, importing this module raises -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcax.so")

DCAX_ABI_VERSION = 1
DCAX_FP64 = 0
REPLAY_STATIC_MAX = 65536     # dcax.h DCAX_REPLAY_STATIC_MAX
DCAX_VARIANT_AUTO, DCAX_VARIANT_TILED, DCAX_VARIANT_WIDE, DCAX_VARIANT_NARROW = 0, 1, 2, 3
DCAX_FP32_MIXED = 1

STATUS = {0: "DCAX_OK", -1: "DCAX_E_INVAL", -2: "DCAX_E_NOMEM", -3: "DCAX_E_HIP", -4: "DCAX_E_NUMERIC",
          -5: "DCAX_E_CAPACITY", -6: "DCAX_E_TRACE", -7: "DCAX_E_STATE"}


class DcaxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("cluster", ctypes.c_int32 * 4),
                ("t", ctypes.c_double), ("tp", ctypes.c_double), ("U", ctypes.c_double),
                ("beta", ctypes.c_double), ("mu", ctypes.c_double), ("K_exp", ctypes.c_double),
                ("n_tau", ctypes.c_int32), ("precision", ctypes.c_int32), ("submatrix_k", ctypes.c_int32),
                ("refresh_every", ctypes.c_int32), ("max_order", ctypes.c_int32), ("n_freq", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("warmup_sweeps", ctypes.c_int32), ("sweep_length", ctypes.c_int32),
                ("n_spin_tables", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("g0_tau", ctypes.c_void_p), ("g0_Kw", ctypes.c_void_p),
                ("flip_share", ctypes.c_double), ("touched_twice", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("drift_tol", ctypes.c_double)]


class Vertex(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("site", ctypes.c_int32), ("aux_spin", ctypes.c_int32),
                ("tau", ctypes.c_double)]


class Proposal(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("site", ctypes.c_int32), ("aux_spin", ctypes.c_int32),
                ("accepted", ctypes.c_int32), ("tau", ctypes.c_double), ("id", ctypes.c_int64),
                ("u_accept", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("proposals", ctypes.c_int64), ("accepted_insertions", ctypes.c_int64),
                ("accepted_removals", ctypes.c_int64), ("windows", ctypes.c_int64),
                ("flips_folded", ctypes.c_int64), ("decision_mismatches", ctypes.c_int64),
                ("sweeps", ctypes.c_int64), ("sign", ctypes.c_double), ("fold_flops", ctypes.c_double),
                ("fold_bytes", ctypes.c_double), ("fold_seconds", ctypes.c_double),
                ("fold_launches", ctypes.c_int64), ("accept_seconds", ctypes.c_double),
                ("window_seconds", ctypes.c_double), ("aborted_windows", ctypes.c_int64),
                ("last_drift", ctypes.c_double), ("max_drift", ctypes.c_double),
                ("windows_enqueued", ctypes.c_int64), ("fold_rank_hist", ctypes.c_int64 * 17),
                ("cand_flops", ctypes.c_double), ("cand_bytes", ctypes.c_double), ("cand_seconds", ctypes.c_double),
                ("y_flops", ctypes.c_double), ("y_bytes", ctypes.c_double), ("y_seconds", ctypes.c_double),
                ("accepted_flips", ctypes.c_int64), ("neglected", ctypes.c_int64), ("probes", ctypes.c_int64),
                ("probe_refreshes", ctypes.c_int64), ("last_probe", ctypes.c_double)]


class DcaParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("cluster", ctypes.c_int32 * 4),
                ("t", ctypes.c_double), ("tp", ctypes.c_double), ("beta", ctypes.c_double),
                ("mu", ctypes.c_double), ("h", ctypes.c_double), ("n_spin", ctypes.c_int32),
                ("n_freq", ctypes.c_int32), ("n_cg", ctypes.c_int32), ("n_tau", ctypes.c_int32),
                ("patch_points", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class DcaReport(ctypes.Structure):
    _fields_ = [("max_change", ctypes.c_double), ("sign", ctypes.c_double), ("mean_order", ctypes.c_double),
                ("measurements", ctypes.c_int64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


PROPOSAL_DTYPE = np.dtype([("kind", np.int32), ("site", np.int32), ("aux_spin", np.int32),
                           ("accepted", np.int32), ("tau", np.float64), ("id", np.int64),
                           ("u_accept", np.float64)])
VERTEX_DTYPE = np.dtype([("id", np.int64), ("site", np.int32), ("aux_spin", np.int32), ("tau", np.float64)])

# exported symbols, in the order include/dcax.h declares them
EXPORTS = ("dcax_walker_create", "dcax_walker_destroy", "dcax_sweep", "dcax_sweep_replay_static", "dcax_refresh", "dcax_measure_G",
           "dcax_sweep_measure", "dcax_run_rounds", "dcax_measure_G2", "dcax_measure_nfft", "dcax_sweep_measure_nfft",
           "dcax_nfft_transform",
           "dcax_finalize_G", "dcax_get_order", "dcax_copy_N", "dcax_get_config", "dcax_set_config",
           "dcax_set_submatrix_k", "dcax_autotune", "dcax_set_graphs", "dcax_set_variants", "dcax_get_variants", "dcax_probe_N", "dcax_get_stats", "dcax_set_timing", "dcax_copy_g0_table",
           "dcax_cluster", "dcax_dca_create", "dcax_dca_destroy", "dcax_dca_coarse_grain", "dcax_dca_g0_tables",
           "dcax_dca_cluster_G", "dcax_dca_self_energy", "dcax_dca_iterate", "dcax_set_g0", "dcax_last_error")

_lib = None


def load():
    """Load libdcax.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; run paper_1901_01047_amd.build.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "dcax_walker_create": [P(Params), ctypes.c_int32, P(Allocator), vp, P(vp)],
        "dcax_walker_destroy": [vp],
        "dcax_sweep": [vp, ctypes.c_int32, vp, ctypes.c_int64, vp],
        "dcax_sweep_replay_static": [vp, vp, ctypes.c_int64, vp],
        "dcax_refresh": [vp, P(ctypes.c_double)],
        "dcax_measure_G": [vp, vp, vp],
        "dcax_sweep_measure": [vp, ctypes.c_int32, vp, vp],
        "dcax_run_rounds": [vp, ctypes.c_int32, vp, vp],
        "dcax_measure_G2": [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp],
        "dcax_finalize_G": [vp, vp, vp, vp, ctypes.c_int32, vp],
        "dcax_get_order": [vp, ctypes.c_int32, P(ctypes.c_int32)],
        "dcax_copy_N": [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64, vp],
        "dcax_get_config": [vp, ctypes.c_int32, vp, ctypes.c_int32, P(ctypes.c_int32)],
        "dcax_set_config": [vp, ctypes.c_int32, vp, ctypes.c_int32],
        "dcax_get_stats": [vp, ctypes.c_int32, P(Stats)],
        "dcax_set_timing": [vp, ctypes.c_int32],
        "dcax_set_submatrix_k": [vp, ctypes.c_int32, ctypes.c_int32],
        "dcax_autotune": [vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_double)],
        "dcax_set_graphs": [vp, ctypes.c_int32],
        "dcax_set_variants": [vp, ctypes.c_int32, ctypes.c_int32],
        "dcax_get_variants": [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
        "dcax_copy_g0_table": [vp, ctypes.c_int32, vp],
        "dcax_probe_N": [vp, vp],
        "dcax_cluster": [P(Params), P(ctypes.c_int32), vp, vp],
        "dcax_dca_create": [P(DcaParams), P(Allocator), vp, P(vp)],
        "dcax_dca_destroy": [vp],
        "dcax_dca_coarse_grain": [vp, vp, vp, vp],
        "dcax_dca_g0_tables": [vp, vp, vp],
        "dcax_dca_cluster_G": [vp, vp, vp, vp, ctypes.c_int32, vp],
        "dcax_dca_self_energy": [vp, vp, vp, vp, ctypes.c_double, vp, P(ctypes.c_double)],
        "dcax_dca_iterate": [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, vp, vp, P(DcaReport)],
        "dcax_set_g0": [vp, vp, ctypes.c_int32, vp, ctypes.c_int32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.dcax_last_error.argtypes = []
    lib.dcax_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st):
    if st != 0:
        raise DcaxError(st, load().dcax_last_error().decode())


def make_params(cluster=(2, 0, 0, 2), t=1.0, tp=0.0, U=4.0, beta=5.0, mu=0.0, K_exp=1.0, n_tau=1000,
                precision=DCAX_FP64, submatrix_k=16, refresh_every=0, max_order=512, n_freq=64,
                seed=985456376, warmup_sweeps=20, sweep_length=0, g0_tau=None, g0_Kw=None, flip_share=0.0,
                touched_twice=0, drift_tol=0.0):
    """g0_tau: optional bare propagator tables, float64 [n_spin_tables][Nc][n_tau]
    (or [Nc][n_tau] for one table) in the standard convention; g0_Kw: optional
    complex128 [n_spin_tables][Nc][n_freq] G0(K, i w_n) for finalize.  The
    arrays are kept alive with the returned Params (the library copies them
    when a Walker is created)."""
    p = Params()
    p.abi_version = DCAX_ABI_VERSION
    for i in range(4):
        p.cluster[i] = int(cluster[i])
    p.t, p.tp, p.U, p.beta, p.mu, p.K_exp = t, tp, U, beta, mu, K_exp
    p.n_tau, p.precision, p.submatrix_k = n_tau, precision, submatrix_k
    p.refresh_every, p.max_order, p.n_freq, p.seed = refresh_every, max_order, n_freq, seed
    p.warmup_sweeps, p.sweep_length = warmup_sweeps, sweep_length
    p.flip_share, p.touched_twice, p.drift_tol = flip_share, touched_twice, drift_tol
    keep = []
    if g0_tau is not None:
        t = np.ascontiguousarray(g0_tau, dtype=np.float64)
        if t.ndim == 2:
            t = t[None]
        if t.ndim != 3 or t.shape[0] not in (1, 2) or t.shape[2] != n_tau:
            raise ValueError("g0_tau must be [n_spin_tables][Nc][n_tau] with n_spin_tables 1 or 2")
        p.n_spin_tables = t.shape[0]
        p.g0_tau = t.ctypes.data
        keep.append(t)
        if g0_Kw is not None:
            g = np.ascontiguousarray(g0_Kw, dtype=np.complex128)
            if g.ndim == 2:
                g = g[None]
            if g.shape[0] != t.shape[0] or g.shape[1] != t.shape[1] or g.shape[2] != n_freq:
                raise ValueError("g0_Kw must be [n_spin_tables][Nc][n_freq] complex")
            p.g0_Kw = g.ctypes.data
            keep.append(g)
    elif g0_Kw is not None:
        raise ValueError("g0_Kw needs g0_tau")
    p._keep = keep
    return p


def cluster(params):
    """(sites[Nc, 2] int32, momenta[Nc, 2] float64) by the library's enumeration."""
    lib = load()
    n = ctypes.c_int32()
    _check(lib.dcax_cluster(ctypes.byref(params), ctypes.byref(n), None, None))
    sites = np.zeros((n.value, 2), np.int32)
    K = np.zeros((n.value, 2), np.float64)
    _check(lib.dcax_cluster(ctypes.byref(params), ctypes.byref(n), sites.ctypes.data, K.ctypes.data))
    return sites, K


class Walker:
    """A batch of CT-AUX walkers (one by default) on the current torch device and stream.

    `params` is one Params or a sequence of them (one per walker; all share
    the precision).  Per-walker methods take `walker=0`."""

    def __init__(self, params, device=None, stream=None):
        import torch
        self._torch = torch
        lib = load()
        plist = list(params) if isinstance(params, (list, tuple)) else [params]
        self.plist = plist
        self.params = plist[0]
        self.W = len(plist)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        dev_index = self.device.index
        sptr = self.stream.cuda_stream

        def _alloc(nbytes, ctx):
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev_index, sptr)

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self._allocator = Allocator(self._alloc_cb, self._free_cb, None)
        arr = (Params * self.W)(*plist)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.dcax_walker_create(arr, self.W, ctypes.byref(self._allocator), ctypes.c_void_p(sptr),
                                          ctypes.byref(h)))
        self._h = h
        self.sites, self.K, self.Ncs = [], [], []
        for p in plist:
            sites, K = cluster(p)
            self.sites.append(sites)
            self.K.append(K)
            self.Ncs.append(len(sites))
        self.Nc = self.Ncs[0]
        # accumulator layout: walker blocks of [2][Nc][max(n_freq, 1)][2] doubles, in walker order
        self.acc_sizes = [2 * nc * max(p.n_freq, 1) * 2 for nc, p in zip(self.Ncs, plist)]
        self.acc_offsets = np.concatenate([[0], np.cumsum(self.acc_sizes)[:-1]]).astype(np.int64)

    def close(self):
        if getattr(self, "_h", None):
            load().dcax_walker_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- chain ---------------------------------------------------------
    def sweep(self, n=1):
        _check(load().dcax_sweep(self._h, int(n), None, 0, None))

    def replay(self, records):
        """Replay a structured array of PROPOSAL_DTYPE (single-walker handle); returns the ratios."""
        rec = np.ascontiguousarray(records, dtype=PROPOSAL_DTYPE)
        ratios = np.zeros(len(rec), np.float64)
        _check(load().dcax_sweep(self._h, 0, rec.ctypes.data, len(rec), ratios.ctypes.data))
        return ratios

    def replay_static(self, records):
        """As replay, staging the records in the library's fixed per-GPU buffer
        (no allocation; at most REPLAY_STATIC_MAX records per call)."""
        rec = np.ascontiguousarray(records, dtype=PROPOSAL_DTYPE)
        ratios = np.zeros(len(rec), np.float64)
        _check(load().dcax_sweep_replay_static(self._h, rec.ctypes.data, len(rec), ratios.ctypes.data))
        return ratios

    def refresh(self):
        d = ctypes.c_double()
        _check(load().dcax_refresh(self._h, ctypes.byref(d)))
        return d.value

    # -- configuration -------------------------------------------------
    def order_of(self, walker=0):
        k = ctypes.c_int32()
        _check(load().dcax_get_order(self._h, int(walker), ctypes.byref(k)))
        return k.value

    @property
    def order(self):
        return self.order_of(0)

    def orders(self):
        return [self.order_of(i) for i in range(self.W)]

    def set_config(self, site, tau, aux_spin, ids=None, walker=0):
        k = len(site)
        v = np.zeros(k, VERTEX_DTYPE)
        v["site"], v["tau"], v["aux_spin"] = site, tau, aux_spin
        v["id"] = np.arange(k) if ids is None else ids
        _check(load().dcax_set_config(self._h, int(walker), v.ctypes.data if k else None, k))

    def get_config(self, walker=0):
        k = self.order_of(walker)
        v = np.zeros(max(k, 1), VERTEX_DTYPE)
        kk = ctypes.c_int32()
        _check(load().dcax_get_config(self._h, int(walker), v.ctypes.data, len(v), ctypes.byref(kk)))
        return v[:kk.value]

    def copy_N(self, spin, walker=0):
        """(ids, N) in canonical (id ascending) order, float64."""
        k = self.order_of(walker)
        out = np.zeros((k, k), np.float64)
        ids = np.zeros(k, np.int64)
        if k:
            _check(load().dcax_copy_N(self._h, int(walker), int(spin), out.ctypes.data, k, ids.ctypes.data))
        return ids, out

    def stats(self, walker=-1):
        """Counters of one walker, or summed over the batch (walker=-1)."""
        s = Stats()
        _check(load().dcax_get_stats(self._h, int(walker), ctypes.byref(s)))
        out = {f: getattr(s, f) for f, _ in Stats._fields_}
        out["fold_rank_hist"] = list(s.fold_rank_hist)
        return out

    def set_submatrix_k(self, ks, walker=-1):
        _check(load().dcax_set_submatrix_k(self._h, int(walker), int(ks)))

    def autotune(self, sweeps_per_trial=5):
        """Pick the submatrix size with the most accepted updates/s; returns (k_s, rate)."""
        ks = ctypes.c_int32()
        rate = ctypes.c_double()
        _check(load().dcax_autotune(self._h, int(sweeps_per_trial), ctypes.byref(ks), ctypes.byref(rate)))
        return ks.value, rate.value

    def set_graphs(self, on=True):
        _check(load().dcax_set_graphs(self._h, 1 if on else 0))

    def probe(self):
        """Largest sampled residual of each walker's N against its definition
        (see dcax_probe_N), [W]."""
        out = np.zeros(self.W, np.float64)
        _check(load().dcax_probe_N(self._h, out.ctypes.data))
        return out

    def set_variants(self, cand_rows=0, y_columns=0):
        """Kernel forms of the candidate-row and Y-column products: 0 auto,
        1 tiled (LDS), 2 wide, 3 narrow (see dcax_set_variants)."""
        _check(load().dcax_set_variants(self._h, int(cand_rows), int(y_columns)))

    def variants(self):
        """(candidate-row form, Y-column form) in use."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load().dcax_get_variants(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_timing(self, on=True):
        """on: True / 1 times every window, n > 1 a pseudo-random 1/n of them, 0 / False stops."""
        _check(load().dcax_set_timing(self._h, int(on)))

    def g0_table(self, walker=0):
        p = self.plist[walker]
        t = np.zeros((self.Ncs[walker], p.n_tau), np.float64)
        _check(load().dcax_copy_g0_table(self._h, int(walker), t.ctypes.data))
        return t

    # -- measurement ---------------------------------------------------
    def new_accumulator(self):
        """(acc, aux): acc holds every walker's [2][Nc][n_freq][2] block; aux is [W][3]."""
        torch = self._torch
        acc = torch.zeros(int(sum(self.acc_sizes)), dtype=torch.float64, device=self.device)
        aux = torch.zeros((self.W, 3), dtype=torch.float64, device=self.device)
        if self.W == 1:
            acc = acc.view(2, self.Nc, max(self.params.n_freq, 1), 2)
            aux = aux.view(3)
        return acc, aux

    def acc_block(self, acc, walker):
        """One walker's [2][Nc][n_freq][2] view of a batch accumulator."""
        flat = acc.reshape(-1)
        o, n = int(self.acc_offsets[walker]), self.acc_sizes[walker]
        return flat[o:o + n].view(2, self.Ncs[walker], max(self.plist[walker].n_freq, 1), 2)

    def measure(self, acc, aux):
        _check(load().dcax_measure_G(self._h, ctypes.c_void_p(acc.data_ptr()), ctypes.c_void_p(aux.data_ptr())))

    def new_g2_accumulator(self, n_w4, n_q):
        """(g2, sign) for measure_G2: complex [n_q][Nc][2 n_w4][Nc][2 n_w4] as
        float64 (..., 2) and one float64."""
        torch = self._torch
        n4 = 2 * n_w4
        g2 = torch.zeros((n_q, self.Nc, n4, self.Nc, n4, 2), dtype=torch.float64, device=self.device)
        return g2, torch.zeros(1, dtype=torch.float64, device=self.device)

    def measure_G2(self, n_w4, w_transfer, qs, g2, sign):
        """Two-particle (particle-particle up-down) measurement of every
        walker's configuration into (g2, sign); qs: momentum indices."""
        q = np.ascontiguousarray(qs, dtype=np.int32)
        _check(load().dcax_measure_G2(self._h, int(n_w4), int(w_transfer), len(q), q.ctypes.data,
                                      ctypes.c_void_p(g2.data_ptr()), ctypes.c_void_p(sign.data_ptr())))

    def new_nfft_grid(self):
        """Zeroed delayed-NFFT grid: one [2][Nc][4 n_freq] block per walker."""
        torch = self._torch
        return torch.zeros(2 * int(sum(self.acc_sizes)), dtype=torch.float64, device=self.device)

    def measure_nfft(self, grid, aux, half_width=8):
        """Delayed-NFFT measurement: grid += sign * gridded M, aux as for measure."""
        _check(load().dcax_measure_nfft(self._h, int(half_width), ctypes.c_void_p(grid.data_ptr()),
                                        ctypes.c_void_p(aux.data_ptr())))

    def sweep_measure_nfft(self, n_sweeps, grid, aux, half_width=8):
        """n_sweeps device-scheduled sweeps, each followed by a delayed-NFFT measurement."""
        _check(load().dcax_sweep_measure_nfft(self._h, int(n_sweeps), int(half_width),
                                              ctypes.c_void_p(grid.data_ptr()), ctypes.c_void_p(aux.data_ptr())))

    def nfft_transform(self, grid, acc, half_width=8):
        """acc += the transform of an accumulated grid (the layout of measure's acc)."""
        _check(load().dcax_nfft_transform(self._h, int(half_width), ctypes.c_void_p(grid.data_ptr()),
                                          ctypes.c_void_p(acc.data_ptr())))

    def run_rounds(self, n_rounds, acc, aux):
        """Free-running batch: every walker sweeps and measures for n_rounds rounds."""
        _check(load().dcax_run_rounds(self._h, int(n_rounds), ctypes.c_void_p(acc.data_ptr()),
                                      ctypes.c_void_p(aux.data_ptr())))

    def sweep_measure(self, n_sweeps, acc, aux):
        """n_sweeps generator sweeps, each followed by a measurement into (acc, aux)."""
        _check(load().dcax_sweep_measure(self._h, int(n_sweeps), ctypes.c_void_p(acc.data_ptr()),
                                         ctypes.c_void_p(aux.data_ptr())))

    def finalize(self, acc, aux, n_tau_out=0):
        torch = self._torch
        Giw = torch.zeros_like(acc)
        n_gt = 2 * sum(self.Ncs) * max(n_tau_out, 1)
        Gt = torch.zeros(n_gt, dtype=torch.float64, device=self.device)
        _check(load().dcax_finalize_G(self._h, ctypes.c_void_p(acc.data_ptr()), ctypes.c_void_p(aux.data_ptr()),
                                      ctypes.c_void_p(Giw.data_ptr()), int(n_tau_out),
                                      ctypes.c_void_p(Gt.data_ptr()) if n_tau_out else None))
        if self.W == 1:
            Gt = Gt.view(2, self.Nc, max(n_tau_out, 1))
        return Giw, (Gt if n_tau_out else None)

    def set_g0(self, g0_tau, g0_Kw=None):
        """Install a new bare propagator in every walker (device tensors):
        g0_tau float64 [n_spin_tables][Nc][n_tau], g0_Kw float64
        [n_spin_tables][Nc][stride][2] (its first n_freq frequencies are
        taken); N is rebuilt for the current configurations."""
        nt = int(g0_tau.shape[0])
        stride = int(g0_Kw.shape[2]) if g0_Kw is not None else 0
        _check(load().dcax_set_g0(self._h, ctypes.c_void_p(g0_tau.data_ptr()), nt,
                                  ctypes.c_void_p(g0_Kw.data_ptr()) if g0_Kw is not None else None, stride))


def make_dca_params(cluster=(2, 0, 0, 2), t=1.0, tp=0.0, beta=5.0, mu=0.0, h=0.0, n_spin=1, n_freq=64, n_cg=2048,
                    n_tau=1000, patch_points=8):
    p = DcaParams()
    p.abi_version = DCAX_ABI_VERSION
    for i in range(4):
        p.cluster[i] = int(cluster[i])
    p.t, p.tp, p.beta, p.mu, p.h = t, tp, beta, mu, h
    p.n_spin, p.n_freq, p.n_cg, p.n_tau, p.patch_points = n_spin, n_freq, n_cg, n_tau, patch_points
    return p


class DCA:
    """The DCA self-consistency loop (Sec. 2.1) on the current torch device.

    Arrays are torch float64 device tensors; complex quantities carry a last
    axis (re, im): sigma and G [n_spin][Nc][n_freq][2], gbar and g0
    [n_spin][Nc][n_cg][2], tables [n_spin][Nc][n_tau]."""

    def __init__(self, params, device=None, stream=None):
        import torch
        self._torch = torch
        self.p = params
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        dev_index = self.device.index
        sptr = self.stream.cuda_stream

        def _alloc(nbytes, ctx):
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev_index, sptr)

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self._allocator = Allocator(self._alloc_cb, self._free_cb, None)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(load().dcax_dca_create(ctypes.byref(params), ctypes.byref(self._allocator), ctypes.c_void_p(sptr),
                                          ctypes.byref(h)))
        self._h = h
        q = Params()
        q.cluster[:] = params.cluster[:]
        self.Nc = len(cluster(q)[0])

    def close(self):
        if getattr(self, "_h", None):
            load().dcax_dca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _z(self, nf):
        return self._torch.zeros((self.p.n_spin, self.Nc, nf, 2), dtype=self._torch.float64, device=self.device)

    def new_sigma(self):
        return self._z(self.p.n_freq)

    def coarse_grain(self, sigma):
        """(gbar, g0): coarse-grained G and cluster-excluded G0cal."""
        gbar, g0 = self._z(self.p.n_cg), self._z(self.p.n_cg)
        _check(load().dcax_dca_coarse_grain(self._h, ctypes.c_void_p(sigma.data_ptr()),
                                            ctypes.c_void_p(gbar.data_ptr()), ctypes.c_void_p(g0.data_ptr())))
        return gbar, g0

    def g0_tables(self, g0):
        tab = self._torch.zeros((self.p.n_spin, self.Nc, self.p.n_tau), dtype=self._torch.float64,
                                device=self.device)
        _check(load().dcax_dca_g0_tables(self._h, ctypes.c_void_p(g0.data_ptr()), ctypes.c_void_p(tab.data_ptr())))
        return tab

    def cluster_G(self, g0, acc, aux, n_blocks=1):
        G = self._z(self.p.n_freq)
        _check(load().dcax_dca_cluster_G(self._h, ctypes.c_void_p(g0.data_ptr()), ctypes.c_void_p(acc.data_ptr()),
                                         ctypes.c_void_p(aux.data_ptr()), int(n_blocks), ctypes.c_void_p(G.data_ptr())))
        return G

    def self_energy(self, g0, G, sigma_old, alpha=1.0, out=None):
        """(new sigma, max |change|)."""
        out = self._z(self.p.n_freq) if out is None else out
        chg = ctypes.c_double()
        _check(load().dcax_dca_self_energy(self._h, ctypes.c_void_p(g0.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                           ctypes.c_void_p(sigma_old.data_ptr()), float(alpha),
                                           ctypes.c_void_p(out.data_ptr()), ctypes.byref(chg)))
        return out, chg.value

    def walker_params(self, sigma, **kw):
        """Params for walkers of this loop, with G0cal from `sigma` as their
        initial propagator (host copies of the tables)."""
        _, g0 = self.coarse_grain(sigma)
        tab = self.g0_tables(g0).cpu().numpy()
        g = g0.cpu().numpy()
        gkw = g[:, :, :self.p.n_freq, 0] + 1j * g[:, :, :self.p.n_freq, 1]
        return make_params(cluster=tuple(self.p.cluster), beta=self.p.beta, n_tau=self.p.n_tau, n_freq=self.p.n_freq,
                           g0_tau=tab, g0_Kw=gkw, **kw)

    def iterate(self, walker, sigma, warmup_sweeps, measure_sweeps, alpha=1.0, want_G=False):
        """One DCA iteration with `walker` (a Walker) as the cluster solver;
        sigma is updated in place.  Returns (report dict, G or None)."""
        rep = DcaReport()
        G = self._z(self.p.n_freq) if want_G else None
        _check(load().dcax_dca_iterate(self._h, walker._h, int(warmup_sweeps), int(measure_sweeps), float(alpha),
                                       ctypes.c_void_p(sigma.data_ptr()),
                                       ctypes.c_void_p(G.data_ptr()) if G is not None else None,
                                       ctypes.byref(rep)))
        return {f: getattr(rep, f) for f, _ in DcaReport._fields_}, G

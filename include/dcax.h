/*
 * dcax.h -- C ABI of the CT-AUX walker library for AMD MI355X (gfx950).
 *
 * The library implements the hot path of the continuous-time auxiliary-field
 * (CT-AUX) cluster solver of Hahner et al., "DCA++: A software framework to
 * solve correlated electron problems with modern quantum cluster methods",
 * Sec. 2.3: Metropolis insertion and removal of auxiliary-field vertices,
 * their fusion into submatrix (delayed) updates of the walker matrices
 * N_sigma = [e^{V_sigma} - G0 (e^{V_sigma} - 1)]^{-1}, and the measurement of
 * M = (e^V - 1) N that yields G(K, i w_n) = G0 - G0 <M> G0 / beta.
 *
 * Conventions
 *   - All functions return a dcax_status; no C++ exception crosses the ABI.
 *   - Pointers named *_dev are device pointers on the walker's GPU; all other
 *     pointers are host pointers.  The caller owns every buffer it passes.
 *   - Every call enqueues its GPU work on the stream given at creation.  Calls
 *     that return host data (ratio_out, drift_out, the copy/get functions)
 *     synchronise that stream before returning.
 *   - Kernels latch numerical faults (a non-finite ratio, a zero pivot, an
 *     order beyond max_order) in a device status word.  The next synchronising
 *     call returns it; from then on the walker answers DCAX_E_STATE until
 *     dcax_set_config() installs a fresh configuration.
 *   - Handles are not thread-safe; distinct handles are independent.
 *   - Sites are numbered by the cluster enumeration below; vertices carry a
 *     64-bit id, assigned in order of accepted insertion (the initial
 *     configuration takes ids 0..k-1 unless dcax_set_config gives others).
 *
 * Cluster enumeration (App. B, domains group "cluster": superlattice vectors
 * in the lattice basis).  Sites are the quotient Z^2 / (a1 Z + a2 Z); a site's
 * canonical representative is A f with A = [a1 a2] and fractional coordinates
 * f wrapped into [0, 1); sites are ordered by the representative's (y, x).
 * Momenta are K = 2 pi q / |det A| with integer q in [0, |det A|)^2 and
 * q . a_i = 0 mod |det A|, ordered by (q_y, q_x).
 */
#ifndef DCAX_H
#define DCAX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DCAX_ABI_VERSION 1

typedef enum {
  DCAX_OK = 0,
  DCAX_E_INVAL = -1,    /* invalid argument; nothing was enqueued */
  DCAX_E_NOMEM = -2,    /* the allocator returned NULL */
  DCAX_E_HIP = -3,      /* a HIP runtime call failed (message in dcax_last_error) */
  DCAX_E_NUMERIC = -4,  /* a kernel met a non-finite ratio or a zero pivot */
  DCAX_E_CAPACITY = -5, /* the order would exceed max_order */
  DCAX_E_TRACE = -6,    /* a replay record names a vertex id that is not present */
  DCAX_E_STATE = -7     /* the walker holds a latched error; call dcax_set_config */
} dcax_status;

typedef enum {
  DCAX_FP64 = 0,        /* N, candidate GEMMs, fold and measurement in FP64 */
  DCAX_FP32_MIXED = 1   /* N and its GEMMs in FP32 (MFMA, FP32 accumulation);
                           Gamma^{-1}, ratios and the refresh stay FP64 */
} dcax_precision;

typedef struct dcax_walker_s* dcax_walker;

/* Device memory source: every byte of device memory the library uses comes
 * from it (the library never calls hipMalloc itself).  alloc(bytes, ctx)
 * returns a device pointer aligned to 256 bytes or NULL; free(ptr, ctx)
 * releases it.  Required (dcax_walker_create answers DCAX_E_INVAL without
 * one); a C caller may pass a thin wrapper of hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} dcax_allocator;

/* One vertex of a configuration (Sec. 2.3: a site, an imaginary time and an
 * auxiliary spin s = +1/-1 coupling n_up - n_down at that site). */
typedef struct {
  int64_t id;
  int32_t site;
  int32_t aux_spin;
  double tau;           /* in [0, beta) */
} dcax_vertex;

/* One recorded proposal, replayed with its decision forced (dcax_sweep).
 * kind 0 = insertion at (site, tau, aux_spin), taking `id` if accepted;
 * kind 1 = removal of the vertex with id `id` (id -1: removal proposed at
 * order 0, a rejected no-op); kind 2 = flip of the auxiliary spin of the
 * vertex with id `id` (id -1: a no-op at order 0).  u_accept is the uniform the decision was drawn
 * with; the library counts decisions on which its own ratio would disagree. */
typedef struct {
  int32_t kind;
  int32_t site;
  int32_t aux_spin;
  int32_t accepted;
  double tau;
  int64_t id;
  double u_accept;
} dcax_proposal;

/* Model and run parameters (App. B names in quotes). */
typedef struct {
  int32_t abi_version;     /* must be DCAX_ABI_VERSION */
  int32_t cluster[4];      /* "cluster": a1 = (c[0], c[1]), a2 = (c[2], c[3]) */
  double t, tp;            /* nearest and next-nearest neighbour hopping */
  double U;                /* "U", on-site interaction */
  double beta;             /* "beta", inverse temperature */
  double mu;               /* chemical potential measured from U/2 (mu = 0: half filling) */
  double K_exp;            /* "expansion-parameter-K" */
  int32_t n_tau;           /* G0 table points on [0+, beta-], both ends included */
  int32_t precision;       /* dcax_precision */
  int32_t submatrix_k;     /* "max-submatrix-size", 1..64 (changeable later) */
  int32_t refresh_every;   /* sweeps between FP64 refreshes of N inside dcax_sweep; 0 = never */
  int32_t max_order;       /* largest expansion order the walker may reach */
  int32_t n_freq;          /* Matsubara frequencies measured, n = 0 .. n_freq-1; with n_freq > 0
                              the cluster may have at most 256 sites */
  uint64_t seed;           /* "seed" of the walker's counter-based generator */
  int32_t warmup_sweeps;   /* "warm-up-sweeps": generator sweeps after which the sweep length freezes */
  int32_t sweep_length;    /* proposals per sweep (rounded up to a multiple of submatrix_k);
                              0 = taken from the warm-up, see dcax_sweep */
  /* The bare propagator of the cluster problem (Sec. 2.1: the cluster-
   * excluded G0 is the solver's input in the DCA loop).
   *   n_spin_tables = 0: the library builds G0 of the isolated periodic
   *     cluster from t, tp and mu (finite-size mode), one table for both spins;
   *   1: g0_tau holds one table for both spins; 2: one per spin (up, then
   *     down), e.g. for a magnetic field or a symmetry-broken G0.
   * g0_tau (host, [n_spin_tables][Nc][n_tau], copied by dcax_walker_create):
   *   G0_sigma(r_d, tau_l) in the standard convention G0 = -<T c c+>_0, d the
   *   displacement r_i - r_j as a site of the cluster enumeration below,
   *   tau_l = l beta / (n_tau - 1), point 0 the 0+ value and point n_tau - 1
   *   the beta- value (interpolated linearly between points).
   * g0_Kw (host, nullable, complex [n_spin_tables][Nc][n_freq] as (re, im),
   *   copied): G0_sigma(K, i w_n), n = 0 .. n_freq - 1, for dcax_finalize_G;
   *   without it dcax_finalize_G answers DCAX_E_INVAL for this walker.
   * t, tp and mu are ignored when n_spin_tables > 0. */
  int32_t n_spin_tables;
  int32_t reserved;        /* must be 0 */
  const double* g0_tau;
  const double* g0_Kw;
  /* Spin-flip proposals (Sec. 2.3's figure of the CT-AUX moves): a share
   * flip_share in [0, 1) of the generator's proposals flips the auxiliary
   * spin of a uniformly chosen vertex (accepted with |prod_sigma ratio|);
   * insertions and removals share the rest equally.
   * touched_twice (Sec. 2.3, a spin touched twice within one submatrix
   * window; App. B "neglect-Bennett-updates"):
   *   0 = exact: the window closes before such a proposal, which opens the
   *       next one ("abort"; a removal of a spin inserted in the same window
   *       is still done exactly);
   *   1 = neglect: such a proposal is rejected outright.  This breaks detailed
   *       balance; its bias is measured against the exact chain. */
  double flip_share;
  int32_t touched_twice;
  int32_t reserved2;       /* must be 0 */
  /* Drift control (finite, >= 0; 0 = off; walker 0's value governs the
   * handle): at the end of each of a walker's sweeps its N is probed against
   * its definition (sampled entries of N^{-1} N, as dcax_probe_N) and, when
   * the largest sampled residual exceeds drift_tol, rebuilt in FP64 before
   * the sweep's measurement is taken (all such walkers of a batch in one
   * rebuild pass).  Device-scheduled sweeps (dcax_sweep_measure,
   * dcax_run_rounds) probe on the device before each measurement and hold
   * the walker until the host has rebuilt it; dcax_sweep probes after each
   * sweep.  Meant for FP32-mixed chains, whose rounding grows between
   * refreshes and can be amplified by an update with a small ratio. */
  double drift_tol;
} dcax_params;

/* Counters since creation or the last dcax_set_config (timings and drifts
 * are per handle). */
typedef struct {
  int64_t proposals;
  int64_t accepted_insertions;
  int64_t accepted_removals;
  int64_t windows;          /* submatrix windows folded */
  int64_t flips_folded;     /* sum over windows of the fold rank m */
  int64_t decision_mismatches; /* replay: u_accept on the other side of |R| */
  int64_t sweeps;
  double sign;              /* sign of the current configuration */
  double fold_flops;        /* algorithmic flops of the rank-m folds, 2 k'^2 m per spin */
  double fold_bytes;        /* algorithmic bytes of the folds: N read and written once */
  double fold_seconds;      /* fold kernel time summed over the timed windows (dcax_set_timing) */
  int64_t fold_launches;    /* timed windows (one fold launch each) */
  double accept_seconds;    /* accept-loop kernel time summed over the timed windows */
  double window_seconds;    /* whole-window time summed over the timed windows */
  int64_t aborted_windows;  /* windows closed early by a carried removal */
  double last_drift;        /* drift of the last refresh inside dcax_sweep */
  double max_drift;         /* largest such drift */
  int64_t windows_enqueued; /* windows launched while timing was on, timed or not
                               (fold_launches / windows_enqueued is the sampled share) */
  int64_t fold_rank_hist[17]; /* windows by fold rank m: [0] m = 0, [b] 4b-3 <= m <= 4b */
  double cand_flops;        /* algorithmic flops of the candidate-row products X_C = W_C N, 2 k^2 n_C per spin */
  double cand_bytes;        /* their algorithmic bytes: N read once, W_C read and X_C written */
  double cand_seconds;      /* candidate-row kernel time summed over the timed windows */
  double y_flops;           /* algorithmic flops of the Y columns N g_{I,c} of inserted spins, 2 k^2 m_i per spin */
  double y_bytes;           /* their algorithmic bytes: N read once, g columns read and Y written */
  double y_seconds;         /* Y-column kernel time summed over the timed windows */
  int64_t accepted_flips;   /* accepted spin flips */
  int64_t neglected;        /* proposals rejected as touching a spin twice (touched_twice = 1) */
  int64_t probes;           /* probe passes of N (dcax_probe_N, the drift control after a
                               dcax_sweep sweep or a round of device-scheduled sweeps) */
  int64_t probe_refreshes;  /* walkers rebuilt by the drift control */
  double last_probe;        /* largest residual of the last probe pass over the walkers (of
                               device-scheduled sweeps: over the walkers it held) */
} dcax_stats;

/* Create a batch of n_walkers independent walkers (Markov chains; Sec. 3.1,
 * "Parallelization": all walkers of a process on its GPU).  p points to
 * n_walkers parameter sets, which may differ in every field except
 * precision.  Copies the parameters, builds each walker's cluster tables and
 * G0(r, tau) table on the GPU (the bare propagator of the isolated cluster,
 * Sec. 2.1) and allocates memory for its max_order.  Configurations start
 * empty.  Every later call covers the whole batch in one launch per kernel.
 * `stream` is a hipStream_t (NULL: the default stream). */
dcax_status dcax_walker_create(const dcax_params* p, int32_t n_walkers, const dcax_allocator* a,
                               void* stream, dcax_walker* out);
dcax_status dcax_walker_destroy(dcax_walker w);

/* Run Markov-chain proposals (Sec. 2.3, Metropolis insertion/removal fused
 * into submatrix updates of at most submatrix_k proposals).
 *   replay == NULL: n_sweeps sweeps of every walker from its own generator.
 *     A sweep is a fixed number L of proposals, rounded up to a multiple of
 *     submatrix_k: L = sweep_length if that is positive; otherwise, during
 *     the first warmup_sweeps sweeps L = max(k, 1) with k the order at the
 *     sweep's start, and when they end L freezes at the mean order over
 *     their second half, which holds at least the last of them (rounded,
 *     at least 1).  A length that depends on the
 *     current state would bias every quantity measured between sweeps, so
 *     measurements belong after the warm-up.  dcax_set_config restarts the
 *     warm-up count.  N is refreshed every refresh_every sweeps (walker 0's
 *     parameter).
 *   replay != NULL (single-walker handles only): the n_replay records are
 *     replayed in order with forced decisions (n_sweeps is ignored);
 *     ratio_out (nullable, length n_replay) receives the library's full
 *     acceptance ratio R for each record. */
dcax_status dcax_sweep(dcax_walker w, int32_t n_sweeps, const dcax_proposal* replay,
                       int64_t n_replay, double* ratio_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the replay
 * of dcax_sweep (same records, same kernels, same ratios and N), with the
 * records and their ratios staged in a fixed device buffer the library holds
 * on each GPU (DCAX_REPLAY_STATIC_MAX records, 3 MiB, kept until the process
 * ends) instead of memory from the walker's allocator, which dcax_sweep's
 * replay obtains on first use and grows.  n_replay above the limit answers
 * DCAX_E_INVAL before any work.  Every call on one GPU shares that buffer:
 * calls that overlap (other threads or streams of the same GPU) race. */
#define DCAX_REPLAY_STATIC_MAX 65536
dcax_status dcax_sweep_replay_static(dcax_walker w, const dcax_proposal* replay, int64_t n_replay,
                                     double* ratio_out);

/* Rebuild N_sigma = [e^V - g (e^V - 1)]^{-1} of every walker from scratch in
 * FP64 (gathers plus Gauss-Jordan inversion with partial pivoting).
 * drift_out (nullable) receives max|N_before - N_after| / max|N_after|, the
 * largest over spins and walkers. */
dcax_status dcax_refresh(dcax_walker w, double* drift_out);

/* Accumulate the measurement of every walker's configuration (Sec. 2.3):
 *   acc_dev holds one block per walker, in walker order, each complex128
 *   [2 spins][Nc momenta][max(n_freq, 1)] (interleaved re, im), so walker i's
 *   block starts 4 sum_{j<i} Nc_j max(n_freq_j, 1) doubles in;
 *   each block += sign * M_sigma(K, i w_n), with
 *     M_sigma(K, i w_n) = (1/Nc) sum_ij e^{i (w_n tau_i - K r_i)} [(e^V - 1) N]_ij
 *                                        e^{-i (w_n tau_j - K r_j)};
 *   aux_dev ([n_walkers][3] doubles) += [sign, sign (1/Nc) tr M_up, sign (1/Nc) tr M_down].
 * The trace terms are the equal-time coefficient of G's 1/(i w)^2 tail. */
dcax_status dcax_measure_G(dcax_walker w, double* acc_dev, double* aux_dev);

/* The Monte Carlo loop with one measurement per sweep (the paper's
 * sweeps-per-measurement = 1): the result of n_sweeps times dcax_sweep(w, 1,
 * NULL, 0, NULL) followed by dcax_measure_G(w, acc_dev, aux_dev), bit for
 * bit, except that refreshes fall at other sweeps.  The sweeps are scheduled
 * on the device: each walker begins its next sweep when its previous one has
 * been measured, without host round trips; the call returns when every
 * walker has made n_sweeps sweeps.  Same errors and accumulator layout as
 * those two calls. */
dcax_status dcax_sweep_measure(dcax_walker w, int32_t n_sweeps, double* acc_dev, double* aux_dev);

/* Free-running batch (Sec. 3.1: walkers of a process run independently):
 * every walker sweeps continuously, with a measurement after each of its
 * sweeps, for n_rounds rounds of windows (four windows per round for a
 * batch, one sweep's worth for a single walker), then finishes the sweep it
 * is in.  Walkers with short sweeps therefore make more sweeps than long
 * ones instead of waiting for them; each walker's chain, sweep boundaries
 * and measurements are exactly those of dcax_sweep_measure.  Same
 * accumulators and errors as dcax_measure_G. */
dcax_status dcax_run_rounds(dcax_walker w, int32_t n_rounds, double* acc_dev, double* aux_dev);

/* G(K, i w_n) = G0 - G0 <M> G0 / beta with <M> = acc / sign (Sec. 2.3), and
 * G(K, tau) on n_tau_out points tau_l = l beta / (n_tau_out - 1) (l = 0 is 0+,
 * the last point beta-) from the frequency data with the 1/(i w)^2 tail
 * removed and added back in closed form.  Inputs as accumulated by
 * dcax_measure_G; outputs (device): Giw_dev in the layout of acc_dev,
 * Gtau_dev double, one [2][Nc][n_tau_out] block per walker in walker order
 * (nullable when n_tau_out == 0). */
dcax_status dcax_finalize_G(dcax_walker w, const double* acc_dev, const double* aux_dev,
                            double* Giw_dev, int32_t n_tau_out, double* Gtau_dev);

/* Two-particle Green's function of the cluster, particle-particle up-down
 * channel (Sec. 2.5, the G_2 of the Bethe-Salpeter equation; App. B
 * four-point type PARTICLE_PARTICLE_UP_DOWN, momentum and frequency
 * transfer).  For every walker's current configuration (its spins are
 * independent quadratic problems, so Wick's theorem factorises the up-down
 * function):
 *   g2[iq][K1][c1][K2][c2] += sign * G_up(k1, k2) G_down(q - k1, q - k2),
 *   sign_dev[0] += sign,
 * with k = (K, i w_n), n = c - n_w4 (c = 0 .. 2 n_w4 - 1), q = (K_{q_host[iq]},
 * i 2 pi w_transfer / beta), q - k = (K_q - K, i w_{w_transfer - 1 - n}), and
 * the configuration's Green's function (not diagonal in k)
 *   G_sigma(k1, k2) = G0(k1) delta - G0(k1) M(k1, k2) G0(k2) / beta,
 *   M(k1, k2) = (1/Nc) sum_ij e^{i (w1 tau_i - K1 r_i)} [(e^V - 1) N]_ij e^{-i (w2 tau_j - K2 r_j)}
 * (its diagonal is the measurement of dcax_measure_G; G0 at negative
 * frequencies is the conjugate of G0 at positive ones).  G2 / sum(sign) is
 * the Monte Carlo estimate.
 *   n_w4: 1..64 fermionic frequencies per sign ("four-point-fermionic-
 *     frequencies"); w_transfer: 0..64; q_host: n_q (1..4096) momentum
 *     indices of the cluster enumeration (host, copied);
 *   g2_dev: complex [n_q][Nc][2 n_w4][Nc][2 n_w4] (device, +=, summed over
 *     the walkers); sign_dev: one double (device, +=).
 * The walkers of the handle must share cluster and beta; a walker created
 * with g0_tau needs g0_Kw with n_freq >= n_w4 + w_transfer.  Work per walker
 * and spin ~ k^2 n_w + k Nc n_w^2 + 2 Nc^3 n_w^2 complex operations (n_w =
 * 2 n_w4 + w_transfer); scratch from the walker's allocator on first use.
 * Synchronises the stream before returning. */
dcax_status dcax_measure_G2(dcax_walker w, int32_t n_w4, int32_t w_transfer, int32_t n_q, const int32_t* q_host,
                            double* g2_dev, double* sign_dev);

/* Delayed-NFFT measurement (Sec. 2.3, non-equidistant FFT measurements): the
 * same quantity as dcax_measure_G, accumulated as gridded samples.  Every
 * pair (i, j) of every walker's configuration contributes M_ij = (e^{V_i} -
 * 1) N_ij at tau_i - tau_j (a negative difference as its antiperiodic image
 * at + beta with the opposite sign) to row d = r_i - r_j of an equispaced
 * grid of L = 4 n_freq points on [0, beta), spread with the Gaussian kernel
 * of Greengard & Lee (SIAM Review 46, 2004; oversampling ratio 2) over
 * 2 half_width points, and the configuration's sign times that grid is added
 * to grid_dev.
 *   half_width: kernel half-width in grid points, 2..16, the same in every
 *     call on one grid; the transform's error is of order
 *     exp(-(2/3) pi half_width) times sum |M_ij| (3.5e-6 at 6, 5.3e-8 at 8).
 *   grid_dev (device, doubles): one [2][Nc][4 n_freq] block per walker, in
 *     walker order (twice the size of dcax_measure_G's accumulator), +=.
 *   aux_dev: as for dcax_measure_G.
 * Needs 1 <= n_freq <= 2048 and 2 half_width <= 4 n_freq for every walker
 * (DCAX_E_INVAL otherwise).  Enqueued on the walker's stream. */
dcax_status dcax_measure_nfft(dcax_walker w, int32_t half_width, double* grid_dev, double* aux_dev);

/* dcax_sweep_measure with the delayed-NFFT measurement: the result of
 * n_sweeps times dcax_sweep(w, 1, NULL, 0, NULL) followed by
 * dcax_measure_nfft(w, half_width, grid_dev, aux_dev), scheduled on the
 * device the same way (each walker's chain, sweep boundaries and measured
 * configurations as with dcax_sweep_measure).  Same arguments and errors as
 * dcax_measure_nfft. */
dcax_status dcax_sweep_measure_nfft(dcax_walker w, int32_t n_sweeps, int32_t half_width, double* grid_dev,
                                    double* aux_dev);

/* The single transform at the end of a delayed-NFFT run: for every walker,
 * spin, displacement row d and frequency w_n = (2n+1) pi / beta,
 *   F_d(w_n) = h sum_l G_d[l] e^{i w_n l h} / g(w_n),  h = beta / (4 n_freq),
 * with g the kernel's Fourier transform, and
 *   acc_dev[K][n] += (1/Nc) sum_d e^{-i K r_d} F_d(w_n),
 * i.e. what dcax_measure_G would have accumulated over the same
 * configurations, to the NFFT error.  grid_dev as filled by dcax_measure_nfft
 * with the same half_width; acc_dev in dcax_measure_G's layout (start from
 * zeros to obtain that accumulator; then dcax_finalize_G applies).  Uses the
 * walker's measurement scratch; enqueued on the walker's stream. */
dcax_status dcax_nfft_transform(dcax_walker w, int32_t half_width, const double* grid_dev, double* acc_dev);

/* Change the submatrix size of one walker (walker >= 0) or of all (-1),
 * 1..64; takes effect at the next window.  The Markov chain is unaffected:
 * the submatrix size only groups proposals (Sec. 2.3, submatrix updates). */
dcax_status dcax_set_submatrix_k(dcax_walker w, int32_t walker, int32_t ks);

/* Autotuner (App. A lists auto-tuning among the build options): runs
 * sweeps_per_trial generator-mode sweeps of the whole batch with each k_s in
 * {8, 16, 24, 32, 48, 64}, timed with HIP events, and keeps the k_s with the
 * most accepted updates per second; then, with that k_s, tries each kernel
 * form of the candidate-row product and then of the Y-column product (tiled,
 * wide, narrow; dcax_set_variants) and keeps the fastest of each.  The chosen
 * k_s is written to *chosen_ks and the best rate to *rate_out (both nullable);
 * dcax_get_variants reports the chosen forms.  The trial sweeps are ordinary
 * Markov-chain sweeps (they count as warm-up). */
dcax_status dcax_autotune(dcax_walker w, int32_t sweeps_per_trial, int32_t* chosen_ks, double* rate_out);

/* Replay generator-mode sweeps as hipGraphs (on != 0): one graph per
 * (order bound rounded up to 64, window count), captured on first use and
 * launched on a library-owned stream that is ordered after and before the
 * caller's stream with events.  The device-scheduled calls (dcax_sweep_measure,
 * dcax_run_rounds, dcax_sweep_measure_nfft) then replay each round - sweep
 * starts, windows, gated measurement - as one graph per (order bound,
 * windows, accumulators).  Off by default.  With timing on, a replayed
 * sweep is timed as a whole (window_seconds); the fold and accept kernel
 * times of dcax_stats come from eagerly launched windows only. */
dcax_status dcax_set_graphs(dcax_walker w, int32_t on);

/* Kernel forms of the two candidate products of a window (Sec. 2.3's
 * "large matrix-matrix multiplications" of the submatrix update): X_C = W_C N
 * (candidate rows) and N g_{I,c} (Y columns of inserted spins).
 *   DCAX_VARIANT_AUTO   chosen per launch from its size (default);
 *   DCAX_VARIANT_TILED  64-wide tiles of N staged in LDS, one workgroup per
 *                       tile over the whole inner dimension (fits launches
 *                       with many workgroups: batches of walkers);
 *   DCAX_VARIANT_WIDE   16-wide tiles, the inner dimension split over 16
 *                       (candidate rows) or 8 (Y columns) wavefronts (few
 *                       workgroups: a single walker);
 *   DCAX_VARIANT_NARROW 16-wide tiles over 4 wavefronts.
 * Every form computes the same products; they differ in summation order
 * only.  Answers DCAX_E_INVAL for an unknown value. */
typedef enum { DCAX_VARIANT_AUTO = 0, DCAX_VARIANT_TILED = 1, DCAX_VARIANT_WIDE = 2,
               DCAX_VARIANT_NARROW = 3 } dcax_variant;
dcax_status dcax_set_variants(dcax_walker w, int32_t cand_rows, int32_t y_columns);
/* The forms in use (DCAX_VARIANT_AUTO until set or autotuned); both nullable. */
dcax_status dcax_get_variants(dcax_walker w, int32_t* cand_rows, int32_t* y_columns);

/* Probe every walker's N against its definition without rebuilding it:
 * for 64 index pairs (p, q) per spin (a quarter of them diagonal), drawn
 * afresh at each probe, the normalised residual
 *   |sum_i A_pi N_iq - delta_pq| / sum_i |A_pi N_iq|,  A = N^{-1} = e^V - g (e^V - 1)
 * with A assembled from the propagator (O(k) work per pair).  A freshly
 * rebuilt N gives the unit roundoff of its precision; the residual grows
 * with the drift N accumulates between refreshes.  residual_out (host,
 * nullable, [n_walkers]): the largest residual per walker over both spins. */
dcax_status dcax_probe_N(dcax_walker w, double* residual_out);

/* Introspection and checkpointing; `walker` indexes the batch (0-based). */
dcax_status dcax_get_order(dcax_walker w, int32_t walker, int32_t* k);
/* Copy N_spin in canonical order (vertex id ascending) into host[ld * k];
 * ids_host (nullable) receives the k ids in that order.  FP32 walkers are
 * widened to double. */
dcax_status dcax_copy_N(dcax_walker w, int32_t walker, int32_t spin, double* host, int64_t ld, int64_t* ids_host);
dcax_status dcax_get_config(dcax_walker w, int32_t walker, dcax_vertex* host, int32_t cap, int32_t* k);
/* Install a configuration (ids must be distinct and >= 0) and rebuild N by
 * dcax_refresh; clears a latched error and the counters. */
dcax_status dcax_set_config(dcax_walker w, int32_t walker, const dcax_vertex* host, int32_t k);
/* walker = -1 sums the counters over the batch (sign: walker 0's). */
dcax_status dcax_get_stats(dcax_walker w, int32_t walker, dcax_stats* out);
/* Time the fold and accept kernels and whole windows with HIP events on the
 * walker's stream: on = n > 0 times every n-th window, on = 0 stops timing
 * (on < 0: DCAX_E_INVAL).  The events ride on the kernels' own dispatches;
 * a timed window still leaves the queue idle for a few microseconds per
 * event, so sampling keeps the overhead out of throughput measurements.
 * Timings accumulate into dcax_stats over the timed windows. */
dcax_status dcax_set_timing(dcax_walker w, int32_t on);
/* The G0(r, tau) table the walker uses for spin up (the only one unless two
 * tables were given), [Nc][n_tau], standard sign convention G0 = -<T c c+>. */
dcax_status dcax_copy_g0_table(dcax_walker w, int32_t walker, double* host);
/* Cluster geometry: sites [Nc][2] (int32) and momenta [Nc][2] (double). */
dcax_status dcax_cluster(const dcax_params* p, int32_t* n_sites, int32_t* sites, double* momenta);

/* ------------------------------------------------------------ DCA loop
 * The DCA self-consistency loop around the walkers (Sec. 2.1, the DCA loop
 * figure and its equations): the lattice self-energy is the cluster one,
 * constant on each of the Nc patches of the Brillouin zone (the patch of K
 * is the Brillouin zone of the superlattice centred on K); the coarse-
 * grained G averages the lattice G over each patch; the cluster-exclusion
 * step gives the bare propagator G0cal of the cluster problem, which the
 * walkers solve; Dyson's equation turns their G_c into a new self-energy,
 * mixed with the previous one.
 *
 * Layouts (device, FP64; complex as interleaved (re, im)):
 *   sigma, G:   [n_spin][Nc][n_freq] complex, the measured frequencies
 *               w_n = (2n+1) pi / beta, n = 0 .. n_freq-1;
 *   gbar, g0:   [n_spin][Nc][n_cg] complex (n_cg >= n_freq frequencies, for
 *               the transform to tau);
 *   g0_tau:     [n_spin][Nc][n_tau], G0cal(r_d, tau_l) in the layout and
 *               convention of dcax_params.g0_tau.
 * Spin blocks: n_spin = 1 carries one self-energy for both spins (G_c is
 * the average of the walkers' two spins); n_spin = 2 one per spin (up,
 * down), needed when h != 0.  Sites and momenta follow the cluster
 * enumeration above.
 *
 * Quadrature of the patch average: the L x L points ((i+1/2)/L - 1/2) b1 +
 * ((j+1/2)/L - 1/2) b2 of the reciprocal superlattice cell (a_i . b_j =
 * 2 pi delta_ij), each moved to its least-length image under b1, b2 (the
 * Wigner-Seitz cell); a point with several such images (within 1e-12 in
 * squared length) gives each an equal share of its weight.  Sigma above the
 * measured frequencies keeps its last real part and an imaginary part
 * falling as 1/w_n.  The transform to tau removes the tail 1/(i w) +
 * c2/(i w)^2 + c3/(i w)^3 and adds it back in closed form, with the exact
 * moments c2 = (patch mean of eps) - mu - sigma h and c3 = c2^2 + (patch
 * variance of eps). */
typedef struct dcax_dca_s* dcax_dca;

typedef struct {
  int32_t abi_version;     /* must be DCAX_ABI_VERSION */
  int32_t cluster[4];      /* superlattice vectors, as in dcax_params */
  double t, tp;            /* lattice dispersion eps_k = -2t (cos kx + cos ky) - 4 tp cos kx cos ky */
  double beta;
  double mu;               /* measured from U/2, as in dcax_params */
  double h;                /* Zeeman field: eps_k - mu - sigma h (needs n_spin = 2 when nonzero) */
  int32_t n_spin;          /* 1 or 2 self-energy blocks */
  int32_t n_freq;          /* measured frequencies (the walkers' n_freq), >= 1 */
  int32_t n_cg;            /* frequencies of the coarse-graining and the transform, n_freq .. 2^20 */
  int32_t n_tau;           /* points of the G0cal(r, tau) tables (the walkers' n_tau), >= 2 */
  int32_t patch_points;    /* L, 1 .. 256: L x L points per patch (1: the isolated cluster) */
  int32_t reserved;        /* must be 0 */
} dcax_dca_params;

/* What one dcax_dca_iterate call did. */
typedef struct {
  double max_change;       /* max over spin blocks, K, n of |Sigma_new - Sigma_old| */
  double sign;             /* mean sign of the measured configurations */
  double mean_order;       /* mean expansion order of the walkers at the end */
  int64_t measurements;    /* measured configurations, summed over the walkers */
} dcax_dca_report;

/* Create a DCA handle: builds the patch quadrature and eps(K + k~) on the
 * GPU.  Memory from the allocator (required), work on `stream`. */
dcax_status dcax_dca_create(const dcax_dca_params* p, const dcax_allocator* a, void* stream, dcax_dca* out);
dcax_status dcax_dca_destroy(dcax_dca d);

/* Coarse-graining and cluster exclusion (Sec. 2.1): from sigma_dev, writes
 * Gbar(K, i w_n) to gbar_dev (nullable) and G0cal = [Gbar^{-1} + Sigma]^{-1}
 * to g0_dev, for n < n_cg. */
dcax_status dcax_dca_coarse_grain(dcax_dca d, const double* sigma_dev, double* gbar_dev, double* g0_dev);

/* The walkers' tables G0cal(r_d, tau_l) = (1/Nc) sum_K e^{i K r_d}
 * G0cal(K, tau_l) from g0_dev (n_cg frequencies), into g0_tau_dev. */
dcax_status dcax_dca_g0_tables(dcax_dca d, const double* g0_dev, double* g0_tau_dev);

/* The cluster G (Sec. 2.3's estimator with G0cal): G_sigma = G0cal -
 * G0cal <M_sigma> G0cal / beta with <M> = sum of n_blocks accumulator blocks
 * over the sum of their signs; acc_dev and aux_dev in dcax_measure_G's
 * layout for n_blocks walkers of this cluster and n_freq; G_dev [n_spin][Nc]
 * [n_freq] (the spin average when n_spin = 1). */
dcax_status dcax_dca_cluster_G(dcax_dca d, const double* g0_dev, const double* acc_dev, const double* aux_dev,
                               int32_t n_blocks, double* G_dev);

/* Dyson's equation and mixing: sigma_new = alpha (G0cal^{-1} - G^{-1}) +
 * (1 - alpha) sigma_old on the measured frequencies, 0 < alpha <= 1
 * (sigma_new may be sigma_old).  max_change_out (host, nullable): the
 * largest |sigma_new - sigma_old|. */
dcax_status dcax_dca_self_energy(dcax_dca d, const double* g0_dev, const double* G_dev, const double* sigma_old_dev,
                                 double alpha, double* sigma_new_dev, double* max_change_out);

/* One iteration of the loop with the walkers as the cluster solver:
 * coarse-grain and exclude from sigma_dev, install G0cal in every walker
 * (dcax_set_g0), warmup_sweeps sweeps, measure_sweeps sweeps with one
 * measurement each (dcax_sweep_measure), the cluster G of all walkers, and
 * sigma_dev <- the mixed new self-energy.  The walkers must all have this
 * handle's cluster, beta, n_tau and n_freq and n_spin_tables = n_spin, and
 * have been created with g0_tau and g0_Kw.  G_dev (nullable) receives G_c;
 * report (host, nullable). */
dcax_status dcax_dca_iterate(dcax_dca d, dcax_walker w, int32_t warmup_sweeps, int32_t measure_sweeps, double alpha,
                             double* sigma_dev, double* G_dev, dcax_dca_report* report);

/* Replace the bare propagator of every walker of a handle (Sec. 2.1: the
 * solver's input changes at each DCA iteration) and rebuild N from scratch
 * for the current configurations, with their signs.
 *   g0_tau_dev: [n_spin_tables][Nc][n_tau] (device), as dcax_params.g0_tau;
 *   g0_Kw_dev:  complex [n_spin_tables][Nc][g0_Kw_stride] (device; the first
 *               n_freq entries of each row are taken), g0_Kw_stride >= n_freq.
 * The walkers must share Nc, n_tau and n_freq, and have been created with
 * g0_tau and g0_Kw of n_spin_tables tables. */
dcax_status dcax_set_g0(dcax_walker w, const double* g0_tau_dev, int32_t n_spin_tables, const double* g0_Kw_dev,
                        int32_t g0_Kw_stride);

/* Thread-local message for the last non-OK status. */
const char* dcax_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DCAX_H */

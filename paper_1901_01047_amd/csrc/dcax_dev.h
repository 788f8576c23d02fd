// Internal device-side definitions of the CT-AUX walker library (gfx950).
//
// One walker owns, in HBM: its vertex arrays (structure of arrays), the two
// walker matrices N_up and N_down (column-major, leading dimension `ld`,
// capacity `cap` = max_order + submatrix_k so that a window's inserted rows
// fit before compaction), the G0(r, tau) table, and the window scratch
// buffers below.  Mutable scalars (order, sign, cursors, counters, the
// latched status) live in a device-resident control block so that a whole
// sweep can be enqueued without host round trips.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "dcax.h"

namespace dcax {

constexpr int KS_MAX = 64;   // largest submatrix size (window proposals)
constexpr int WG = 256;      // threads per workgroup of the streaming kernels

enum StatusCode { ST_OK = 0, ST_NUMERIC = 1, ST_CAPACITY = 2, ST_TRACE = 3 };

constexpr int FOLD_RANK_BINS = 17;  // m = 0 and sixteen bins of four up to m = 64

struct Ctl {
  int k;            // current expansion order
  int status;       // latched StatusCode
  int active;       // the current window has work
  int nP;           // proposals in the window
  int nE;           // window elements (candidates + removal targets)
  int nC;           // insertion candidates
  int m;            // |S| after the accept loop (fold rank)
  int mi;           // inserted spins in S
  int mr;           // removed spins in S
  int k0;           // order at the window start
  int kx;           // extended order k0 + mi
  int knew;         // order after compaction
  long long next_id;
  long long pos;    // replay cursor or global proposal counter
  long long end;    // end of the replay batch or of the sweep
  double sign;
  long long n_prop, n_acc_ins, n_acc_rem, n_windows, sum_m, n_mismatch, n_sweeps;
  double fold_flops;
  long long carry_id;  // removal target carried into the next window, -1 none
  long long n_abort;   // windows closed early by a carried removal
  double fold_bytes;   // algorithmic bytes of the folds (N read and written)
  long long n_folds;   // windows with a non-empty fold
  double drift;        // drift measured by the last refresh
  long long sweep_len; // frozen proposals per sweep before rounding to k_s, 0 while warming up
  double warm_sum;     // sum of the order at sweep starts over the warm-up's second half
  long long warm_n;    // number of such sweeps
  // sweeps scheduled on the device (dcax_sweep_measure): sweeps still to
  // begin, and whether the finished sweep still awaits its measurement
  long long sweeps_left;
  int meas_due;
  // order the refresh kernels rebuild (k, set by the refresh's first kernel)
  int k_ref;
  // windows by fold rank: bin 0 is m = 0, bin b holds 4b - 3 <= m <= 4b
  long long m_hist[FOLD_RANK_BINS];
  // algorithmic work of the candidate-row (X_C = W_C N) and Y-column
  // (N g_{I,c}) products: flops, and bytes with N read once
  double cand_flops, cand_bytes, y_flops, y_bytes;
  long long n_acc_flip;  // accepted spin flips
  long long n_neglect;   // proposals rejected as touching a spin twice
  int carry_kind;        // kind (1 removal, 2 flip) of the carried proposal's target
  // the drift probe at the end of this walker's sweep found N beyond the
  // tolerance: its measurement and next sweep wait for the rebuild
  int hold;
};

struct WinProp {      // one proposal of the current window
  int kind;           // 0 insertion, 1 removal, 2 spin flip
  int el;             // window element, -1 for a no-op removal at k = 0
  int forced;         // replay decision (-1: decide from u)
  int carried;        // removal whose target was fixed before this window
  double u;           // acceptance uniform
  double ub0, ui0;    // a removal's first target attempt (generator mode)
  long long ridx;     // replay index (ratio output), -1 if none
  long long gidx;     // global proposal index (generator counter)
};

// Everything a kernel needs about one walker.  A launch covers a batch of
// walkers: kernels receive a device array of views and pick theirs by
// blockIdx.z (or blockIdx.z / 2 where z also carries the spin).  T is the
// storage type of N and of its GEMM operands (double, or float in the mixed
// mode).
template <typename T>
struct View {
  // model
  int Nc, n_tau, ks, cap, ld, max_order, warmup;
  double beta, h, gamma, K_exp;
  double ev[2][2];            // e^{V}: [spin][0 for s = +1, 1 for s = -1]
  double flip_share;          // share of spin-flip proposals
  int neglect;                // touched twice: 0 close the window, 1 reject
  uint64_t seed;              // generator key
  const int* diff;            // [Nc * Nc] index of r_i - r_j
  const double* table[2];     // [Nc][n_tau] G0_sigma(r, tau_l), standard convention (one shared table or one per spin)
  int spin_tables;            // 1: table[1] == table[0]; 2: a table per spin
  const double* g0Kw;         // [spin_tables][Nc][n_freq][2] caller's G0(K, i w_n), or null
  int ext_g0;                 // the tables came from the caller (G0(K, .) from them in the finalisation)
  const int* sites;           // [Nc][2]
  const double* Kp;           // [Nc][2]
  const double* xi;           // [Nc] eps_K - mu
  // state
  Ctl* ctl;
  int* v_site;
  double* v_tau;
  int* v_s;
  long long* v_id;
  T* N[2];
  // window scratch
  WinProp* wp;
  int* el_site;
  double* el_tau;
  int* el_s;
  int* el_slot;               // slot of a removal or flip target, -1 for a candidate
  int* el_flip;               // 1 for a flip target (its column of Gt and of A differ from a removal's)
  int* el_cand;               // candidate index or -1
  int* el_row;                // row of each element in the extended N
  int* cand_el;
  long long* cand_id;
  int* S;                     // element of each fold column, S order
  int* ins_el;                // inserted elements in S order (mi)
  int* remap;                 // [cap] compaction source of each destination
  int* moves;                 // [2 KS_MAX + 1] compaction (dst, src) pairs, count
  T* gcol[2];                 // [ks][cap] g_{I,c} per spin (gcol[1] == gcol[0] for one table)
  T* W[2];                    // [ks][cap] g_{c,I} (e^{V_I} - 1)
  double* gCC[2];             // [ks][ks] g_{c,c'} per spin (shared like gcol)
  T* R[2];                    // [KS_MAX][cap] rows of the extended N per element
  double* gram[2];            // [ks][ks] G restricted to the window elements
  double* ginv[2];            // [ks][ks] Gamma_S^{-1}
  T* Y[2];                    // [ks][cap] N g_{I,c} for inserted spins
  T* A[2];                    // [ks][cap] fold left factor, column-major
  T* B[2];                    // [ks][cap] fold right factor, row-major
  double* ratio_out;          // device copy of the replay ratios
  const dcax_proposal* replay;
  // refresh scratch (FP64)
  double* M[2];               // [cap][cap]
  double* P[2];               // [cap][NB] panel columns
  double* Tm[2];              // [NB][cap] panel rows
  int* ipiv[2];               // [cap]
  int* perm[2];               // [cap]
  double* gjc[2];             // column-step pivot records (gjc_len(cap))
  double* blkmax;             // per-block maxima of the drift
  double* detsign;            // [2]
  // measurement scratch
  int n_freq;
  int kpad_cap;
  int* m_order;               // [kpad_cap]
  int* m_off;                 // [Nc + 1]
  T* m_Ms[2];                 // [kpad_cap][kpad_cap]
  T* m_E;                     // [kpad_cap][n_freq][2]
  double* m_Mab[2];           // [Nc][Nc][n_freq][2]
  long long acc_off;          // offset (doubles) of this walker's accumulator block
  int nc_prefix;              // sum of Nc over the preceding walkers
  int wid;
};

// ---------------------------------------------------------------- helpers
__device__ inline void latch(Ctl* c, int code) { atomicCAS(&c->status, 0, code); }

// A gated measurement covers the walkers whose sweep has ended and not yet
// been measured (device-scheduled sweeps), unless held for a rebuild; an
// ungated one covers all.
__device__ inline bool meas_skip(const Ctl* c, int gated) {
  return gated && !(c->status == 0 && c->meas_due && c->pos >= c->end && !c->hold);
}

__device__ inline int s01(int s) { return s > 0 ? 0 : 1; }

// Maximum that propagates NaN from either operand (fmax drops a NaN operand,
// so a reduction built on it would report a NaN matrix as drift 0).
__host__ __device__ inline double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

// Linear interpolation of the table at dtau in [0, beta]: l = floor(dtau/h),
// f = dtau/h - l, (1 - f) T[l] + f T[l+1], l clamped to n_tau - 2; dtau = 0
// gives the 0+ value.
template <typename T>
__device__ inline double g0_interp(const View<T>& w, int sp, int d, double dtau) {
  double x = dtau / w.h;
  int l = (int)floor(x);
  l = l < 0 ? 0 : (l > w.n_tau - 2 ? w.n_tau - 2 : l);
  double f = x - (double)l;
  const double* t = w.table[sp] + (size_t)d * w.n_tau;
  return (1.0 - f) * t[l] + f * t[l + 1];
}

// g(i, j) = <T c_i(tau_i) c+_j(tau_j)>_0 = -G0(r_i - r_j, tau_i - tau_j) for
// tau_i >= tau_j (0+ at equal times), and +G0(r_i - r_j, tau_i - tau_j + beta)
// for tau_i < tau_j (antiperiodicity).
template <typename T>
__device__ inline double gfun(const View<T>& w, int sp, int ri, double ti, int rj, double tj) {
  int d = w.diff[ri * w.Nc + rj];
  double dt = ti - tj;
  if (dt < 0.0) return g0_interp(w, sp, d, dt + w.beta);
  return -g0_interp(w, sp, d, dt);
}

// ------------------------------------------------------------------ MFMA
// 16x16x4 matrix-core instructions.  Operand layout (both precisions): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16].  Result register i of lane l
// holds D[row(l, i)][l % 16] with row = 4 i + l / 16 in FP64 and
// 4 (l / 16) + i in FP32.
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4_t acc_t;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef f4_t acc_t;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// ------------------------------------------------------------ generator
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): a keyed bijection of a 128-bit counter.  The
// counter is (proposal index, draw slot), the key the walker's seed, so every
// proposal's uniforms are a pure function of its index.
__host__ __device__ inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__host__ __device__ inline void philox4x32(uint32_t c[4], uint64_t seed) {
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
}

// Two uniforms in [0, 1) with 53 random bits each, for draw slot `slot` of
// proposal `g`.
__host__ __device__ inline void uniforms2(uint64_t seed, long long g, uint32_t slot, double& u, double& v) {
  uint32_t c[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), slot, 0x43545841u};
  philox4x32(c, seed);
  u = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * (1.0 / 9007199254740992.0);
  v = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * (1.0 / 9007199254740992.0);
}

// Global-memory view of a pointer held in a View.  Pointers loaded from a
// struct in memory are generic (flat) to the compiler; flat accesses count
// against the LDS wait counter too, so a flat store inside an LDS-bound loop
// stalls every later LDS read until the store has reached memory.
template <typename P>
__device__ inline __attribute__((address_space(1))) P* gp(P* p) {
  return (__attribute__((address_space(1))) P*)p;
}

// Values every lane of the wavefront holds, moved to scalar registers so
// that loops and branches on them stay uniform (the compiler cannot prove
// uniformity of values read from LDS or memory).
__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline long long uni(long long x) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline double uni(double x) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

// The value a uniform-indexed lane holds (v_readlane, no LDS round trip).
__device__ inline int lane_value(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ inline double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
__device__ inline long long lane_value(long long v, int src) {
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace dcax

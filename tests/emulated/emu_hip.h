// Host emulation of the HIP constructs the accept kernel uses: one std::thread
// per work-item, wavefront collectives (readlane, ballot, shuffles) as
// 64-party exchanges, __syncthreads as a 256-party barrier.  Every rendezvous
// checks that all parties arrived from the same source line (a lane that
// skips a collective is reported, not silently mixed) and times out with a
// deadlock report.  Test infrastructure only.
#pragma once
#include <cstdint>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <condition_variable>
#include <thread>
#include <vector>
#include <chrono>
#include <algorithm>
#include <atomic>
#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __launch_bounds__(x)
struct emu_dim3 { unsigned x = 0, y = 0, z = 0; };
extern thread_local emu_dim3 threadIdx, blockIdx;

struct EmuRendezvous {
  int parties;
  std::mutex mu;
  std::condition_variable cv;
  int arrived = 0;
  long gen = 0;
  uint64_t buf[2][256];
  int site[2][256];
  explicit EmuRendezvous(int p) : parties(p) {}
  // deposit v, wait for all, return a copy of all values
  void exchange(int me, uint64_t v, int st, uint64_t* out) {
    std::unique_lock<std::mutex> lk(mu);
    const int b = gen & 1;
    buf[b][me] = v;
    site[b][me] = st;
    if (++arrived == parties) {
      for (int i = 0; i < parties; ++i)
        if (site[b][i] != st) {
          fprintf(stderr, "EMU: divergent rendezvous: party %d at line %d, party %d at line %d\n", me, st, i,
                  site[b][i]);
          abort();
        }
      arrived = 0;
      ++gen;
      cv.notify_all();
    } else {
      const long g = gen;
      if (!cv.wait_for(lk, std::chrono::seconds(20), [&] { return gen != g; })) {
        fprintf(stderr, "EMU: deadlock at line %d (party %d; %d of %d arrived)\n", st, me, arrived, parties);
        abort();
      }
    }
    if (out) std::memcpy(out, buf[b], sizeof(uint64_t) * parties);
  }
};
extern EmuRendezvous* emu_wave[4];
extern EmuRendezvous* emu_block;

inline int emu_lane() { return threadIdx.x & 63; }
inline int emu_wv() { return threadIdx.x >> 6; }
inline uint64_t emu_coll(uint64_t v, int st, uint64_t* all) {
  emu_wave[emu_wv()]->exchange(emu_lane(), v, st, all);
  return 0;
}
inline void emu_syncthreads(int st) { emu_block->exchange(threadIdx.x, 0, st, nullptr); }
inline void emu_wave_sync(int st) { emu_coll(0, st, nullptr); }
#define __syncthreads() emu_syncthreads(__LINE__)
#define EMU_WAVE_SYNC() emu_wave_sync(__LINE__)

inline int emu_readlane(int v, int src, int st) {
  uint64_t all[64];
  emu_coll((uint64_t)(uint32_t)v, st, all);
  if (src < 0 || src > 63) { fprintf(stderr, "EMU: readlane index %d at line %d\n", src, st); abort(); }
  return (int)(uint32_t)all[src];
}
#define __builtin_amdgcn_readlane(v, s) emu_readlane((v), (s), __LINE__)
#define __builtin_amdgcn_readfirstlane(v) emu_readlane((v), 0, __LINE__)
inline unsigned long long emu_ballot(int p, int st) {
  uint64_t all[64];
  emu_coll((uint64_t)(p != 0), st, all);
  unsigned long long m = 0;
  for (int i = 0; i < 64; ++i) if (all[i]) m |= 1ull << i;
  return m;
}
#define __ballot(p) emu_ballot((p), __LINE__)
inline int emu_shfl(int v, int src, int st) {
  uint64_t all[64];
  emu_coll((uint64_t)(uint32_t)v, st, all);
  return (int)(uint32_t)all[src & 63];
}
#define __shfl(v, s, w) emu_shfl((v), (s), __LINE__)
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __double2loint(double d) { uint64_t u; std::memcpy(&u, &d, 8); return (int)(uint32_t)u; }
inline int __double2hiint(double d) { uint64_t u; std::memcpy(&u, &d, 8); return (int)(uint32_t)(u >> 32); }
inline double __hiloint2double(int hi, int lo) {
  uint64_t u = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  double d; std::memcpy(&d, &u, 8); return d;
}
extern std::mutex emu_atomic_mu;
inline int atomicCAS(int* p, int cmp, int val) {
  std::lock_guard<std::mutex> g(emu_atomic_mu);
  int old = *p; if (old == cmp) *p = val; return old;
}
using std::min;
using std::max;
inline double emu_shfl_xor_d(double v, int mask, int st) {
  uint64_t all[64], u; std::memcpy(&u, &v, 8);
  emu_coll(u, st, all);
  uint64_t r = all[(emu_lane() ^ mask) & 63]; double d; std::memcpy(&d, &r, 8); return d;
}
#define __shfl_xor(v, m, w) emu_shfl_xor_d((v), (m), __LINE__)
using std::isfinite;
using std::fabs;
using std::fma;
using std::floor;

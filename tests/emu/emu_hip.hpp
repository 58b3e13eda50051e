// CPU stand-in for the few HIP device features the sweep kernels use, so that
// the kernel sources (paper_2605_17230_amd/csrc) can run one work-group at a
// time on the host for tests: a work-group is NT std::threads, __syncthreads a
// std::barrier, cross-lane moves go through a shared buffer between barriers
// of the lanes involved.  Test infrastructure only.
#pragma once
#define TNMLD_EMU 1
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <thread>

#define __device__
#define __host__
#define __global__
#define __shared__ static
#define __launch_bounds__(x)
#define __align__(x) alignas(x)

struct EmuDim {
  unsigned x = 0, y = 0, z = 0;
};
inline thread_local EmuDim threadIdx;
inline EmuDim blockIdx, blockDim{512, 1, 1};
inline std::barrier<>* g_block_bar = nullptr;   // all threads of the work-group
inline std::barrier<>* g_wave_bar[16] = {};     // the 64 lanes of each wave
inline std::barrier<>* g_row_bar[64] = {};      // each row of 16 lanes
template <class T>
inline T g_xchg[1024];

inline void __syncthreads() { g_block_bar->arrive_and_wait(); }

// __syncthreads_or / __syncthreads_and: a barrier that also combines one int
// per thread
inline std::atomic<int> g_sync_acc{0};
template <class Op>
int emu_sync_combine(int v, int init, Op op) {
  g_block_bar->arrive_and_wait();
  if (threadIdx.x == 0) g_sync_acc.store(init);
  g_block_bar->arrive_and_wait();
  int cur = g_sync_acc.load();
  while (!g_sync_acc.compare_exchange_weak(cur, op(cur, v))) {
  }
  g_block_bar->arrive_and_wait();
  const int r = g_sync_acc.load();
  g_block_bar->arrive_and_wait();
  return r;
}
inline int __syncthreads_or(int v) { return emu_sync_combine(v ? 1 : 0, 0, [](int a, int b) { return a | b; }); }
inline int __syncthreads_and(int v) { return emu_sync_combine(v ? 1 : 0, 1, [](int a, int b) { return a & b; }); }
inline unsigned atomicOr(unsigned* p, unsigned v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}

// lane t reads the value of lane t ^ off; all lanes of the wave take part
template <class T>
T __shfl_xor(T v, int off, int) {
  const int t = threadIdx.x, w = t / 64;
  g_xchg<T>[t] = v;
  g_wave_bar[w]->arrive_and_wait();
  const T r = g_xchg<T>[(t & ~63) | ((t & 63) ^ off)];
  g_wave_bar[w]->arrive_and_wait();
  return r;
}

// xor exchange inside aligned groups of G lanes; groups of <= 16 lanes only
// synchronise their own row, so they may diverge from each other
template <class T>
T emu_shfl_xor(T v, int off, int G) {
  if (G > 16) return __shfl_xor(v, off, 64);
  const int t = threadIdx.x, row = t / 16;
  g_xchg<T>[t] = v;
  g_row_bar[row]->arrive_and_wait();
  const T r = g_xchg<T>[t ^ off];
  g_row_bar[row]->arrive_and_wait();
  return r;
}

using std::exp;
using std::fabs;
using std::log;
using std::sqrt;

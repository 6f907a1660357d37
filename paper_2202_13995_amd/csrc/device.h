// Device-side helpers shared by the panel kernels: coherent cross-workgroup
// loads/stores, the bounded grid barrier, the pivot-candidate order and the
// 16x16 MFMA traits used by the triangular solves and the in-panel updates.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace lp {

// --------------------------------------------------------- grid barrier
// All workgroups of a launch meet here.  Every workgroup is resident at once
// (the launcher keeps the grid at most one workgroup per compute unit, and no
// other kernel depends on this one), so the wait ends; it is still bounded by
// the device's constant 100 MHz clock so that a stuck launch drains instead of
// hanging.  Returns false on timeout.
//
// Cross-workgroup data goes through relaxed agent-scope atomic loads and
// stores, which the compiler emits as L2-coherent (sc1) accesses; each thread
// waits for its own stores to be acknowledged before the workgroup arrives.
// This avoids release/acquire fences, which on this chip write back and
// invalidate the whole L2 of the compute die and would stall the concurrent
// trailing update.
constexpr unsigned long long kBarrierTimeoutTicks = 2000000000ull;  // 20 s at 100 MHz

template <typename V>
__device__ __forceinline__ void xstore(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ V xload(const V* p) {
  return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline bool grid_barrier(unsigned* ctr, unsigned target, int* s_flag) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have landed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int ok = 1;
    while (xload(ctr) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeoutTicks) {
        ok = 0;
        break;
      }
    }
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}


__device__ __forceinline__ bool better(double ka, int ia, double kb, int ib) {
  // is (ka, ia) a better pivot candidate than (kb, ib)?
  return ka > kb || (ka == kb && ia < ib);
}

// The best (key, index) pair of a wave, in every lane: four DPP exchanges
// inside each row of 16 lanes (quad swaps, then half-row and row mirrors,
// each pairing a lane with one from the other half), then the four rows'
// winners read across lanes.  `first(a, ia, b, ib)` must be a strict order
// (as `better` is), so the result does not depend on the reduction's shape.
// Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_move(unsigned v) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL, typename F>
__device__ __forceinline__ void wave_best_step(unsigned long long& key, int& idx, F& first) {
  const unsigned lo = dpp_move<CTRL>((unsigned)key);
  const unsigned hi = dpp_move<CTRL>((unsigned)(key >> 32));
  const int oi = (int)dpp_move<CTRL>((unsigned)idx);
  const unsigned long long ok = ((unsigned long long)hi << 32) | lo;
  if (first(ok, oi, key, idx)) {
    key = ok;
    idx = oi;
  }
}
template <typename F>
__device__ __forceinline__ void wave_best(unsigned long long& key, int& idx, F first) {
  wave_best_step<0xB1>(key, idx, first);   // quad_perm [1, 0, 3, 2]
  wave_best_step<0x4E>(key, idx, first);   // quad_perm [2, 3, 0, 1]
  wave_best_step<0x141>(key, idx, first);  // row_half_mirror
  wave_best_step<0x140>(key, idx, first);  // row_mirror
  unsigned long long bk = 0;
  int bi = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)key, 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(key >> 32), 16 * r);
    const int ri = __builtin_amdgcn_readlane(idx, 16 * r);
    const unsigned long long rk = ((unsigned long long)hi << 32) | lo;
    if (r == 0 || first(rk, ri, bk, bi)) {
      bk = rk;
      bi = ri;
    }
  }
  key = bk;
  idx = bi;
}

template <typename T>
struct Mfma16;

template <>
struct Mfma16<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int g, int v) { return g + 4 * v; }
  static __device__ __forceinline__ int kidx(int g, int t) { return g + 4 * t; }
};

template <>
struct Mfma16<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int g, int v) { return 4 * g + v; }
  static __device__ __forceinline__ int kidx(int g, int t) { return 4 * g + t; }
};

// Cross-workgroup pivot-candidate slots (double-buffered by barrier parity):
// per workgroup a key, a row index and the candidate row, plus the diagonal row
// and its NaN flag.
// Exchange records of one column parity: G candidate records, then the
// diagonal record.  A record is kRecWords 64-bit words; word w < 2 * kLeafMax
// holds 32 bits of the row (a double takes two words, low half first, a float
// one), word 2 * kLeafMax the row index (candidate) or the NaN flag (diagonal).
// Every word carries the writer's column tag in its upper 32 bits, so a reader
// validates each word on its own: no word needs to be acknowledged before the
// column's key is published.  Tags are unique within one factorization (the
// records are zeroed when it starts).
constexpr int kRecWords = 2 * kLeafMax + 2;

struct LeafLayout {
  size_t rec_off, drec_off, buf_bytes;
};

__host__ __device__ inline LeafLayout leaf_layout(int G) {
  LeafLayout L;
  L.rec_off = 0;
  L.drec_off = sizeof(unsigned long long) * kRecWords * (size_t)G;
  L.buf_bytes = (L.drec_off + sizeof(unsigned long long) * kRecWords + 255) & ~(size_t)255;
  return L;
}

__device__ __forceinline__ unsigned long long tagged(unsigned tag, unsigned payload) {
  return ((unsigned long long)tag << 32) | payload;
}

}  // namespace lp

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
struct LeafLayout {
  size_t key_off, idx_off, rows_off, diag_off, flag_off, buf_bytes;
};

template <typename T>
__host__ __device__ inline LeafLayout leaf_layout(int G) {
  LeafLayout L;
  size_t off = 0;
  L.key_off = off;
  off += sizeof(double) * (size_t)G;
  L.idx_off = off;
  off += sizeof(int) * (size_t)G;
  off = (off + 15) & ~(size_t)15;
  L.rows_off = off;
  off += sizeof(T) * (size_t)G * kLeafMax;
  L.diag_off = off;
  off += sizeof(T) * kLeafMax;
  L.flag_off = off;
  off += 16;
  off = (off + 255) & ~(size_t)255;
  L.buf_bytes = off;
  return L;
}

}  // namespace lp

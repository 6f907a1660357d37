// Parallel construction of the net permutation of a run of row interchanges
// (shared by the factorization's row exchanges and the solve's B := P B).
#pragma once

#include <hip/hip_runtime.h>

namespace lp {

// Builds the plan for the k = k2 - k1 <= kPlanMax swaps in `piv` (LDS or
// registers of this workgroup, blockDim.x >= k).  Results go to dst/src
// (either LDS or global) and the count to *nent.  Needs scratch LDS arrays of
// kPlanMax ints: nxt, Bv, scan (2 kPlanMax).
__device__ inline void build_swap_plan(const int* piv, int k1, int k2, int* nxt, int* Bv, int* Fv,
                                int* flag, int* dst, int* src, int* nent) {
  const int k = k2 - k1;
  const int t = threadIdx.x;
  int pt = 0, pred = -1, h = -1, last = 1;
  if (t < k) {
    pt = piv[t];
    const int me = k1 + t;
    for (int j = 0; j < t; ++j) {
      const int pj = piv[j];
      if (pj == me) h = j;
      if (pj == pt) pred = j;
    }
    for (int j = t + 1; j < k; ++j)
      if (piv[j] == pt) last = 0;
    nxt[t] = (h >= 0) ? h : t;
  }
  __syncthreads();
  // pointer jumping to the root of each backward chain
  for (int len = 1; len < k; len <<= 1) {
    int v = 0;
    if (t < k) v = nxt[nxt[t]];
    __syncthreads();
    if (t < k) nxt[t] = v;
    __syncthreads();
  }
  if (t < k) Bv[t] = k1 + nxt[t];
  __syncthreads();
  int f_top = 0, f_out = 0, s_top = 0, s_out = 0, d_out = 0;
  if (t < k) {
    const int me = k1 + t;
    if (pt == me)
      s_top = Bv[t];
    else
      s_top = (pred >= 0) ? Bv[pred] : pt;
    f_top = (s_top != me) ? 1 : 0;
    if (pt >= k2 && last) {
      f_out = 1;
      d_out = pt;
      s_out = Bv[t];
    }
  }
  // exclusive scan of the 2k flags (top entries first, then outside ones)
  if (t < k) {
    flag[t] = f_top;
    flag[k + t] = f_out;
  }
  __syncthreads();
  for (int off = 1; off < 2 * k; off <<= 1) {
    int a0 = 0, a1 = 0;
    if (t < k) {
      a0 = (t >= off) ? flag[t - off] : 0;
      a1 = (k + t >= off) ? flag[k + t - off] : 0;
    }
    __syncthreads();
    if (t < k) {
      flag[t] += a0;
      flag[k + t] += a1;
    }
    __syncthreads();
  }
  if (t < k) {
    if (f_top) {
      const int pos = flag[t] - 1;
      dst[pos] = k1 + t;
      src[pos] = s_top;
    }
    if (f_out) {
      const int pos = flag[k + t] - 1;
      dst[pos] = d_out;
      src[pos] = s_out;
    }
    if (t == k - 1) *nent = flag[2 * k - 1];
  }
  (void)Fv;
}

}  // namespace lp

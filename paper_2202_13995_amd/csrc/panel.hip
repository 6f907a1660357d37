// Panel-side kernels of the blocked LU: the pivoted panel leaf, the row
// interchanges, and the unit-lower triangular solve.
//
// Paper, section "High Performance Linpack", "Base Implementation": each
// iteration factors the diagonal block into L and U, updates the blocks to its
// right with L (the "top" blocks, a triangular solve here) and the blocks
// below it with U (the "left" blocks).  With partial pivoting the left blocks
// are factored together with the diagonal block as one tall column panel,
// and every chosen pivot row is exchanged with the diagonal row across the
// whole matrix.
#include <climits>

#include "common.h"
#include "device.h"
#include "swap_plan.h"

namespace lp {

// ------------------------------------------------------------------ helpers

__global__ void zero_words_kernel(uint32_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

int launch_zero_words(void* p, size_t nwords, hipStream_t s) {
  if (nwords == 0) return LP_OK;
  size_t blocks = (nwords + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p,
                     nwords);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

template <typename S, typename D>
__global__ void convert_kernel(int rows, int cols, const S* __restrict__ src, long long lds,
                               D* __restrict__ dst, long long ldd) {
  const long long total = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / cols;
    const long long c = e - r * cols;
    dst[r * ldd + c] = (D)src[r * lds + c];
  }
}

int launch_convert(int to_f32, int rows, int cols, const void* src, long long lds, void* dst,
                   long long ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return LP_OK;
  long long blocks = ((long long)rows * cols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (to_f32)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3((unsigned)blocks), dim3(256), 0, s,
                       rows, cols, (const double*)src, lds, (float*)dst, ldd);
  else
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3((unsigned)blocks), dim3(256), 0, s,
                       rows, cols, (const float*)src, lds, (double*)dst, ldd);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

// ----------------------------------------------------- candidate slots
size_t leaf_slots_bytes(int m, int w) {
  (void)m;
  (void)w;
  // G <= 1024 workgroups, two column parities
  return 2 * leaf_layout(1024).buf_bytes;
}

// ------------------------------------------------------- row interchanges
// The interchanges of steps k1..k2-1 (row j <-> row ipiv[j] >= j, in order)
// form one permutation of at most 2 (k2 - k1) rows.  Writing T for the rows
// k1..k2-1 and B[t] for the original row whose contents sit in row k1 + t just
// before step t:
//   B[t] = B[h] if h, the last earlier step whose pivot row was k1 + t, exists,
//          else k1 + t;
//   the final contents of row k1 + t come from B[pred] (pred = last earlier
//   step with the same pivot row) or from the pivot row itself if it was never
//   a pivot before (or B[t] when the step keeps its own row);
//   a row outside T ends with B[t] of the last step that chose it.
// B follows chains that only point backwards, resolved by pointer jumping, so
// the whole plan is built in parallel with O(k) work per thread; the
// exchange itself is then a gather: every (dst, src) pair reads before any
// write.  Contents of the plan: nent, then dst[], src[] (compacted).
constexpr int kPlanMax = 1024;                 // swaps per plan
constexpr int kPlanDst = 4;                    // int offsets inside a plan
constexpr int kPlanSrc = 4 + 2 * kPlanMax;
constexpr int kPlanInts = 4 + 4 * kPlanMax;

size_t swap_plan_bytes(int nswaps) {
  (void)nswaps;
  return sizeof(int) * (size_t)kPlanInts;
}

__global__ __launch_bounds__(1024) void swap_plan_kernel(const int32_t* __restrict__ ipiv,
                                                         int k1, int k2, int* __restrict__ plan) {
  __shared__ int piv[kPlanMax];
  __shared__ int nxt[kPlanMax];
  __shared__ int Bv[kPlanMax];
  __shared__ int flag[2 * kPlanMax];
  const int k = k2 - k1;
  if ((int)threadIdx.x < k) piv[threadIdx.x] = ipiv[k1 + threadIdx.x];
  __syncthreads();
  build_swap_plan(piv, k1, k2, nxt, Bv, nullptr, flag, plan + kPlanDst, plan + kPlanSrc, plan);
}

int launch_swap_plan(const int32_t* ipiv, int k1, int k2, void* plan, hipStream_t s) {
  const int k = k2 - k1;
  if (k <= 0) return launch_zero_words(plan, 1, s);
  if (k > kPlanMax) return LP_ENOTSUP;
  hipLaunchKernelGGL(swap_plan_kernel, dim3(1), dim3(1024), 0, s, ipiv, k1, k2, (int*)plan);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

template <typename T, int Q>
__global__ __launch_bounds__(1024) void swap_apply_kernel(T* __restrict__ A, long long lda,
                                                          int c0, int c1, int c2, int c3, int CW,
                                                          const int* __restrict__ plan) {
  const int nent = plan[0];
  const int* dst = plan + kPlanDst;
  const int* src = plan + kPlanSrc;
  const int chunks1 = (c1 - c0 + CW - 1) / CW;
  int cs, ce;
  if ((int)blockIdx.x < chunks1) {
    cs = c0 + blockIdx.x * CW;
    ce = min(c1, cs + CW);
  } else {
    cs = c2 + (blockIdx.x - chunks1) * CW;
    ce = min(c3, cs + CW);
  }
  const int width = ce - cs;
  T v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + 1024 * q;
    const int ent = e / CW;
    const int col = e - ent * CW;
    if (ent < nent && col < width) v[q] = A[(long long)src[ent] * lda + cs + col];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + 1024 * q;
    const int ent = e / CW;
    const int col = e - ent * CW;
    if (ent < nent && col < width) A[(long long)dst[ent] * lda + cs + col] = v[q];
  }
}

template <typename T>
int launch_swap_apply(T* A, long long lda, int c0, int c1, int c2, int c3, int nswaps,
                      const void* plan, hipStream_t s) {
  constexpr int Q = 16;
  if (c1 < c0) c1 = c0;
  if (c3 < c2) c3 = c2;
  if (nswaps <= 0 || (c1 == c0 && c3 == c2)) return LP_OK;
  const int maxent = 2 * nswaps;
  int CW = 64;
  while (CW > 1 && maxent * CW > 1024 * Q) CW >>= 1;
  const long long blocks = cdiv(c1 - c0, CW) + cdiv(c3 - c2, CW);
  hipLaunchKernelGGL((swap_apply_kernel<T, Q>), dim3((unsigned)blocks), dim3(1024), 0, s, A, lda,
                     c0, c1, c2, c3, CW, (const int*)plan);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

// The interchanges k1 .. k2-1 applied to columns [c0, c1) in one launch:
// every workgroup builds the plan in LDS from ipiv (the same parallel
// construction as swap_plan_kernel) and gathers its column chunk.  For the
// narrow column ranges inside a split panel, where the separate plan launch
// cost more than building it once per workgroup.
template <typename T, int Q>
__global__ __launch_bounds__(1024) void swap_fused_kernel(T* __restrict__ A, long long lda, int c0,
                                                          int c1, int CW,
                                                          const int32_t* __restrict__ ipiv,
                                                          int k1, int k2) {
  __shared__ int piv[kPlanMax];
  __shared__ int nxt[kPlanMax];
  __shared__ int Bv[kPlanMax];
  __shared__ int flag[2 * kPlanMax];
  __shared__ int dst[2 * kPlanMax];
  __shared__ int src[2 * kPlanMax];
  __shared__ int nent_s;
  const int k = k2 - k1;
  if ((int)threadIdx.x < k) piv[threadIdx.x] = ipiv[k1 + threadIdx.x];
  __syncthreads();
  build_swap_plan(piv, k1, k2, nxt, Bv, nullptr, flag, dst, src, &nent_s);
  __syncthreads();
  const int nent = nent_s;
  const int cs = c0 + blockIdx.x * CW;
  const int width = min(c1, cs + CW) - cs;
  T v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + 1024 * q;
    const int ent = e / CW;
    const int col = e - ent * CW;
    if (ent < nent && col < width) v[q] = A[(long long)src[ent] * lda + cs + col];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int e = threadIdx.x + 1024 * q;
    const int ent = e / CW;
    const int col = e - ent * CW;
    if (ent < nent && col < width) A[(long long)dst[ent] * lda + cs + col] = v[q];
  }
}

template <typename T>
int launch_swap_fused(T* A, long long lda, int c0, int c1, const int32_t* ipiv, int k1, int k2,
                      hipStream_t s) {
  constexpr int Q = 16;
  const int k = k2 - k1;
  if (k <= 0 || c1 <= c0) return LP_OK;
  if (k > kPlanMax) return LP_ENOTSUP;
  int CW = 64;
  while (CW > 1 && 2 * k * CW > 1024 * Q) CW >>= 1;
  hipLaunchKernelGGL((swap_fused_kernel<T, Q>), dim3((unsigned)cdiv(c1 - c0, CW)), dim3(1024), 0,
                     s, A, lda, c0, c1, CW, ipiv, k1, k2);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

template int launch_swap_fused<double>(double*, long long, int, int, const int32_t*, int, int,
                                       hipStream_t);
template int launch_swap_fused<float>(float*, long long, int, int, const int32_t*, int, int,
                                      hipStream_t);

template int launch_swap_apply<double>(double*, long long, int, int, int, int, int, const void*,
                                       hipStream_t);
template int launch_swap_apply<float>(float*, long long, int, int, int, int, int, const void*,
                                      hipStream_t);

// ------------------------------------------------ unit lower triangular solve
// B := L^-1 B, L unit lower m x m: the paper's "top blocks" update of the
// blocks right of the diagonal block with its lower factor.
//
// Columns of B are independent.  The triangle is taken in 128-row leaves, the
// rows below each leaf brought up to date by the inner-block kernel between
// leaf launches.  In a leaf launch one wave owns a strip of 16 columns and
// keeps the strip's 128 rows (as 16 x 16 tiles) in registers in the MFMA
// output layout, and the workgroup first stages the leaf's strictly lower
// 16 x 16 blocks in LDS.  Block row r is solved by multiplying with the
// precomputed inverse of the 16 x 16 diagonal block L_rr, then subtracted
// from every later block row (X_q -= L_qr X_r), all on the matrix cores.  For
// both MFMA shapes
// used here there is an ordering of the 4-long k-steps for which output
// register t of a lane is exactly that lane's B operand in k-step t, so solved
// tiles feed the next products without leaving registers:
//   FP64 16x16x4: output (lane l, reg v) = D[l/16 + 4v][l%16]; step t uses k = l/16 + 4t
//   FP32 16x16x4: output (lane l, reg v) = D[4(l/16) + v][l%16]; step t uses k = 4(l/16) + t
// (A operand: lane l supplies row l % 16 at that k; layouts checked on the device.)
// Inverse of each 16 x 16 unit lower diagonal block of L (rows beyond m are
// treated as identity).  Linv[r] is stored row-major, 256 entries per block.
template <typename T>
__global__ __launch_bounds__(64) void diag_block_inverse_kernel(int m, const T* __restrict__ L,
                                                                long long ldl,
                                                                T* __restrict__ Linv) {
  const int r = blockIdx.x;
  const int j = threadIdx.x;
  __shared__ T Ls[16][17];
  for (int e = threadIdx.x; e < 256; e += 64) {
    const int i = e >> 4, k = e & 15;
    const int gi = 16 * r + i, gk = 16 * r + k;
    Ls[i][k] = (gi < m && gk < m) ? L[(long long)gi * ldl + gk] : T(0);
  }
  __syncthreads();
  if (j < 16) {
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = (i == j) ? T(1) : T(0);
#pragma unroll
    for (int i = 1; i < 16; ++i) {
      T acc = x[i];
#pragma unroll
      for (int k = 0; k < i; ++k) acc -= Ls[i][k] * x[k];
      x[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Linv[(long long)r * 256 + i * 16 + j] = x[i];
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(256) void trsm_mfma_kernel(int m, int ncols, const T* __restrict__ L,
                                                        long long ldl,
                                                        const T* __restrict__ Linv,
                                                        T* __restrict__ B, long long ldb) {
  typedef Mfma16<T> M;
  typedef typename M::acc acc_t;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int c16 = lane & 15;
  const int col = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + c16;
  const bool colok = col < ncols;
  const int nt = (m + 15) >> 4;
  // the strictly lower 16 x 16 blocks of the leaf, L(q, r) for q > r, staged
  // in LDS by the whole workgroup with one round trip (rows past m as zeros):
  // the solve below then waits on LDS, not on memory, at every step
  constexpr int kPairs = NT * (NT - 1) / 2;
  __shared__ T Ls[kPairs > 0 ? kPairs : 1][16][17];
  if constexpr (kPairs > 0) {
    const int i = threadIdx.x >> 4, k = threadIdx.x & 15;
    T v[kPairs];
    int u = 0;
#pragma unroll
    for (int q = 1; q < NT; ++q)
#pragma unroll
      for (int r = 0; r < q; ++r, ++u) {
        const int row = 16 * q + i;
        const bool ok = q < nt && row < m;
        const T a = L[(long long)(ok ? row : 0) * ldl + (ok ? 16 * r + k : 0)];
        v[u] = ok ? a : T(0);
      }
    u = 0;
#pragma unroll
    for (int q = 1; q < NT; ++q)
#pragma unroll
      for (int r = 0; r < q; ++r, ++u) Ls[u][i][k] = v[u];
    __syncthreads();
  }
  acc_t X[NT];
#pragma unroll
  for (int r = 0; r < NT; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * r + M::drow(g, v);
      X[r][v] = (r < nt && row < m && colok) ? B[(long long)row * ldb + col] : T(0);
    }
  }
#pragma unroll
  for (int r = 0; r < NT; ++r) {
    if (r < nt) {
      acc_t Y = {0, 0, 0, 0};
      const T* li = Linv + (long long)r * 256 + c16 * 16;
#pragma unroll
      for (int t = 0; t < 4; ++t) Y = M::mma(li[M::kidx(g, t)], X[r][t], Y);
      X[r] = Y;
#pragma unroll
      for (int q = r + 1; q < NT; ++q) {
        if (q < nt) {
          const int pq = q * (q - 1) / 2 + r;
#pragma unroll
          for (int t = 0; t < 4; ++t) X[q] = M::mma(-Ls[pq][c16][M::kidx(g, t)], X[r][t], X[q]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NT; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * r + M::drow(g, v);
      if (r < nt && row < m && colok) B[(long long)row * ldb + col] = X[r][v];
    }
  }
}

size_t trsm_workspace_bytes(int m) { return sizeof(double) * 256 * (size_t)cdiv(m, 16); }

// The inverses of every 16 x 16 diagonal block of L depend on L only: one
// launch for all of them.
template <typename T>
int launch_diag_block_inverse(int m, const T* L, long long ldl, void* work, hipStream_t s) {
  if (m <= 0) return LP_OK;
  hipLaunchKernelGGL((diag_block_inverse_kernel<T>), dim3((unsigned)cdiv(m, 16)), dim3(64), 0, s,
                     m, L, ldl, (T*)work);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

// Triangles taller than 128 rows: solve the first 128 rows, subtract their
// contribution from the rows below with the inner-block update kernel, repeat.
template <typename T>
int launch_trsm_lower_unit(int m, int ncols, const T* L, long long ldl, T* B, long long ldb,
                           void* work, hipStream_t s, bool inverses_ready) {
  if (m <= 0 || ncols <= 0) return LP_OK;
  // 128-row leaves: a shorter dependency chain per wave than 256, and the
  // updates between leaves run on the GEMM kernel (1.7x faster than 256-row
  // leaves at nb = 256 and 512)
  constexpr int kChunk = 128;
  if (!inverses_ready) {
    const int rc = launch_diag_block_inverse<T>(m, L, ldl, work, s);
    if (rc != LP_OK) return rc;
  }
  for (int r0 = 0; r0 < m; r0 += kChunk) {
    const int mc = min(kChunk, m - r0);
    const T* Lc = L + (long long)r0 * ldl + r0;
    T* Bc = B + (long long)r0 * ldb;
    const int nt = (int)cdiv(mc, 16);
    const T* Linv = (const T*)work + (size_t)(r0 / 16) * 256;
    const dim3 grid((unsigned)cdiv(ncols, 64));
    bool done = false;
#define LP_TRSM_CASE(NTV)                                                                     \
    if (!done && nt <= NTV) {                                                                 \
      hipLaunchKernelGGL((trsm_mfma_kernel<T, NTV>), grid, dim3(256), 0, s, mc, ncols, Lc, ldl, \
                         (const T*)Linv, Bc, ldb);                                            \
      LP_LAUNCH_CHECK();                                                                      \
      done = true;                                                                            \
    }
    LP_TRSM_CASE(1)
    LP_TRSM_CASE(2)
    LP_TRSM_CASE(4)
    LP_TRSM_CASE(8)
#undef LP_TRSM_CASE
    if (!done) return LP_ENOTSUP;
    const int rest = m - r0 - mc;
    if (rest > 0) {
      const int prec = sizeof(T) == 8 ? LP_FP64 : LP_FP32;
      int rc = launch_gemm_update(prec, rest, ncols, mc, L + (long long)(r0 + mc) * ldl + r0, ldl,
                                  Bc, ldb, B + (long long)(r0 + mc) * ldb, ldb, s, kGemmPanel);
      if (rc != LP_OK) return rc;
    }
  }
  return LP_OK;
}

template int launch_diag_block_inverse<double>(int, const double*, long long, void*,
                                               hipStream_t);
template int launch_diag_block_inverse<float>(int, const float*, long long, void*, hipStream_t);
template int launch_trsm_lower_unit<double>(int, int, const double*, long long, double*,
                                            long long, void*, hipStream_t, bool);
template int launch_trsm_lower_unit<float>(int, int, const float*, long long, float*, long long,
                                           void*, hipStream_t, bool);

}  // namespace lp

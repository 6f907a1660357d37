// The "left blocks" of the no-pivot LU: L21 = A21 U11^-1.
//
// Paper, section "High Performance Linpack", "Base Implementation" (figure
// fig:lu_iteration): without pivoting each iteration decomposes the diagonal
// block into L11 U11, then updates the blocks below it with U11 (the "left"
// blocks, L21 U11 = A21), the blocks right of it with L11 (the "top" blocks,
// L11 U12 = A12) and the inner blocks with one multiplication.  The left
// update here is a right-side solve with an upper, non-unit triangle, done on
// the matrix cores: rows of A21 are independent, so the work spreads over the
// whole device instead of the one column at a time of a pivoted panel.
//
// X U = B is solved as U^T X^T = B^T, the mirror of the unit-lower solve of
// the top blocks (panel.hip): one wave keeps 16 rows of B as the columns of
// 16 x 16 tiles of B^T in registers (MFMA output layout), solves tile r by
// multiplying with the transposed inverse of the 16 x 16 diagonal block U_rr,
// and subtracts U_rq^T X_r from every later tile q.  Triangles wider than 128
// columns go in 128-column chunks with the inner-block kernel between them.
#include "common.h"
#include "device.h"

namespace lp {
namespace {

// For each 16 x 16 diagonal block U_rr of the upper triangle U (m x m), the
// transpose of its inverse: S_r[i][k] = (U_rr^-1)[k][i], row-major, 256
// values per block.  Column j of U_rr^-1 is found by back substitution with
// correctly rounded divisions by the diagonal; rows past m act as identity.
template <typename T>
__global__ __launch_bounds__(64) void upper_block_inverse_kernel(int m, const T* __restrict__ U,
                                                                 long long ldu,
                                                                 T* __restrict__ S) {
  const int r = blockIdx.x;
  const int j = threadIdx.x;
  __shared__ T Us[16][17];
  for (int e = threadIdx.x; e < 256; e += 64) {
    const int i = e >> 4, k = e & 15;
    const int gi = 16 * r + i, gk = 16 * r + k;
    Us[i][k] = (gi < m && gk < m) ? U[(long long)gi * ldu + gk] : (i == k ? T(1) : T(0));
  }
  __syncthreads();
  if (j < 16) {
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = (i == j) ? T(1) : T(0);
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      T acc = x[i];
#pragma unroll
      for (int k = i + 1; k < 16; ++k) acc -= Us[i][k] * x[k];
      x[i] = acc / Us[i][i];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) S[(long long)r * 256 + j * 16 + k] = x[k];
  }
}

// B := B U^-1 for one chunk of w <= 16 NT columns (U: the chunk's diagonal
// triangle, ld ldu; S: its block inverses).  Lane (g, c16) of a wave holds
// row (strip + c16) of B; register v of tile r is column 16 r + drow(g, v),
// i.e. entry (drow(g, v), c16) of the tile of B^T, which for both MFMA shapes
// is that lane's B operand in k-step v of the next product.
template <typename T, int NT>
__global__ __launch_bounds__(256) void trsm_right_upper_kernel(int m, int w,
                                                               const T* __restrict__ U,
                                                               long long ldu,
                                                               const T* __restrict__ S,
                                                               T* __restrict__ B, long long ldb) {
  typedef Mfma16<T> M;
  typedef typename M::acc acc_t;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int c16 = lane & 15;
  const int row = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + c16;
  const bool rowok = row < m;
  const int nt = (w + 15) >> 4;
  const long long rbase = (long long)(rowok ? row : 0) * ldb;
  // the blocks above the diagonal, transposed: Ut[p(q, r)][i][k] =
  // U[16 r + k][16 q + i] for q > r, staged in LDS by the whole workgroup with
  // one round trip (coalesced along U's rows; entries past w as zeros)
  constexpr int kPairs = NT * (NT - 1) / 2;
  __shared__ T Ut[kPairs > 0 ? kPairs : 1][16][17];
  if constexpr (kPairs > 0) {
    const int a = threadIdx.x >> 4, b = threadIdx.x & 15;
    T v[kPairs];
    int u = 0;
#pragma unroll
    for (int q = 1; q < NT; ++q)
#pragma unroll
      for (int r = 0; r < q; ++r, ++u) {
        const int ur = 16 * r + a, uc = 16 * q + b;
        const bool ok = q < nt && ur < w && uc < w;
        const T x = U[(long long)(ok ? ur : 0) * ldu + (ok ? uc : 0)];
        v[u] = ok ? x : T(0);
      }
    u = 0;
#pragma unroll
    for (int q = 1; q < NT; ++q)
#pragma unroll
      for (int r = 0; r < q; ++r, ++u) Ut[u][b][a] = v[u];
    __syncthreads();
  }
  acc_t X[NT];
#pragma unroll
  for (int r = 0; r < NT; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * r + M::drow(g, v);
      const bool ok = r < nt && col < w && rowok;
      const T raw = B[rbase + (ok ? col : 0)];
      X[r][v] = ok ? raw : T(0);
    }
  }
#pragma unroll
  for (int r = 0; r < NT; ++r) {
    if (r < nt) {
      acc_t Y = {0, 0, 0, 0};
      const T* si = S + (long long)r * 256 + c16 * 16;
#pragma unroll
      for (int t = 0; t < 4; ++t) Y = M::mma(si[M::kidx(g, t)], X[r][t], Y);
      X[r] = Y;
#pragma unroll
      for (int q = r + 1; q < NT; ++q) {
        if (q < nt) {
          // (U^T)_qr[i][k] = U[16 r + k][16 q + i]: lane c16 supplies i
          const int pq = q * (q - 1) / 2 + r;
#pragma unroll
          for (int t = 0; t < 4; ++t) X[q] = M::mma(-Ut[pq][c16][M::kidx(g, t)], X[r][t], X[q]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NT; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * r + M::drow(g, v);
      if (r < nt && col < w && rowok) B[rbase + col] = X[r][v];
    }
  }
}

constexpr int kRightChunk = 128;

}  // namespace

template <typename T>
int launch_trsm_right_upper(int m, int w, const T* U, long long ldu, T* B, long long ldb,
                            void* work, hipStream_t s) {
  if (m <= 0 || w <= 0) return LP_OK;
  const dim3 grid((unsigned)cdiv(m, 64));
  for (int c0 = 0; c0 < w; c0 += kRightChunk) {
    const int wc = min(kRightChunk, w - c0);
    const T* Uc = U + (long long)c0 * ldu + c0;
    T* Bc = B + c0;
    const int nt = (int)cdiv(wc, 16);
    T* Sinv = (T*)work;
    hipLaunchKernelGGL((upper_block_inverse_kernel<T>), dim3(nt), dim3(64), 0, s, wc, Uc, ldu,
                       Sinv);
    LP_LAUNCH_CHECK();
    bool done = false;
#define LP_RTRSM_CASE(NTV)                                                                    \
    if (!done && nt <= NTV) {                                                                 \
      hipLaunchKernelGGL((trsm_right_upper_kernel<T, NTV>), grid, dim3(256), 0, s, m, wc, Uc, \
                         ldu, (const T*)Sinv, Bc, ldb);                                       \
      LP_LAUNCH_CHECK();                                                                      \
      done = true;                                                                            \
    }
    LP_RTRSM_CASE(1)
    LP_RTRSM_CASE(2)
    LP_RTRSM_CASE(4)
    LP_RTRSM_CASE(8)
#undef LP_RTRSM_CASE
    if (!done) return LP_ENOTSUP;
    const int rest = w - c0 - wc;
    if (rest > 0) {
      // the solved columns' contribution to the columns right of the chunk
      const int prec = sizeof(T) == 8 ? LP_FP64 : LP_FP32;
      int rc = launch_gemm_update(prec, m, rest, wc, Bc, ldb, Uc + wc, ldu, Bc + wc, ldb, s,
                                  kGemmPanel);
      if (rc != LP_OK) return rc;
    }
  }
  return LP_OK;
}

template int launch_trsm_right_upper<double>(int, int, const double*, long long, double*,
                                             long long, void*, hipStream_t);
template int launch_trsm_right_upper<float>(int, int, const float*, long long, float*, long long,
                                            void*, hipStream_t);

}  // namespace lp

// Matrix transposition with addition, C = B + A^T.
//
// Paper, section "Parallel Matrix Transposition": the PTRANS benchmark adds
// the transpose of A to B and stores the result in C, block by block; its
// kernel reads a block of A into a local buffer, reads it back transposed
// while streaming the matching block of B, and writes the sum.  Here one
// workgroup owns a 64 x 64 tile: the A tile (rows r0.., columns c0..) comes
// in with row-contiguous, coalesced loads and is stored in LDS with an odd
// row stride, then each wave reads one row of the transposed tile from LDS
// (consecutive lanes hit consecutive bank pairs), adds the row-contiguous B
// tile (rows c0.., columns r0..) and writes C the same way.  Every element of
// A, B and C crosses HBM once: the kernel is bound by HBM bandwidth
// (3 n^2 elements per call), and the addition is one correctly rounded add
// per element, so the result is exact to the bit against any plain
// implementation.
#include "common.h"

namespace lp {
namespace {

constexpr int kTile = 64;
constexpr int kRowsPerPass = 4;                 // 256 threads = 4 rows of 64 per pass
constexpr int kPasses = kTile / kRowsPerPass;  // 16 loads in flight per thread

template <typename T>
__global__ __launch_bounds__(256) void ptrans_kernel(int n, const T* __restrict__ A,
                                                     long long lda, const T* B,
                                                     long long ldb, T* C, long long ldc,
                                                     int tiles_per_row) {
  __shared__ T tile[kTile][kTile + 1];
  const int tr = blockIdx.x / tiles_per_row;  // tile row of A
  const int tc = blockIdx.x % tiles_per_row;  // tile column of A
  const int r0 = tr * kTile, c0 = tc * kTile;
  const int j = threadIdx.x & (kTile - 1);
  const int i0 = threadIdx.x >> 6;
  T v[kPasses];
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int r = r0 + i0 + kRowsPerPass * p, c = c0 + j;
    const bool ok = r < n && c < n;
    v[p] = ok ? A[(long long)r * lda + c] : T(0);
  }
#pragma unroll
  for (int p = 0; p < kPasses; ++p) tile[i0 + kRowsPerPass * p][j] = v[p];
  __syncthreads();
  // C rows c0.., columns r0..: C[c0 + i][r0 + j] = B[c0 + i][r0 + j] + A[r0 + j][c0 + i]
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int i = i0 + kRowsPerPass * p;
    const int row = c0 + i, col = r0 + j;
    const bool ok = row < n && col < n;
    v[p] = ok ? B[(long long)row * ldb + col] : T(0);
  }
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int i = i0 + kRowsPerPass * p;
    const int row = c0 + i, col = r0 + j;
    if (row < n && col < n) C[(long long)row * ldc + col] = v[p] + tile[j][i];
  }
}

}  // namespace

int launch_ptrans(int prec, int n, const void* A, long long lda, const void* B, long long ldb,
                  void* C, long long ldc, hipStream_t s) {
  if (n <= 0) return LP_OK;
  const int t = (int)cdiv(n, kTile);
  const long long ntiles = (long long)t * t;
  if (ntiles > 0x7fffffffLL) return LP_ENOTSUP;
  if (prec == LP_FP64)
    hipLaunchKernelGGL((ptrans_kernel<double>), dim3((unsigned)ntiles), dim3(256), 0, s, n,
                       (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, t);
  else
    hipLaunchKernelGGL((ptrans_kernel<float>), dim3((unsigned)ntiles), dim3(256), 0, s, n,
                       (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, t);
  LP_LAUNCH_CHECK();
  return LP_OK;
}

}  // namespace lp

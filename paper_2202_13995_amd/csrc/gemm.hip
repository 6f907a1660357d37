// Inner-block update C := C - A B on the gfx950 matrix cores.
//
// This is the "inner blocks" step of the blocked right-looking LU (paper,
// section "High Performance Linpack", "Base Implementation": the left and top
// blocks update all inner blocks by matrix multiplication), which carries
// almost all of the flops.  The paper's FPGA kernel unrolls a register block
// in three dimensions; here the register block is the MFMA fragment and the
// local-memory block is an LDS tile.
//
// FP64 kernel: v_mfma_f64_16x16x4_f64.  Operand layout of one wave (64 lanes):
//   A operand: lane l supplies A[row = l % 16][k = l / 16]
//   B operand: lane l supplies B[k = l / 16][col = l % 16]
//   C/D:       lane l, element v holds D[row = l / 16 + 4 * v][col = l % 16]
// (checked on the device with a one-hot probe of the builtin).
// A workgroup (4 waves) owns a 128 x 128 tile of C; wave w owns the 64 x 64
// quadrant (w / 2, w % 2) as 4 x 4 fragments.  K advances in slabs of 16 through
// two LDS buffers (one barrier per slab).  Within a slab the four MFMA k-steps
// take k = 4 q + s for lane group q = l / 16 and step s, so each lane reads its
// four A values as one contiguous 32-byte run (the summation order inside a
// dot product is free).  The accumulators start at -C and the tile is written
// back negated, which gives C - A B with one rounding per MFMA step.
//
// Tile order: hardware dispatches workgroup b to XCD b % 8.  The launcher
// numbers tiles so that each XCD receives a contiguous range of tile ids, and
// ids walk 8-row groups column by column, so tiles resident on one XCD share A
// row panels and B column panels in that XCD's L2.
#include "common.h"

namespace lp {
namespace {

constexpr int DBM = 128;
constexpr int DBN = 128;
constexpr int DBK = 16;
constexpr int DAS = DBK + 2;  // A tile row stride in LDS (doubles): conflict-free b128 reads
constexpr int GROUP_M = 8;

__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int loc = bid >> 3;
  const int per = T >> 3;
  const int rem = T & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + loc;
  const int group_size = GROUP_M * tiles_n;
  const int g = tile / group_size;
  const int first_m = g * GROUP_M;
  const int gm = min(GROUP_M, tiles_m - first_m);
  const int within = tile - g * group_size;
  tm = first_m + within % gm;
  tn = within / gm;
}

__device__ __forceinline__ void dgemm_update_body(
    int M, int N, int K, const double* __restrict__ A, long long lda,
    const double* __restrict__ B, long long ldb, double* __restrict__ C, long long ldc,
    int tiles_m, int tiles_n) {
  __shared__ __align__(16) double As[2][DBM * DAS];
  __shared__ __align__(16) double Bs[2][DBK * DBN];

  int tm, tn;
  tile_coords(tiles_m, tiles_n, tm, tn);
  const int row0 = tm * DBM;
  const int col0 = tn * DBN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const int l16 = lane & 15;
  const int q = lane >> 4;

  // accumulators start at -C
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + wn + 16 * j + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wm + 16 * i + q + 4 * v;
        acc[i][j][v] = (r < M && c < N) ? -C[(long long)r * ldc + c] : 0.0;
      }
    }
  }

  // global -> register staging: A tile (128 x 16): k = tid & 15, rows (tid >> 4) + 16 p;
  // B tile (16 x 128): col = tid & 127, k = (tid >> 7) + 2 p.
  double ra[8], rb[8];
  const int a_k = tid & 15;
  const int a_r = tid >> 4;
  const int b_c = tid & 127;
  const int b_k = tid >> 7;
  const bool b_col_ok = (col0 + b_c) < N;

  auto gload = [&](int k0) {
    const int ka = k0 + a_k;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int r = row0 + a_r + 16 * p;
      ra[p] = (r < M && ka < K) ? A[(long long)r * lda + ka] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int kb = k0 + b_k + 2 * p;
      rb[p] = (kb < K && b_col_ok) ? B[(long long)kb * ldb + col0 + b_c] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 8; ++p) As[buf][(a_r + 16 * p) * DAS + a_k] = ra[p];
#pragma unroll
    for (int p = 0; p < 8; ++p) Bs[buf][(b_k + 2 * p) * DBN + b_c] = rb[p];
  };

  const int nk = (K + DBK - 1) / DBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int s = 0; s < nk; ++s) {
    const int buf = s & 1;
    if (s + 1 < nk) gload((s + 1) * DBK);
    const double* as = As[buf] + (wm + l16) * DAS + 4 * q;
    const double* bs = Bs[buf] + (4 * q) * DBN + wn + l16;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = as[16 * i * DAS + ks];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = bs[ks * DBN + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      }
    }
    if (s + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + wn + 16 * j + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wm + 16 * i + q + 4 * v;
        if (r < M && c < N) C[(long long)r * ldc + c] = -acc[i][j][v];
      }
    }
  }
}

// The trailing-matrix update and the updates inside a panel run the same body
// under two names so that traces separate them.
__global__ __launch_bounds__(256, 2) void dgemm_trailing_update(
    int M, int N, int K, const double* __restrict__ A, long long lda,
    const double* __restrict__ B, long long ldb, double* __restrict__ C, long long ldc,
    int tiles_m, int tiles_n) {
  dgemm_update_body(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
}

__global__ __launch_bounds__(256, 2) void dgemm_panel_update(
    int M, int N, int K, const double* __restrict__ A, long long lda,
    const double* __restrict__ B, long long ldb, double* __restrict__ C, long long ldc,
    int tiles_m, int tiles_n) {
  dgemm_update_body(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
}

}  // namespace

int launch_gemm_update(int prec, int M, int N, int K, const void* A, long long lda,
                       const void* B, long long ldb, void* C, long long ldc, hipStream_t s,
                       int kind) {
  if (M <= 0 || N <= 0 || K <= 0) return LP_OK;
  if (prec == LP_FP64) {
    const int tiles_m = (int)cdiv(M, DBM);
    const int tiles_n = (int)cdiv(N, DBN);
    const long long T = (long long)tiles_m * tiles_n;
    if (T > 0x7fffffffLL) return LP_ENOTSUP;
    if (kind == kGemmPanel)
      hipLaunchKernelGGL(dgemm_panel_update, dim3((unsigned)T), dim3(256), 0, s, M, N, K,
                         (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, tiles_m,
                         tiles_n);
    else
      hipLaunchKernelGGL(dgemm_trailing_update, dim3((unsigned)T), dim3(256), 0, s, M, N, K,
                         (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, tiles_m,
                         tiles_n);
    LP_LAUNCH_CHECK();
    return LP_OK;
  }
  return launch_gemm_update_lp(prec, M, N, K, (const float*)A, lda, (const float*)B, ldb,
                               (float*)C, ldc, s);
}

}  // namespace lp

// Inner-block update C := C - A B for binary32 storage (the low-precision
// factorization).  The paper lets the LINPACK kernels run in single or double
// precision (section "High Performance Linpack"); here the trailing matrix is
// kept in binary32 and the multiplication's operands are fed to the matrix
// cores as binary32 (v_mfma_f32_16x16x4_f32), bfloat16 or half
// (v_mfma_f32_16x16x32_{bf16,f16}); accumulation is always binary32.  The
// narrowing to bfloat16 / half is round-to-nearest-even and happens once per
// element on the way from memory into LDS.
//
// Layout facts used here (checked on the device with one-hot probes):
//   output (lane l, reg v) = D[4 (l/16) + v][l % 16] for all three shapes;
//   A operand: lane l supplies row l % 16, B operand column l % 16, and the
//   k slots of a lane group g = l / 16 pair up between A and B.  We give group
//   g the k range [4g, 4g+4) (f32, one value per step, four steps) or
//   [8g, 8g+8) (bf16/f16, eight values in one step), so each lane reads its
//   operands as one 16-byte run from LDS.  The B tile is stored transposed
//   (column-major in k) for the same reason.
//
// A workgroup (4 waves) owns a 128 x 128 tile of C, wave w the 64 x 64 quadrant
// (w / 2, w % 2) as 4 x 4 fragments; K advances in slabs through two LDS
// buffers (one barrier per slab); accumulators start at -C and the tile is
// written back negated.  Tiles are numbered XCD-aware as in the FP64 kernel.
#include "common.h"

namespace lp {
namespace {

enum class Op { F32, BF16, F16 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <Op OP>
struct OpTraits;
template <>
struct OpTraits<Op::F32> {
  typedef float elem;
  static constexpr int BK = 16;   // four k-steps of 4
  static constexpr int KSTEPS = 4;
};
template <>
struct OpTraits<Op::BF16> {
  typedef __bf16 elem;
  static constexpr int BK = 32;   // one k-step of 32
  static constexpr int KSTEPS = 1;
};
template <>
struct OpTraits<Op::F16> {
  typedef _Float16 elem;
  static constexpr int BK = 32;
  static constexpr int KSTEPS = 1;
};

constexpr int SBM = 128;
constexpr int SBN = 128;
constexpr int SGROUP_M = 8;

__device__ __forceinline__ void tile_coords_lp(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int loc = bid >> 3;
  const int per = T >> 3;
  const int rem = T & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + loc;
  const int group_size = SGROUP_M * tiles_n;
  const int g = tile / group_size;
  const int first_m = g * SGROUP_M;
  const int gm = min(SGROUP_M, tiles_m - first_m);
  const int within = tile - g * group_size;
  tm = first_m + within % gm;
  tn = within / gm;
}

template <Op OP>
__global__ __launch_bounds__(256, 2) void sgemm_update_kernel(
    int M, int N, int K, const float* __restrict__ A, long long lda, const float* __restrict__ B,
    long long ldb, float* __restrict__ C, long long ldc, int tiles_m, int tiles_n) {
  typedef typename OpTraits<OP>::elem E;
  constexpr int BK = OpTraits<OP>::BK;
  constexpr int KS = OpTraits<OP>::KSTEPS;
  constexpr int PAD = 16 / sizeof(E);     // 16-byte pad per row: conflict-free 16 B reads
  constexpr int LS = BK + PAD;            // LDS row stride (elements)
  __shared__ __align__(16) E As[2][SBM * LS];
  __shared__ __align__(16) E Bs[2][SBN * LS];  // transposed: [col][k]

  int tm, tn;
  tile_coords_lp(tiles_m, tiles_n, tm, tn);
  const int row0 = tm * SBM;
  const int col0 = tn * SBN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const int l16 = lane & 15;
  const int g = lane >> 4;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + wn + 16 * j + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wm + 16 * i + 4 * g + v;
        acc[i][j][v] = (r < M && c < N) ? -C[(long long)r * ldc + c] : 0.0f;
      }
    }

  // global -> registers: A tile SBM x BK (k fastest), B tile BK x SBN (col fastest)
  constexpr int NA = SBM * BK / 256;
  constexpr int NB = BK * SBN / 256;
  float ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + 256 * i;
      const int r = e / BK, k = e - r * BK;
      const int gr = row0 + r, gk = k0 + k;
      ra[i] = (gr < M && gk < K) ? A[(long long)gr * lda + gk] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      const int k = e / SBN, c = e - k * SBN;
      const int gk = k0 + k, gc = col0 + c;
      rb[i] = (gk < K && gc < N) ? B[(long long)gk * ldb + gc] : 0.0f;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + 256 * i;
      const int r = e / BK, k = e - r * BK;
      As[buf][r * LS + k] = (E)ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      const int k = e / SBN, c = e - k * SBN;
      Bs[buf][c * LS + k] = (E)rb[i];
    }
  };

  const int nk = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int s = 0; s < nk; ++s) {
    const int buf = s & 1;
    if (s + 1 < nk) gload((s + 1) * BK);
    const E* as = As[buf];
    const E* bs = Bs[buf];
    if constexpr (OP == Op::F32) {
      // lane group g owns k = 4g .. 4g+3; step t uses k = 4g + t
      f4 a4[4], b4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a4[i] = *reinterpret_cast<const f4*>(as + (wm + 16 * i + l16) * LS + 4 * g);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b4[j] = *reinterpret_cast<const f4*>(bs + (wn + 16 * j + l16) * LS + 4 * g);
#pragma unroll
      for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[i][t], b4[j][t], acc[i][j], 0, 0, 0);
    } else {
      // lane group g owns k = 8g .. 8g+7 in the single 32-deep step
      typedef typename std::conditional<OP == Op::BF16, bf16x8, f16x8>::type v8;
      v8 a8[4], b8[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a8[i] = *reinterpret_cast<const v8*>(as + (wm + 16 * i + l16) * LS + 8 * g);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b8[j] = *reinterpret_cast<const v8*>(bs + (wn + 16 * j + l16) * LS + 8 * g);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if constexpr (OP == Op::BF16)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8[i], b8[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a8[i], b8[j], acc[i][j], 0, 0, 0);
        }
    }
    if (s + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + wn + 16 * j + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wm + 16 * i + 4 * g + v;
        if (r < M && c < N) C[(long long)r * ldc + c] = -acc[i][j][v];
      }
    }
}

}  // namespace

int launch_gemm_update_lp(int prec, int M, int N, int K, const float* A, long long lda,
                          const float* B, long long ldb, float* C, long long ldc, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return LP_OK;
  const int tiles_m = (int)cdiv(M, SBM);
  const int tiles_n = (int)cdiv(N, SBN);
  const long long T = (long long)tiles_m * tiles_n;
  if (T > 0x7fffffffLL) return LP_ENOTSUP;
  const dim3 grid((unsigned)T);
  if (prec == LP_FP32)
    hipLaunchKernelGGL(sgemm_update_kernel<Op::F32>, grid, dim3(256), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, tiles_m, tiles_n);
  else if (prec == LP_BF16)
    hipLaunchKernelGGL(sgemm_update_kernel<Op::BF16>, grid, dim3(256), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, tiles_m, tiles_n);
  else if (prec == LP_FP16)
    hipLaunchKernelGGL(sgemm_update_kernel<Op::F16>, grid, dim3(256), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, tiles_m, tiles_n);
  else
    return LP_ENOTSUP;
  LP_LAUNCH_CHECK();
  return LP_OK;
}

}  // namespace lp

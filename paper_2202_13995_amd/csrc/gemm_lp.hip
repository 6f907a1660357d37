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
// Three kernels share these conventions:
//   sgemm_update_body / sgemm_update_kernel: any tile, any K.  A workgroup
//     (4 waves) owns a 128 x 128 tile of C, wave w the 64 x 64 quadrant
//     (w / 2, w % 2) as 4 x 4 fragments; K advances in slabs through two LDS
//     buffers (one barrier per slab); accumulators start at -C and the tile is
//     written back negated.
//   sgemm_update_fast: interior 128 x 128 tiles for bfloat16 / half with
//     K = 64 NK, binary32 operands narrowed into LDS (A negated there),
//     accumulators started at C.
//   hgemm_update_packed: operands packed once per block step as 16-bit -A and
//     B^T, 256 x 256 tiles on 8 waves (the factorization's large updates).
// Tiles are numbered XCD-aware as in the FP64 kernel.
#include <type_traits>

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
struct LdsShape {
  typedef typename OpTraits<OP>::elem E;
  static constexpr int BK = OpTraits<OP>::BK;
  static constexpr int PAD = 16 / sizeof(E);  // 16-byte pad per row: conflict-free 16 B reads
  static constexpr int LS = BK + PAD;         // LDS row stride (elements)
  static constexpr int A_ELEMS = SBM * LS;    // one buffer of the A tile
  static constexpr int B_ELEMS = SBN * LS;    // one buffer of the B tile, transposed [col][k]
};

// Any tile, any K: rolled slab loop with predicated loads, one slab of prefetch.
template <Op OP>
__device__ __forceinline__ void sgemm_update_body(
    int M, int N, int K, const float* __restrict__ A, long long lda, const float* __restrict__ B,
    long long ldb, float* __restrict__ C, long long ldc, int row0, int col0,
    typename OpTraits<OP>::elem* As0, typename OpTraits<OP>::elem* Bs0) {
  typedef typename OpTraits<OP>::elem E;
  typedef LdsShape<OP> SH;
  constexpr int BK = OpTraits<OP>::BK;
  constexpr int KS = OpTraits<OP>::KSTEPS;
  constexpr int LS = SH::LS;

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
      As0[buf * SH::A_ELEMS + r * LS + k] = (E)ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      const int k = e / SBN, c = e - k * SBN;
      Bs0[buf * SH::B_ELEMS + c * LS + k] = (E)rb[i];
    }
  };

  const int nk = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int s = 0; s < nk; ++s) {
    const int buf = s & 1;
    if (s + 1 < nk) gload((s + 1) * BK);
    const E* as = As0 + buf * SH::A_ELEMS;
    const E* bs = Bs0 + buf * SH::B_ELEMS;
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

template <Op OP>
__global__ __launch_bounds__(256, 2) void sgemm_update_kernel(
    int M, int N, int K, const float* __restrict__ A, long long lda, const float* __restrict__ B,
    long long ldb, float* __restrict__ C, long long ldc, int tiles_m, int tiles_n) {
  typedef typename OpTraits<OP>::elem E;
  __shared__ __align__(16) E As[2 * LdsShape<OP>::A_ELEMS];
  __shared__ __align__(16) E Bs[2 * LdsShape<OP>::B_ELEMS];
  int tm, tn;
  tile_coords_lp(tiles_m, tiles_n, tm, tn);
  sgemm_update_body<OP>(M, N, K, A, lda, B, ldb, C, ldc, tm * SBM, tn * SBN, As, Bs);
}

template <int I, int END>
struct StaticForLp {
  template <typename F>
  __device__ __forceinline__ static void run(F&& f) {
    if constexpr (I < END) {
      f(std::integral_constant<int, I>{});
      StaticForLp<I + 1, END>::run(f);
    }
  }
};

constexpr unsigned kRsrcWord3Lp = 0x00020000u;  // raw buffer, 32-bit data format

// Interior tiles of the bfloat16 / half update with K = 64 * NK.  The binary32
// operand slabs (64 deep: two MFMA k-steps) are prefetched two slabs ahead
// through two register sets (16-byte buffer loads with 32-bit offsets),
// narrowed as they are written to LDS (A negated there), the accumulators
// start at C (read in the prologue beside the first two slabs) and the slab
// sequence is unrolled, so each LDS write waits only for its own slab.  A
// bfloat16 MFMA step is short, so the bytes in flight, not the multiply,
// set the pace: two 64 KB slabs per workgroup, two workgroups per CU.
// Edge tiles and other K take sgemm_update_body.  Both compute every element
// as the same sequence of rounded steps.
constexpr int kFastBK = 64;
constexpr int kFastLS = kFastBK + 8;  // LDS row stride (16-bit elements): 16-byte pad

template <Op OP, int NK>
__global__ __launch_bounds__(256, 2) void sgemm_update_fast(
    int M, int N, int K, const float* __restrict__ A, long long lda, const float* __restrict__ B,
    long long ldb, float* __restrict__ C, long long ldc, int tiles_m, int tiles_n) {
  typedef typename OpTraits<OP>::elem E;
  typedef LdsShape<OP> SH;
  constexpr int LS = kFastLS;
  constexpr int BUF = SBM * LS;  // elements of one A (or B) buffer
  static_assert(BUF >= SH::A_ELEMS && BUF >= SH::B_ELEMS, "edge body fits the buffers");
  typedef typename std::conditional<OP == Op::BF16, bf16x8, f16x8>::type v8;
  typedef E e4 __attribute__((ext_vector_type(4)));
  __shared__ __align__(16) E As[2 * BUF];
  __shared__ __align__(16) E Bs[2 * BUF];
  int tm, tn;
  tile_coords_lp(tiles_m, tiles_n, tm, tn);
  const int row0 = tm * SBM, col0 = tn * SBN;
  if (!(row0 + SBM <= M && col0 + SBN <= N && K == kFastBK * NK)) {
    sgemm_update_body<OP>(M, N, K, A, lda, B, ldb, C, ldc, row0, col0, As, Bs);
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int l16 = lane & 15, g = lane >> 4;
  const int a_k = (tid & 15) * 4, a_r = tid >> 4;  // A: k quad, rows a_r + 16 p
  // B: one column per lane and four consecutive k (8 p + 4 b_kg + i) per
  // register, so each LDS write of the transposed tile is one 8-byte store
  // (16-bit stores of a column quad hit two banks per wave)
  const int b_n = tid & 127, b_kg = tid >> 7;

  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + (long long)row0 * lda), (short)0, 0x7fffffff, kRsrcWord3Lp);
  const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(B + col0), (short)0, 0x7fffffff, kRsrcWord3Lp);
  const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(C + (long long)(row0 + wm) * ldc + col0 + wn), (short)0, 0x7fffffff, kRsrcWord3Lp);
  const int a_vo = (int)(((long long)a_r * lda + a_k) * 4);
  const int b_vo = (int)(((long long)(4 * b_kg) * ldb + b_n) * 4);
  const int c_vo = (int)(((long long)(4 * g) * ldc + l16) * 4);
  const int a_so = (int)(16 * lda * 4);
  const int b_slab = (int)(kFastBK * ldb * 4);

  f4 rA[2][8], rB[2][8];
  auto load = [&](f4* xa, f4* xb, int s) {
#pragma unroll
    for (int p = 0; p < 8; ++p)
      xa[p] = __builtin_bit_cast(
          f4, __builtin_amdgcn_raw_buffer_load_b128(ra, a_vo + s * kFastBK * 4, p * a_so, 0));
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        xb[p][i] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rb, b_vo + s * b_slab,
                                                        (int)((8 * p + i) * ldb * 4), 0));
  };
  auto store = [&](const f4* xa, const f4* xb, int buf) {
    E* as = As + buf * BUF;
    E* bs = Bs + buf * BUF;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      e4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = -(E)xa[p][i];
      *reinterpret_cast<e4*>(as + (a_r + 16 * p) * LS + a_k) = v;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      e4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (E)xb[p][i];
      *reinterpret_cast<e4*>(bs + b_n * LS + 8 * p + 4 * b_kg) = v;
    }
  };
  f4 acc[4][4];
  // one 32-deep MFMA k-step (kk = 0 or 1) over fragment rows [i0, i1)
  auto mfma_step = [&](int buf, int kk, int i0, int i1) {
    const E* as = As + buf * BUF + 32 * kk + 8 * g;
    const E* bs = Bs + buf * BUF + 32 * kk + 8 * g;
    v8 b8[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b8[j] = *reinterpret_cast<const v8*>(bs + (wn + 16 * j + l16) * LS);
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      const v8 a8 = *reinterpret_cast<const v8*>(as + (wm + 16 * i + l16) * LS);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (OP == Op::BF16)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8[j], acc[i][j], 0, 0, 0);
        else
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a8, b8[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  load(rA[0], rB[0], 0);
  if constexpr (NK > 1) load(rA[1], rB[1], 1);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j][v] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(
                       rc, c_vo + j * 64, (int)((long long)(16 * i + v) * ldc * 4), 0));
  store(rA[0], rB[0], 0);
  __syncthreads();
  StaticForLp<0, NK>::run([&](auto S) {
    constexpr int s = decltype(S)::value;
    constexpr int cur = s & 1, nxt = cur ^ 1;
    if constexpr (s + 2 < NK) load(rA[cur], rB[cur], s + 2);
    mfma_step(cur, 0, 0, 4);
    if constexpr (s + 1 < NK) store(rA[nxt], rB[nxt], nxt);
    mfma_step(cur, 1, 0, 4);
    __syncthreads();
  });
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + wn + 16 * j + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wm + 16 * i + 4 * g + v;
        C[(long long)r * ldc + c] = acc[i][j][v];
      }
    }
}

template <Op OP>
bool launch_fast(int M, int N, int K, const float* A, long long lda, const float* B,
                 long long ldb, float* C, long long ldc, int tiles_m, int tiles_n, hipStream_t s) {
  const bool ok = ((((uintptr_t)A | (uintptr_t)B) & 15) == 0) && ((lda | ldb) & 3) == 0 &&
                  (long long)SBM * lda * 4 < 0x7fffffffLL &&
                  (long long)K * ldb * 4 < 0x7fffffffLL &&
                  (long long)64 * ldc * 4 < 0x7fffffffLL && K % kFastBK == 0;
  if (!ok) return false;
  const dim3 grid((unsigned)((long long)tiles_m * tiles_n));
  switch (K / kFastBK) {
#define LP_FAST_CASE(NKV)                                                                        \
  case NKV:                                                                                      \
    hipLaunchKernelGGL((sgemm_update_fast<OP, NKV>), grid, dim3(256), 0, s, M, N, K, A, lda, B, \
                       ldb, C, ldc, tiles_m, tiles_n);                                           \
    return true;
    LP_FAST_CASE(1)
    LP_FAST_CASE(2)
    LP_FAST_CASE(4)
    LP_FAST_CASE(8)
    LP_FAST_CASE(16)
#undef LP_FAST_CASE
    default:
      return false;
  }
}

// ------------------------------------------------------------ packed operands
// Inside a factorization the bfloat16 / half update takes its operands from
// copies packed once per block step: -A rounded (rows of Kp contiguous 16-bit
// values) and B transposed the same way.  Both tiles then reach LDS through
// 16-byte loads and stores, with half the bytes of the binary32 originals,
// and a workgroup of 8 waves owns a 256 x 256 tile (each wave 128 x 64), so
// every operand byte fetched feeds twice the multiply-adds of the 128 x 128
// kernel.  Rows past M (N) and k past K are packed as zeros, so no operand
// access needs a bound; only C is read and written under one.
constexpr int kPkBK = 64;            // k per slab (two MFMA k-steps)
constexpr int kPkLS = kPkBK + 8;     // LDS row stride (elements): 16-byte pad
constexpr int kPkTile = 256;         // rows (columns) of the C tile
constexpr int kPkBuf = kPkTile * kPkLS;

// A (M x K, lda) -> P (Mp x Kp) as -A; B (K x N, ldb) -> P (Np x Kp) as B^T.
// One thread packs 8 consecutive k of one row (a 16-byte store).
template <Op OP>
__global__ __launch_bounds__(256) void pack_neg_a(int M, int K, const float* __restrict__ A,
                                                  long long lda, int Mp, int Kp,
                                                  typename OpTraits<OP>::elem* __restrict__ P) {
  typedef typename OpTraits<OP>::elem E;
  typedef typename std::conditional<OP == Op::BF16, bf16x8, f16x8>::type v8;
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  const int chunks = Kp / 8;
  if (q >= (long long)Mp * chunks) return;
  const int r = (int)(q / chunks), k0 = (int)(q % chunks) * 8;
  v8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e;
    v[e] = (r < M && k < K) ? -(E)A[(long long)r * lda + k] : (E)0.0f;
  }
  *reinterpret_cast<v8*>(P + (long long)r * Kp + k0) = v;
}

// 64 x 64 blocks through LDS: coalesced reads along B's rows, 16-byte writes
// along P's rows.
template <Op OP>
__global__ __launch_bounds__(256) void pack_bt(int K, int N, const float* __restrict__ B,
                                               long long ldb, int Kp,
                                               typename OpTraits<OP>::elem* __restrict__ P) {
  typedef typename OpTraits<OP>::elem E;
  typedef typename std::conditional<OP == Op::BF16, bf16x8, f16x8>::type v8;
  __shared__ float t[64][65];
  const int k0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  const int c = tid & 63;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int kr = (tid >> 6) + 4 * i;
    const int k = k0 + kr, col = c0 + c;
    t[kr][c] = (k < K && col < N) ? B[(long long)k * ldb + col] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = tid + 256 * h;
    const int cc = q >> 3, kc = (q & 7) * 8;
    v8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (E)t[kc + e][cc];
    *reinterpret_cast<v8*>(P + (long long)(c0 + cc) * Kp + k0 + kc) = v;
  }
}

template <Op OP, int NK>
__global__ __launch_bounds__(512, 1) void hgemm_update_packed(
    int M, int N, const typename OpTraits<OP>::elem* __restrict__ Pa,
    const typename OpTraits<OP>::elem* __restrict__ Pb, float* __restrict__ C, long long ldc,
    int tiles_m, int tiles_n) {
  typedef typename OpTraits<OP>::elem E;
  typedef typename std::conditional<OP == Op::BF16, bf16x8, f16x8>::type v8;
  constexpr int Kp = kPkBK * NK;
  constexpr int LS = kPkLS;
  __shared__ __align__(16) E As[2 * kPkBuf];
  __shared__ __align__(16) E Bs[2 * kPkBuf];
  int tm, tn;
  tile_coords_lp(tiles_m, tiles_n, tm, tn);
  const int row0 = tm * kPkTile, col0 = tn * kPkTile;
  // the wave index is uniform; saying so keeps buffer descriptors in SGPRs
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave & 1) * 128, wn = (wave >> 1) * 64;
  const int l16 = lane & 15, g = lane >> 4;
  const int ld_c = tid & 7, ld_r = tid >> 3;  // 16-byte chunk, rows ld_r + 64 p

  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Pa + (long long)row0 * Kp), (short)0, 0x7fffffff, kRsrcWord3Lp);
  const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Pb + (long long)col0 * Kp), (short)0, 0x7fffffff, kRsrcWord3Lp);
  const int vo = (ld_r * Kp + ld_c * 8) * 2;

  v8 rA[2][4], rB[2][4];
  auto load = [&](v8* xa, v8* xb, int s) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
      xa[p] = __builtin_bit_cast(
          v8, __builtin_amdgcn_raw_buffer_load_b128(ra, vo + s * kPkBK * 2, p * 64 * Kp * 2, 0));
#pragma unroll
    for (int p = 0; p < 4; ++p)
      xb[p] = __builtin_bit_cast(
          v8, __builtin_amdgcn_raw_buffer_load_b128(rb, vo + s * kPkBK * 2, p * 64 * Kp * 2, 0));
  };
  auto store = [&](const v8* xa, const v8* xb, int buf) {
    E* as = As + buf * kPkBuf;
    E* bs = Bs + buf * kPkBuf;
#pragma unroll
    for (int p = 0; p < 4; ++p)
      *reinterpret_cast<v8*>(as + (ld_r + 64 * p) * LS + ld_c * 8) = xa[p];
#pragma unroll
    for (int p = 0; p < 4; ++p)
      *reinterpret_cast<v8*>(bs + (ld_r + 64 * p) * LS + ld_c * 8) = xb[p];
  };
  f4 acc[8][4];
  auto mfma_step = [&](int buf, int kk) {
    const E* as = As + buf * kPkBuf + 32 * kk + 8 * g;
    const E* bs = Bs + buf * kPkBuf + 32 * kk + 8 * g;
    v8 b8[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b8[j] = *reinterpret_cast<const v8*>(bs + (wn + 16 * j + l16) * LS);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const v8 a8 = *reinterpret_cast<const v8*>(as + (wm + 16 * i + l16) * LS);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (OP == Op::BF16)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8[j], acc[i][j], 0, 0, 0);
        else
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a8, b8[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  load(rA[0], rB[0], 0);
  if constexpr (NK > 1) load(rA[1], rB[1], 1);
  const bool interior = row0 + kPkTile <= M && col0 + kPkTile <= N;
  float* Cw = C + (long long)(row0 + wm) * ldc + col0 + wn;  // the wave's block
  float* Ct = Cw + (long long)(4 * g) * ldc + l16;              // the lane's first element
  if (interior) {
    const __amdgpu_buffer_rsrc_t rc =
        __builtin_amdgcn_make_buffer_rsrc((void*)Cw, (short)0, 0x7fffffff, kRsrcWord3Lp);
    const int c_vo = (int)(((long long)(4 * g) * ldc + l16) * 4);
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j][v] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(
                         rc, c_vo + j * 64, (int)((long long)(16 * i + v) * ldc * 4), 0));
  } else {
    const int rlim = M - (row0 + wm + 4 * g), clim = N - (col0 + wn + l16);
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j][v] = (16 * i + v < rlim && 16 * j < clim)
                             ? Ct[(long long)(16 * i + v) * ldc + 16 * j]
                             : 0.0f;
  }
  store(rA[0], rB[0], 0);
  __syncthreads();
  StaticForLp<0, NK>::run([&](auto S) {
    constexpr int s = decltype(S)::value;
    constexpr int cur = s & 1, nxt = cur ^ 1;
    if constexpr (s + 2 < NK) load(rA[cur], rB[cur], s + 2);
    mfma_step(cur, 0);
    if constexpr (s + 1 < NK) store(rA[nxt], rB[nxt], nxt);
    mfma_step(cur, 1);
    __syncthreads();
  });
  if (interior) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < 4; ++j) Ct[(long long)(16 * i + v) * ldc + 16 * j] = acc[i][j][v];
  } else {
    const int rlim = M - (row0 + wm + 4 * g), clim = N - (col0 + wn + l16);
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (16 * i + v < rlim && 16 * j < clim)
            Ct[(long long)(16 * i + v) * ldc + 16 * j] = acc[i][j][v];
  }
}

int packed_kdim(int K) {
  int nk = 1;
  while (kPkBK * nk < K) nk *= 2;
  return kPkBK * nk;
}

template <Op OP>
int launch_packed(int M, int N, int K, const float* A, long long lda, const float* B,
                  long long ldb, float* C, long long ldc, void* pa, void* pb, bool pack_a,
                  hipStream_t s) {
  typedef typename OpTraits<OP>::elem E;
  const int Kp = packed_kdim(K);
  const int tiles_m = (int)cdiv(M, kPkTile), tiles_n = (int)cdiv(N, kPkTile);
  const int Mp = tiles_m * kPkTile, Np = tiles_n * kPkTile;
  if (pack_a) {
    const long long q = (long long)Mp * (Kp / 8);
    hipLaunchKernelGGL(pack_neg_a<OP>, dim3((unsigned)cdiv(q, 256)), dim3(256), 0, s, M, K, A,
                       lda, Mp, Kp, (E*)pa);
    LP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(pack_bt<OP>, dim3((unsigned)(Kp / 64), (unsigned)(Np / 64)), dim3(256), 0, s,
                     K, N, B, ldb, Kp, (E*)pb);
  LP_LAUNCH_CHECK();
  const dim3 grid((unsigned)((long long)tiles_m * tiles_n));
  switch (Kp / kPkBK) {
#define LP_PK_CASE(NKV)                                                                        \
  case NKV:                                                                                    \
    hipLaunchKernelGGL((hgemm_update_packed<OP, NKV>), grid, dim3(512), 0, s, M, N,           \
                       (const E*)pa, (const E*)pb, C, ldc, tiles_m, tiles_n);                  \
    break;
    LP_PK_CASE(1)
    LP_PK_CASE(2)
    LP_PK_CASE(4)
    LP_PK_CASE(8)
    LP_PK_CASE(16)
#undef LP_PK_CASE
    default:
      return LP_ENOTSUP;
  }
  LP_LAUNCH_CHECK();
  return LP_OK;
}

}  // namespace

size_t gemm_lp_packed_bytes(int rows, int K) {
  if (rows <= 0 || K <= 0 || K > kPkBK * 16) return 0;
  return (size_t)cdiv(rows, kPkTile) * kPkTile * packed_kdim(K) * 2;
}

bool gemm_lp_packed_pays(int prec, int M, int N, int K) {
  return (prec == LP_BF16 || prec == LP_FP16) && K <= kPkBK * 16 &&
         cdiv(M, kPkTile) * cdiv(N, kPkTile) >= 256;
}

int launch_gemm_update_lp_packed(int prec, int M, int N, int K, const float* A, long long lda,
                                 const float* B, long long ldb, float* C, long long ldc,
                                 void* pa, void* pb, bool pack_a, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return LP_OK;
  if (K > kPkBK * 16 || (long long)kPkTile * ldc * 4 >= 0x7fffffffLL ||
      (long long)cdiv(M, kPkTile) * cdiv(N, kPkTile) > 0x7fffffffLL)
    return LP_ENOTSUP;
  if (((uintptr_t)pa | (uintptr_t)pb) & 15) return LP_ENOTSUP;
  if (prec == LP_BF16)
    return launch_packed<Op::BF16>(M, N, K, A, lda, B, ldb, C, ldc, pa, pb, pack_a, s);
  if (prec == LP_FP16)
    return launch_packed<Op::F16>(M, N, K, A, lda, B, ldb, C, ldc, pa, pb, pack_a, s);
  return LP_ENOTSUP;
}

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
  else if (prec == LP_BF16) {
    if (!launch_fast<Op::BF16>(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, s))
      hipLaunchKernelGGL(sgemm_update_kernel<Op::BF16>, grid, dim3(256), 0, s, M, N, K, A, lda,
                         B, ldb, C, ldc, tiles_m, tiles_n);
  } else if (prec == LP_FP16) {
    if (!launch_fast<Op::F16>(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, s))
      hipLaunchKernelGGL(sgemm_update_kernel<Op::F16>, grid, dim3(256), 0, s, M, N, K, A, lda, B,
                         ldb, C, ldc, tiles_m, tiles_n);
  }
  else
    return LP_ENOTSUP;
  LP_LAUNCH_CHECK();
  return LP_OK;
}

}  // namespace lp

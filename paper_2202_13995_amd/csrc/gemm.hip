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
//
// A workgroup (4 waves, two workgroups per CU) owns a 128 x 128 tile of C;
// wave w owns the 64 x 64 quadrant (w / 2, w % 2) as 4 x 4 fragments.  K
// advances in slabs of 16.  Within a slab the four MFMA k-steps take
// k = 4 q + s for lane group q = l / 16 and step s, so each lane reads its A
// values as contiguous 16-byte pairs (the summation order inside a dot product
// is free).
//
// The accumulators start at C and the A operand is negated once, when it is
// written to LDS, so the tile ends holding C - A B with one rounding per MFMA
// step and is stored without reading C again.  The C loads are issued in the
// prologue together with the first two slabs, so their latency overlaps.
//
// Interior tiles whose K is a multiple of 16 up to 512 run a fully unrolled
// slab sequence: global loads run two slabs ahead through two register sets
// (buffer loads with 32-bit offsets keep the address registers few), the next
// slab is written to LDS between the two halves of the current slab's MFMAs,
// and one barrier closes each slab.  Unrolling the K loop lets the compiler
// count outstanding loads exactly, so each LDS write waits only for its own
// slab.  Edge tiles (and other K) run the same arithmetic through a rolled loop
// with predicated loads.
//
// Tile order: hardware dispatches workgroup b to XCD b % 8.  The launcher
// numbers tiles so that each XCD receives a contiguous range of tile ids, and
// ids walk 8-row groups column by column, so tiles resident on one XCD share A
// row panels and B column panels in that XCD's L2.
#include <type_traits>

#include "common.h"

namespace lp {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int DBM = 128;
constexpr int DBN = 128;
constexpr int DBK = 16;
constexpr int DAS = DBK + 2;  // A tile row stride in LDS (doubles)
constexpr int GROUP_M = 8;
constexpr unsigned kRsrcWord3 = 0x00020000u;  // raw buffer, 32-bit data format

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

template <int I, int E>
struct StaticFor {
  template <typename F>
  __device__ __forceinline__ static void run(F&& f) {
    if constexpr (I < E) {
      f(std::integral_constant<int, I>{});
      StaticFor<I + 1, E>::run(f);
    }
  }
};

// Thread roles shared by both bodies.
struct Roles {
  int wm, wn, l16, q;  // wave quadrant and lane coordinates
  int a_k, a_r;        // A staging: k pair a_k, rows a_r + 32 p
  int b_c, b_k;        // B staging: column pair b_c, k rows b_k + 4 p
  __device__ __forceinline__ Roles() {
    // the wave index is uniform; saying so keeps buffer descriptors built from
    // it in SGPRs (no per-lane descriptor loops)
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    wm = (wave >> 1) * 64;
    wn = (wave & 1) * 64;
    l16 = lane & 15;
    q = lane >> 4;
    a_k = (tid & 7) * 2;
    a_r = tid >> 3;
    b_c = (tid & 63) * 2;
    b_k = tid >> 6;
  }
};

__device__ __forceinline__ void stage_store(double* As, double* Bs, const Roles& t, const d2* ra,
                                            const d2* rb) {
#pragma unroll
  for (int p = 0; p < 4; ++p) *(d2*)&As[(t.a_r + 32 * p) * DAS + t.a_k] = -ra[p];
#pragma unroll
  for (int p = 0; p < 4; ++p) *(d2*)&Bs[(t.b_k + 4 * p) * DBN + t.b_c] = rb[p];
}

// MFMA k-steps [ks0, ks1) of one slab held in As/Bs.
__device__ __forceinline__ void slab_mfma(d4 (&acc)[4][4], const double* As, const double* Bs,
                                          const Roles& t, int ks0, int ks1) {
  const double* as = As + (t.wm + t.l16) * DAS + 4 * t.q;
  const double* bs = Bs + (4 * t.q) * DBN + t.wn + t.l16;
#pragma unroll
  for (int ks = ks0; ks < ks1; ++ks) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = as[16 * i * DAS + ks];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = bs[ks * DBN + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// Interior tile, K = 16 * NK.  All rows, columns and k of the tile are in range.
template <int NK>
__device__ __forceinline__ void dgemm_interior(const double* __restrict__ A, long long lda,
                                               const double* __restrict__ B, long long ldb,
                                               double* __restrict__ C, long long ldc, int row0,
                                               int col0, double* As0, double* Bs0) {
  const Roles t;
  const __amdgpu_buffer_rsrc_t ra_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + (long long)row0 * lda), (short)0, 0x7fffffff, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rb_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(B + col0), (short)0, 0x7fffffff, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rc_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(C + (long long)(row0 + t.wm) * ldc + col0 + t.wn), (short)0, 0x7fffffff,
      kRsrcWord3);
  const int a_vo = (int)(((long long)t.a_r * lda + t.a_k) * 8);
  const int b_vo = (int)(((long long)t.b_k * ldb + t.b_c) * 8);
  const int c_vo = (int)(((long long)t.q * ldc + t.l16) * 8);
  const int a_so = (int)(32 * lda * 8);
  const int b_so = (int)(4 * ldb * 8);
  const int b_slab = (int)(DBK * ldb * 8);

  d2 rA[2][4], rB[2][4];
  auto load = [&](d2* ra, d2* rb, int s) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
      ra[p] = __builtin_bit_cast(
          d2, __builtin_amdgcn_raw_buffer_load_b128(ra_rsrc, a_vo + s * DBK * 8, p * a_so, 0));
#pragma unroll
    for (int p = 0; p < 4; ++p)
      rb[p] = __builtin_bit_cast(
          d2, __builtin_amdgcn_raw_buffer_load_b128(rb_rsrc, b_vo + s * b_slab, p * b_so, 0));
  };

  d4 acc[4][4];
  load(rA[0], rB[0], 0);
  if constexpr (NK > 1) load(rA[1], rB[1], 1);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j][v] = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(
                        rc_rsrc, c_vo + j * 128, (int)((long long)(16 * i + 4 * v) * ldc * 8), 0));
  stage_store(As0, Bs0, t, rA[0], rB[0]);
  __syncthreads();
  // slab s: LDS buffer s & 1 holds slab s, register set (s + 1) & 1 holds slab
  // s + 1 (possibly still in flight), register set s & 1 receives slab s + 2.
  StaticFor<0, NK>::run([&](auto S) {
    constexpr int s = decltype(S)::value;
    constexpr int cur = s & 1, nxt = cur ^ 1;
    if constexpr (s + 2 < NK) load(rA[cur], rB[cur], s + 2);
    slab_mfma(acc, As0 + cur * DBM * DAS, Bs0 + cur * DBK * DBN, t, 0, 2);
    if constexpr (s + 1 < NK)
      stage_store(As0 + nxt * DBM * DAS, Bs0 + nxt * DBK * DBN, t, rA[nxt], rB[nxt]);
    slab_mfma(acc, As0 + cur * DBM * DAS, Bs0 + cur * DBK * DBN, t, 2, 4);
    __syncthreads();
  });

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + t.wn + 16 * j + t.l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + t.wm + 16 * i + t.q + 4 * v;
        C[(long long)r * ldc + c] = acc[i][j][v];
      }
    }
}

// Any tile, any K: rolled slab loop with predicated loads, one slab of prefetch.
__device__ __forceinline__ void dgemm_edge(int M, int N, int K, const double* __restrict__ A,
                                           long long lda, const double* __restrict__ B,
                                           long long ldb, double* __restrict__ C, long long ldc,
                                           int row0, int col0, double* As0, double* Bs0) {
  const Roles t;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + t.wn + 16 * j + t.l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + t.wm + 16 * i + t.q + 4 * v;
        acc[i][j][v] = (r < M && c < N) ? C[(long long)r * ldc + c] : 0.0;
      }
    }
  d2 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = row0 + t.a_r + 32 * p;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = k0 + t.a_k + e;
        ra[p][e] = (r < M && k < K) ? A[(long long)r * lda + k] : 0.0;
      }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int k = k0 + t.b_k + 4 * p;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int c = col0 + t.b_c + e;
        rb[p][e] = (k < K && c < N) ? B[(long long)k * ldb + c] : 0.0;
      }
    }
  };
  const int nk = (K + DBK - 1) / DBK;
  load(0);
  stage_store(As0, Bs0, t, ra, rb);
  __syncthreads();
  for (int s = 0; s < nk; ++s) {
    const int cur = s & 1;
    if (s + 1 < nk) load((s + 1) * DBK);
    slab_mfma(acc, As0 + cur * DBM * DAS, Bs0 + cur * DBK * DBN, t, 0, 4);
    if (s + 1 < nk) stage_store(As0 + (cur ^ 1) * DBM * DAS, Bs0 + (cur ^ 1) * DBK * DBN, t, ra, rb);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + t.wn + 16 * j + t.l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + t.wm + 16 * i + t.q + 4 * v;
        if (r < M && c < N) C[(long long)r * ldc + c] = acc[i][j][v];
      }
    }
}

// NK > 0: interior tiles with K == 16 * NK take the unrolled body (the launcher
// guarantees 16-byte aligned A and B, even lda and ldb, and 32-bit offsets).
template <int NK>
__device__ __forceinline__ void dgemm_update_body(int M, int N, int K, const double* A,
                                                  long long lda, const double* B, long long ldb,
                                                  double* C, long long ldc, int tiles_m,
                                                  int tiles_n) {
  __shared__ __align__(16) double As[2 * DBM * DAS];
  __shared__ __align__(16) double Bs[2 * DBK * DBN];
  int tm, tn;
  tile_coords(tiles_m, tiles_n, tm, tn);
  const int row0 = tm * DBM, col0 = tn * DBN;
  if constexpr (NK > 0) {
    if (row0 + DBM <= M && col0 + DBN <= N) {
      dgemm_interior<NK>(A, lda, B, ldb, C, ldc, row0, col0, As, Bs);
      return;
    }
  }
  dgemm_edge(M, N, K, A, lda, B, ldb, C, ldc, row0, col0, As, Bs);
}

// The trailing-matrix update and the updates inside a panel run the same body
// under two names so that traces separate them.
template <int NK>
__global__ __launch_bounds__(256, 2) void dgemm_trailing_update(
    int M, int N, int K, const double* __restrict__ A, long long lda,
    const double* __restrict__ B, long long ldb, double* __restrict__ C, long long ldc,
    int tiles_m, int tiles_n) {
  dgemm_update_body<NK>(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
}

template <int NK>
__global__ __launch_bounds__(256, 2) void dgemm_panel_update(
    int M, int N, int K, const double* __restrict__ A, long long lda,
    const double* __restrict__ B, long long ldb, double* __restrict__ C, long long ldc,
    int tiles_m, int tiles_n) {
  dgemm_update_body<NK>(M, N, K, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
}

template <int NK>
void launch_nk(int kind, unsigned T, int M, int N, int K, const double* A, long long lda,
               const double* B, long long ldb, double* C, long long ldc, int tiles_m,
               int tiles_n, hipStream_t s) {
  if (kind == kGemmPanel)
    hipLaunchKernelGGL((dgemm_panel_update<NK>), dim3(T), dim3(256), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((dgemm_trailing_update<NK>), dim3(T), dim3(256), 0, s, M, N, K, A, lda, B,
                       ldb, C, ldc, tiles_m, tiles_n);
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
    const double* a = (const double*)A;
    const double* b = (const double*)B;
    double* c = (double*)C;
    // the unrolled interior body uses 16-byte loads and 32-bit buffer offsets
    const bool vec_ok = ((((uintptr_t)a | (uintptr_t)b) & 15) == 0) && ((lda | ldb) & 1) == 0 &&
                        (long long)DBM * lda * 8 < 0x7fffffffLL &&
                        (long long)K * ldb * 8 < 0x7fffffffLL &&
                        (long long)64 * ldc * 8 < 0x7fffffffLL;
    const int nk = (vec_ok && K % DBK == 0) ? K / DBK : 0;
    const unsigned grid = (unsigned)T;
    switch (nk) {
      case 2: launch_nk<2>(kind, grid, M, N, K, a, lda, b, ldb, c, ldc, tiles_m, tiles_n, s); break;
      case 4: launch_nk<4>(kind, grid, M, N, K, a, lda, b, ldb, c, ldc, tiles_m, tiles_n, s); break;
      case 8: launch_nk<8>(kind, grid, M, N, K, a, lda, b, ldb, c, ldc, tiles_m, tiles_n, s); break;
      case 16: launch_nk<16>(kind, grid, M, N, K, a, lda, b, ldb, c, ldc, tiles_m, tiles_n, s); break;
      case 32: launch_nk<32>(kind, grid, M, N, K, a, lda, b, ldb, c, ldc, tiles_m, tiles_n, s); break;
      default: launch_nk<0>(kind, grid, M, N, K, a, lda, b, ldb, c, ldc, tiles_m, tiles_n, s); break;
    }
    LP_LAUNCH_CHECK();
    return LP_OK;
  }
  return launch_gemm_update_lp(prec, M, N, K, (const float*)A, lda, (const float*)B, ldb,
                               (float*)C, ldc, s);
}

}  // namespace lp

// Triangular solves with the LU factors and the benchmark's residual check.
//
// Paper, section "High Performance Linpack": after A = L U, solve L y = b and
// then U x = y.  (The paper runs this part on CPUs; here it stays on the GPU.)
// Right-hand sides are row-major n x nrhs.  The interchanges recorded by the
// factorization are applied to B first, in chunks of up to 1024 swaps with the
// same parallel swap plan the factorization uses.  Each triangle is then
// solved block by block (128 rows): one wave per right-hand side solves the
// diagonal block with the block held in LDS, and a grid of threads (one per
// row) subtracts that block's contribution from all later rows.
#include <cmath>

#include "common.h"
#include "device.h"
#include "swap_plan.h"

namespace lp {

namespace {

constexpr int kTB = 128;       // triangular block
constexpr int kRhsChunk = 8;   // right-hand sides per pass

// ---------------------------------------------------------- B := P B
template <typename T>
__global__ __launch_bounds__(1024) void permute_rows_kernel(int n, const int32_t* __restrict__ ipiv,
                                                            T* __restrict__ B, long long ldb,
                                                            int nrhs,
                                                            const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  __shared__ int piv[1024];
  __shared__ int nxt[1024];
  __shared__ int Bv[1024];
  __shared__ int flag[2048];
  __shared__ int dst[2048];
  __shared__ int src[2048];
  __shared__ int nent;
  constexpr int Q = 16;  // values per thread: 2048 entries x 8 columns / 1024 threads
  for (int k1 = 0; k1 < n; k1 += 1024) {
    const int k2 = min(n, k1 + 1024);
    if ((int)threadIdx.x < k2 - k1) piv[threadIdx.x] = ipiv[k1 + threadIdx.x];
    __syncthreads();
    build_swap_plan(piv, k1, k2, nxt, Bv, nullptr, flag, dst, src, &nent);
    __syncthreads();
    const int ne = nent;
    for (int c0 = 0; c0 < nrhs; c0 += kRhsChunk) {
      const int cw = min(kRhsChunk, nrhs - c0);
      T v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + 1024 * q;
        const int ent = e >> 3;
        const int col = e & 7;
        if (ent < ne && col < cw) v[q] = B[(long long)src[ent] * ldb + c0 + col];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + 1024 * q;
        const int ent = e >> 3;
        const int col = e & 7;
        if (ent < ne && col < cw) B[(long long)dst[ent] * ldb + c0 + col] = v[q];
      }
      __syncthreads();
    }
  }
}

// The same B := P B in two launches: the net permutation of every chunk of
// 1024 interchanges is built at once (one workgroup per chunk: a chunk's plan
// depends only on its own entries of ipiv), then one workgroup applies the
// chunks' gathers to B in order.  Plans: per chunk one count and up to 2048
// (destination, source) row pairs.
constexpr int kPlanChunk = 1024;
constexpr int kPlanInts = 1 + 4 * kPlanChunk;

__global__ __launch_bounds__(1024) void solve_plans_kernel(int n, const int32_t* __restrict__ ipiv,
                                                           int* __restrict__ plans,
                                                           const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  __shared__ int piv[kPlanChunk];
  __shared__ int nxt[kPlanChunk];
  __shared__ int Bv[kPlanChunk];
  __shared__ int flag[2 * kPlanChunk];
  __shared__ int dst[2 * kPlanChunk];
  __shared__ int src[2 * kPlanChunk];
  __shared__ int nent;
  const int k1 = blockIdx.x * kPlanChunk;
  const int k2 = min(n, k1 + kPlanChunk);
  if ((int)threadIdx.x < k2 - k1) piv[threadIdx.x] = ipiv[k1 + threadIdx.x];
  __syncthreads();
  build_swap_plan(piv, k1, k2, nxt, Bv, nullptr, flag, dst, src, &nent);
  __syncthreads();
  int* out = plans + (size_t)blockIdx.x * kPlanInts;
  const int ne = nent;
  if (threadIdx.x == 0) out[0] = ne;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    out[1 + e] = dst[e];
    out[1 + 2 * kPlanChunk + e] = src[e];
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void apply_plans_kernel(int nchunks, const int* __restrict__ plans,
                                                           T* __restrict__ B, long long ldb,
                                                           int nrhs,
                                                           const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  constexpr int Q = 16;  // 2048 entries x 8 columns / 1024 threads
  for (int ch = 0; ch < nchunks; ++ch) {
    const int* pl = plans + (size_t)ch * kPlanInts;
    const int ne = pl[0];
    for (int c0 = 0; c0 < nrhs; c0 += kRhsChunk) {
      const int cw = min(kRhsChunk, nrhs - c0);
      T v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + 1024 * q;
        const int ent = e >> 3;
        const int col = e & 7;
        if (ent < ne && col < cw) v[q] = B[(long long)pl[1 + 2 * kPlanChunk + ent] * ldb + c0 + col];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + 1024 * q;
        const int ent = e >> 3;
        const int col = e & 7;
        if (ent < ne && col < cw) B[(long long)pl[1 + ent] * ldb + c0 + col] = v[q];
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------- diagonal-block solves
// lower == true: unit lower forward substitution on rows [r0, r0 + bs).
// lower == false: upper back substitution (divides by the diagonal).
// One wave per right-hand side of a chunk; lane l holds rows l and l + 64 of
// the block.  Step j takes row j's value from the lane that holds it (a
// register read across lanes, no barrier) and every lane updates its rows with
// the block's factors from LDS.
template <typename T>
__device__ __forceinline__ T lane_value(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned)lo);
  }
}

template <typename T, bool lower>
__global__ __launch_bounds__(64 * kRhsChunk) void trsv_diag_kernel(
    int n, int r0, const T* __restrict__ LU, long long lda, T* __restrict__ B, long long ldb,
    int nrhs, const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  __shared__ T Ls[kTB][kTB + 1];
  const int bs = min(kTB, n - r0);
  // the block into LDS with 16 loads in flight per thread (a loop that stores
  // each load before issuing the next pays one memory latency per element)
  constexpr int kB = 16;
  const int nel = bs * bs;
  for (int e0 = threadIdx.x; e0 < nel; e0 += kB * (int)blockDim.x) {
    T v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = min(e0 + u * (int)blockDim.x, nel - 1);
      const int i = e / bs;
      v[u] = LU[(long long)(r0 + i) * lda + r0 + (e - i * bs)];
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      if (e < nel) {
        const int i = e / bs;
        Ls[i][e - i * bs] = v[u];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i0 = lane, i1 = lane + 64;
  // rows past the block read a valid LDS row; their values are never stored
  const int l0 = min(i0, bs - 1), l1 = min(i1, bs - 1);
  for (int c = w; c < nrhs; c += kRhsChunk) {
    T b0 = (i0 < bs) ? B[(long long)(r0 + i0) * ldb + c] : T(0);
    T b1 = (i1 < bs) ? B[(long long)(r0 + i1) * ldb + c] : T(0);
    // factors are read unconditionally and the row conditions select
    // afterwards; full blocks unroll the steps so that the LDS reads of later
    // steps are issued ahead of the chain through the broadcast values
    auto fwd = [&](int j) {
      const T a0 = Ls[l0][j], a1 = Ls[l1][j];
      const T yj = lane_value(j < 64 ? b0 : b1, j & 63);
      const T n0 = b0 - a0 * yj, n1 = b1 - a1 * yj;
      b0 = (i0 > j) ? n0 : b0;
      b1 = (i1 > j) ? n1 : b1;
    };
    auto bwd = [&](int j) {
      const T a0 = Ls[l0][j], a1 = Ls[l1][j], d = Ls[j][j];
      const T yj = lane_value(j < 64 ? b0 : b1, j & 63) / d;
      const T n0 = b0 - a0 * yj, n1 = b1 - a1 * yj;
      b0 = (i0 == j) ? yj : ((i0 < j) ? n0 : b0);
      b1 = (i1 == j) ? yj : ((i1 < j) ? n1 : b1);
    };
    if (lower) {
      if (bs == kTB) {
#pragma unroll
        for (int j = 0; j < kTB; ++j) fwd(j);
      } else {
        for (int j = 0; j < bs; ++j) fwd(j);
      }
    } else {
      if (bs == kTB) {
#pragma unroll
        for (int j = kTB - 1; j >= 0; --j) bwd(j);
      } else {
        for (int j = bs - 1; j >= 0; --j) bwd(j);
      }
    }
    if (i0 < bs) B[(long long)(r0 + i0) * ldb + c] = b0;
    if (i1 < bs) B[(long long)(r0 + i1) * ldb + c] = b1;
  }
}

// rows [rb, re) of B -= LU[rows, r0 : r0 + bs] * B[r0 : r0 + bs, :]; with VEC
// each thread reads its row of the factors 16 bytes at a time (bs a multiple
// of the vector width, rows 16-byte aligned)
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void trsv_update_kernel(int rb, int re, int r0, int bs,
                                                          const T* __restrict__ LU, long long lda,
                                                          T* __restrict__ B, long long ldb,
                                                          int nrhs,
                                                          const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  __shared__ T ys[kTB][kRhsChunk];
  constexpr int E = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(E)));
  const int i = rb + blockIdx.x * blockDim.x + threadIdx.x;
  for (int c0 = 0; c0 < nrhs; c0 += kRhsChunk) {
    const int cw = min(kRhsChunk, nrhs - c0);
    {
      // kTB * kRhsChunk / 256 = 4 entries per thread, all loads first
      constexpr int kY = kTB * kRhsChunk / 256;
      T v[kY];
#pragma unroll
      for (int u = 0; u < kY; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int k = min(e >> 3, bs - 1), c = min(e & 7, cw - 1);
        v[u] = B[(long long)(r0 + k) * ldb + c0 + c];
      }
#pragma unroll
      for (int u = 0; u < kY; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int k = e >> 3, c = e & 7;
        if (k < bs) ys[k][c] = (c < cw) ? v[u] : T(0);
      }
    }
    __syncthreads();
    if (i < re) {
      T acc[kRhsChunk];
#pragma unroll
      for (int c = 0; c < kRhsChunk; ++c) acc[c] = T(0);
      const T* row = LU + (long long)i * lda + r0;
      if constexpr (VEC) {
        for (int k0 = 0; k0 < bs; k0 += 4 * E) {
          vec_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            v[u] = (k0 + u * E < bs) ? *reinterpret_cast<const vec_t*>(row + k0 + u * E)
                                     : vec_t(T(0));
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (k0 + u * E >= bs) break;  // the same for every thread
#pragma unroll
            for (int e = 0; e < E; ++e) {
              const int k = k0 + u * E + e;
#pragma unroll
              for (int c = 0; c < kRhsChunk; ++c) acc[c] += v[u][e] * ys[k][c];
            }
          }
        }
      } else {
        for (int k = 0; k < bs; ++k) {
          const T l = row[k];
#pragma unroll
          for (int c = 0; c < kRhsChunk; ++c) acc[c] += l * ys[k][c];
        }
      }
      for (int c = 0; c < cw; ++c) B[(long long)i * ldb + c0 + c] -= acc[c];
    }
    __syncthreads();
  }
}

// ------------------------------------------- one launch per triangle
// The blocked substitution as one persistent launch.  Workgroups take block
// rows in the order they start (an atomic ticket): forward, block 0 first;
// backward, the last block first.  The workgroup of block row I keeps the
// rows' right-hand sides in registers and walks the off-diagonal tiles in the
// order their solved blocks appear, subtracting L_IJ x_J (U_IJ x_J) with its
// threads split over rows and column quarters; each tile's factors are loaded
// before the wait for x_J, so the stream of factors overlaps the dependency
// chain.  It then solves its diagonal block (held in LDS, loaded at the start)
// and publishes x_I twice: into B (the result) and as tagged 64-bit words
// (value bits + block tag, a double as two words) that other workgroups poll
// with coherent loads until every word carries the tag -- no fence and no
// flag-before-data ordering is needed.  A workgroup only ever waits for
// blocks with smaller tickets, which have already started, so the launch
// cannot deadlock whatever the residency; every wait is bounded in time
// (timeout: the launch drains and reports through the status word).
constexpr int kPT = 512;  // threads per persistent workgroup: 128 rows x 4 column quarters

size_t trsv_rec_words(int n, int wpv) { return (size_t)cdiv(n, kTB) * kTB * kRhsChunk * wpv; }

// TF: storage of the factors; T: the right-hand sides and the arithmetic
// (binary32 factors can be applied in binary64, as the refinement's
// preconditioner does).
template <typename TF, typename T, bool lower, bool VEC>
__global__ __launch_bounds__(kPT) void trsv_persistent_kernel(
    int n, const TF* __restrict__ LU, long long lda, T* __restrict__ B, long long ldb, int c0,
    int cw, unsigned long long* __restrict__ rec, unsigned* __restrict__ ctl,
    const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  constexpr int WPV = (int)(sizeof(T) / 4);  // tagged words per value
  constexpr int QW = kTB / 4;                // columns per quarter
  __shared__ T Ld[kTB][kTB + 1];             // the diagonal block
  __shared__ T xs[kTB][kRhsChunk];           // x_J of the tile being applied
  __shared__ T red[kTB][kRhsChunk];          // partial sums of the column quarters
  __shared__ int s_blk, s_to;
  const int nblk = (int)cdiv(n, kTB);
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_blk = (int)__hip_atomic_fetch_add(&ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_to = 0;
  }
  __syncthreads();
  const int tk = s_blk;
  if (tk >= nblk) return;
  const int I = lower ? tk : nblk - 1 - tk;
  const int r0 = I * kTB;
  const int bs = min(kTB, n - r0);
  const int row = tid & (kTB - 1);
  const int q = tid >> 7;  // column quarter
  const bool rowok = row < bs;
  const long long arow = (long long)(r0 + (rowok ? row : 0)) * lda;

  // the diagonal block into LDS, all of a thread's loads in flight at once
  // (its wait overlaps the first tiles)
  {
    constexpr int kD = kTB * kTB / kPT;
    T v[kD];
#pragma unroll
    for (int u = 0; u < kD; ++u) {
      const int e = tid + kPT * u;
      const int i = e >> 7, j = e & (kTB - 1);
      const bool ok = i < bs && j < bs;
      const TF a = LU[(long long)(r0 + (ok ? i : 0)) * lda + r0 + (ok ? j : 0)];
      v[u] = ok ? (T)a : T(0);
    }
#pragma unroll
    for (int u = 0; u < kD; ++u) {
      const int e = tid + kPT * u;
      Ld[e >> 7][e & (kTB - 1)] = v[u];
    }
  }
  for (int e = tid; e < kTB * kRhsChunk; e += kPT) xs[e >> 3][e & 7] = T(0);
  T acc[kRhsChunk];
#pragma unroll
  for (int c = 0; c < kRhsChunk; ++c)
    acc[c] = (q == 0 && rowok && c < cw) ? B[(long long)(r0 + row) * ldb + c0 + c] : T(0);

  // the factors of one tile quarter: row r0 + row, columns cj .. cj + QW
  auto load_tile = [&](int J, T* f) {
    const int cj = J * kTB + q * QW;
    if constexpr (VEC) {
      constexpr int E = 16 / (int)sizeof(TF);
      typedef TF vec_t __attribute__((ext_vector_type(E)));
#pragma unroll
      for (int u = 0; u < QW / E; ++u) {
        const bool ok = cj + u * E < n;  // n is a multiple of E on this path
        const vec_t v = *reinterpret_cast<const vec_t*>(LU + arow + (ok ? cj + u * E : 0));
#pragma unroll
        for (int e = 0; e < E; ++e) f[u * E + e] = ok ? (T)v[e] : T(0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < QW; ++k) {
        const bool ok = cj + k < n;
        const TF v = LU[arow + (ok ? cj + k : 0)];
        f[k] = ok ? (T)v : T(0);
      }
    }
  };
  // x_J from its tagged words into xs
  auto fetch_x = [&](int J) -> bool {
    const unsigned tag = (unsigned)(J + 1);
    const unsigned long long* rj = rec + (size_t)J * kTB * kRhsChunk * WPV;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      int bad = 0;
      // only the cw right-hand sides of this pass (the other slots stay zero)
      for (int e = tid; e < kTB * cw; e += kPT) {
        const int k = e / cw, c = e - k * cw;
        const int ee = k * kRhsChunk + c;
        if constexpr (WPV == 1) {
          const unsigned long long w = xload(&rj[ee]);
          bad |= (unsigned)(w >> 32) != tag;
          xs[k][c] = __builtin_bit_cast(T, (unsigned)w);
        } else {
          const unsigned long long w0 = xload(&rj[2 * ee]), w1 = xload(&rj[2 * ee + 1]);
          bad |= ((unsigned)(w0 >> 32) != tag) | ((unsigned)(w1 >> 32) != tag);
          xs[k][c] = __builtin_bit_cast(
              T, ((unsigned long long)(unsigned)w1 << 32) | (unsigned long long)(unsigned)w0);
        }
      }
      if (!__syncthreads_or(bad)) return true;
      if (tid == 0 && __builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeoutTicks) s_to = 1;
      __syncthreads();
      if (s_to) return false;
      __builtin_amdgcn_s_sleep(1);
    }
  };

  const int nt = lower ? I : nblk - 1 - I;  // off-diagonal tiles of this block row
  T f[QW], g[QW];
  if (nt > 0) load_tile(lower ? 0 : nblk - 1, f);
  for (int t = 0; t < nt; ++t) {
    const int J = lower ? t : nblk - 1 - t;
    if (t + 1 < nt) load_tile(lower ? t + 1 : nblk - 2 - t, g);
    if (!fetch_x(J)) {
      if (tid == 0) xstore(&ctl[1], 1u);
      return;
    }
#pragma unroll
    for (int k = 0; k < QW; ++k) {
#pragma unroll
      for (int c = 0; c < kRhsChunk; ++c) acc[c] -= f[k] * xs[q * QW + k][c];
    }
    __syncthreads();  // xs is rewritten by the next fetch
#pragma unroll
    for (int k = 0; k < QW; ++k) f[k] = g[k];
  }
  // the column quarters' sums, in a fixed order (deterministic)
  for (int qq = 1; qq < 4; ++qq) {
    if (q == qq) {
#pragma unroll
      for (int c = 0; c < kRhsChunk; ++c) red[row][c] = acc[c];
    }
    __syncthreads();
    if (q == 0) {
#pragma unroll
      for (int c = 0; c < kRhsChunk; ++c) acc[c] += red[row][c];
    }
    __syncthreads();
  }
  if (q == 0) {
#pragma unroll
    for (int c = 0; c < kRhsChunk; ++c) red[row][c] = acc[c];
  }
  __syncthreads();

  // the diagonal block: one wave per right-hand side, lane l holds rows l and
  // l + 64 (as in trsv_diag_kernel)
  const int lane = tid & 63;
  const int w = tid >> 6;
  if (w < cw) {
    const int i0 = lane, i1 = lane + 64;
    const int l0 = min(i0, bs - 1), l1 = min(i1, bs - 1);
    T b0 = red[i0][w], b1 = red[i1][w];
    auto fwd = [&](int j) {
      const T a0 = Ld[l0][j], a1 = Ld[l1][j];
      const T yj = lane_value(j < 64 ? b0 : b1, j & 63);
      const T n0 = b0 - a0 * yj, n1 = b1 - a1 * yj;
      b0 = (i0 > j) ? n0 : b0;
      b1 = (i1 > j) ? n1 : b1;
    };
    auto bwd = [&](int j) {
      const T a0 = Ld[l0][j], a1 = Ld[l1][j], d = Ld[j][j];
      const T yj = lane_value(j < 64 ? b0 : b1, j & 63) / d;
      const T n0 = b0 - a0 * yj, n1 = b1 - a1 * yj;
      b0 = (i0 == j) ? yj : ((i0 < j) ? n0 : b0);
      b1 = (i1 == j) ? yj : ((i1 < j) ? n1 : b1);
    };
    if (lower) {
      if (bs == kTB) {
#pragma unroll
        for (int j = 0; j < kTB; ++j) fwd(j);
      } else {
        for (int j = 0; j < bs; ++j) fwd(j);
      }
    } else {
      if (bs == kTB) {
#pragma unroll
        for (int j = kTB - 1; j >= 0; --j) bwd(j);
      } else {
        for (int j = bs - 1; j >= 0; --j) bwd(j);
      }
    }
    red[i0][w] = b0;
    red[i1][w] = b1;
  }
  __syncthreads();
  // publish: B (the result) and the tagged words (zeros for missing rows or
  // right-hand sides, so readers never wait on them)
  const unsigned tag = (unsigned)(I + 1);
  unsigned long long* ri = rec + (size_t)I * kTB * kRhsChunk * WPV;
  for (int e = tid; e < kTB * cw; e += kPT) {
    const int k = e / cw, c = e - k * cw;
    const int ee = k * kRhsChunk + c;
    const bool ok = k < bs;
    const T v = ok ? red[k][c] : T(0);
    if (ok) B[(long long)(r0 + k) * ldb + c0 + c] = v;
    if constexpr (WPV == 1) {
      xstore(&ri[ee], ((unsigned long long)tag << 32) | __builtin_bit_cast(unsigned, v));
    } else {
      const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
      xstore(&ri[2 * ee], ((unsigned long long)tag << 32) | (b & 0xffffffffull));
      xstore(&ri[2 * ee + 1], ((unsigned long long)tag << 32) | (b >> 32));
    }
  }
}

__global__ void trsv_status_kernel(const unsigned* __restrict__ ctl, int32_t* __restrict__ st) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && ctl[1] != 0u && *st == 0)
    *st = LP_INFO_BARRIER_TIMEOUT;
}

// ------------------------------------------------------------- residual
// One workgroup per row: sum_j |a_ij| and sum_j a_ij x_jc, then
// |sum - b_ic|; the maxima over rows are combined with 64-bit atomic max on
// the bit patterns (non-negative doubles order like their bits, and a NaN,
// sign cleared, compares above +inf, so it propagates).  The reductions run
// in a fixed order, so the result is deterministic.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(fabs(v)));
}

__global__ __launch_bounds__(256) void residual_rows_kernel(int n, const double* __restrict__ A,
                                                            long long lda,
                                                            const double* __restrict__ X,
                                                            long long ldx,
                                                            const double* __restrict__ B,
                                                            long long ldb, int nrhs, int c0,
                                                            int with_anorm,
                                                            unsigned long long* __restrict__ tmp,
                                                            double* __restrict__ Rv,
                                                            long long ldr) {
  __shared__ double red[4][kRhsChunk + 1];
  const int i = blockIdx.x;
  const int cw = min(kRhsChunk, nrhs - c0);
  double s[kRhsChunk + 1];
#pragma unroll
  for (int c = 0; c <= kRhsChunk; ++c) s[c] = 0.0;
  const double* row = A + (long long)i * lda;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double a = row[j];
    s[kRhsChunk] += fabs(a);
#pragma unroll
    for (int c = 0; c < kRhsChunk; ++c)
      if (c < cw) s[c] += a * X[(long long)j * ldx + c0 + c];
  }
#pragma unroll
  for (int c = 0; c <= kRhsChunk; ++c) {
    double v = s[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    s[c] = v;
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c <= kRhsChunk; ++c) red[threadIdx.x >> 6][c] = s[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (with_anorm) {
      const double an = ((red[0][kRhsChunk] + red[1][kRhsChunk]) + red[2][kRhsChunk]) +
                        red[3][kRhsChunk];
      atomic_max_nonneg(&tmp[0], an);
    }
    for (int c = 0; c < cw; ++c) {
      const double ax = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      const double r = ax - B[(long long)i * ldb + c0 + c];
      if (Rv != nullptr) Rv[(long long)i * ldr + c0 + c] = -r;
      atomic_max_nonneg(&tmp[1 + c0 + c], r);
      atomic_max_nonneg(&tmp[1 + nrhs + c0 + c], X[(long long)i * ldx + c0 + c]);
      atomic_max_nonneg(&tmp[1 + 2 * nrhs + c0 + c], B[(long long)i * ldb + c0 + c]);
    }
  }
}

__global__ void residual_finalize_kernel(int n, int nrhs, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long* tmp = reinterpret_cast<unsigned long long*>(out);
  const double anorm = __longlong_as_double((long long)tmp[0]);
  // read every temporary before overwriting (they share the array)
  double vals[3 * 64];
  for (int c0 = 0; c0 < nrhs; c0 += 64) {
    const int cw = min(64, nrhs - c0);
    for (int c = 0; c < cw; ++c) {
      vals[3 * c + 0] = __longlong_as_double((long long)tmp[1 + c0 + c]);
      vals[3 * c + 1] = __longlong_as_double((long long)tmp[1 + nrhs + c0 + c]);
      vals[3 * c + 2] = __longlong_as_double((long long)tmp[1 + 2 * nrhs + c0 + c]);
    }
    if (c0 + 64 < nrhs) return;  // launcher never asks for more than 64 at once
    for (int c = 0; c < cw; ++c) {
      const double rn = vals[3 * c], xn = vals[3 * c + 1], bn = vals[3 * c + 2];
      const double denom = 0x1.0p-53 * (anorm * xn + bn) * (double)n;
      double* o = out + 5 * (c0 + c);
      o[0] = rn / denom;
      o[1] = rn;
      o[2] = anorm;
      o[3] = xn;
      o[4] = bn;
    }
  }
}

__global__ void solve_status_kernel(const int32_t* __restrict__ info, int32_t* __restrict__ st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st = (info != nullptr && *info != 0) ? 1 : 0;
}

}  // namespace

// B := A^-1 B with the factors; when *info != 0 every kernel leaves B alone.
template <typename T>
int launch_lu_solve(int n, const T* LU, long long lda, const int32_t* ipiv, const int32_t* info,
                    T* B, long long ldb, int nrhs, int32_t* status, hipStream_t s) {
  if (status != nullptr) {
    hipLaunchKernelGGL(solve_status_kernel, dim3(1), dim3(64), 0, s, info, status);
    LP_LAUNCH_CHECK();
  }
  if (n <= 0 || nrhs <= 0) return LP_OK;
  hipLaunchKernelGGL((permute_rows_kernel<T>), dim3(1), dim3(1024), 0, s, n, ipiv, B, ldb, nrhs,
                     info);
  LP_LAUNCH_CHECK();
  const int nblk = (int)cdiv(n, kTB);
  // 16-byte row reads of the factors: rows aligned (block offsets are
  // multiples of kTB, a multiple of the vector width)
  const int vw = 16 / (int)sizeof(T);
  const bool vec = ((uintptr_t)LU % 16 == 0) && ((lda * (long long)sizeof(T)) % 16 == 0);
  for (int b = 0; b < nblk; ++b) {
    const int r0 = b * kTB;
    const int bs = min(kTB, n - r0);
    hipLaunchKernelGGL((trsv_diag_kernel<T, true>), dim3(1), dim3(64 * kRhsChunk), 0, s, n, r0,
                       LU, lda, B, ldb, nrhs, info);
    LP_LAUNCH_CHECK();
    const int rb = r0 + bs;
    if (rb < n) {
      if (vec && bs % vw == 0)
        hipLaunchKernelGGL((trsv_update_kernel<T, true>), dim3((unsigned)cdiv(n - rb, 256)),
                           dim3(256), 0, s, rb, n, r0, bs, LU, lda, B, ldb, nrhs, info);
      else
        hipLaunchKernelGGL((trsv_update_kernel<T, false>), dim3((unsigned)cdiv(n - rb, 256)),
                           dim3(256), 0, s, rb, n, r0, bs, LU, lda, B, ldb, nrhs, info);
      LP_LAUNCH_CHECK();
    }
  }
  for (int b = nblk - 1; b >= 0; --b) {
    const int r0 = b * kTB;
    const int bs = min(kTB, n - r0);
    hipLaunchKernelGGL((trsv_diag_kernel<T, false>), dim3(1), dim3(64 * kRhsChunk), 0, s, n, r0,
                       LU, lda, B, ldb, nrhs, info);
    LP_LAUNCH_CHECK();
    if (r0 > 0) {
      if (vec && bs % vw == 0)
        hipLaunchKernelGGL((trsv_update_kernel<T, true>), dim3((unsigned)cdiv(r0, 256)),
                           dim3(256), 0, s, 0, r0, r0, bs, LU, lda, B, ldb, nrhs, info);
      else
        hipLaunchKernelGGL((trsv_update_kernel<T, false>), dim3((unsigned)cdiv(r0, 256)),
                           dim3(256), 0, s, 0, r0, r0, bs, LU, lda, B, ldb, nrhs, info);
      LP_LAUNCH_CHECK();
    }
  }
  return LP_OK;
}

// Workspace of the one-launch solves: the tagged words of every block's
// solution (one pass of up to kRhsChunk right-hand sides) and two control
// words per pass (ticket, timeout), both triangles.
size_t plans_bytes(int n) { return sizeof(int) * (size_t)kPlanInts * (size_t)cdiv(n, kPlanChunk); }

size_t lu_solve_workspace_bytes_t(int n, int elem_bytes) {
  if (n <= 0) return 256;
  const size_t rec = trsv_rec_words(n, elem_bytes / 4) * sizeof(unsigned long long);
  return (rec + 255) / 256 * 256 + 256 + (plans_bytes(n) + 255) / 256 * 256;
}

template <typename TF, typename T>
int launch_lu_solve_ws(int n, const TF* LU, long long lda, const int32_t* ipiv,
                       const int32_t* info, T* B, long long ldb, int nrhs, int32_t* status,
                       void* work, hipStream_t s) {
  if (status != nullptr) {
    hipLaunchKernelGGL(solve_status_kernel, dim3(1), dim3(64), 0, s, info, status);
    LP_LAUNCH_CHECK();
  }
  if (n <= 0 || nrhs <= 0) return LP_OK;
  constexpr int WPV = (int)(sizeof(T) / 4);
  unsigned long long* rec = reinterpret_cast<unsigned long long*>(work);
  const size_t rec_words = trsv_rec_words(n, WPV);
  unsigned* ctl = reinterpret_cast<unsigned*>(
      reinterpret_cast<char*>(work) + (rec_words * 8 + 255) / 256 * 256);
  int* plans = reinterpret_cast<int*>(reinterpret_cast<char*>(ctl) + 256);
  const int nchunks = (int)cdiv(n, kPlanChunk);
  hipLaunchKernelGGL(solve_plans_kernel, dim3(nchunks), dim3(1024), 0, s, n, ipiv, plans, info);
  LP_LAUNCH_CHECK();
  hipLaunchKernelGGL((apply_plans_kernel<T>), dim3(1), dim3(1024), 0, s, nchunks,
                     (const int*)plans, B, ldb, nrhs, info);
  LP_LAUNCH_CHECK();
  const int nblk = (int)cdiv(n, kTB);
  // 16-byte factor loads: rows aligned, and no vector straddling column n
  const bool vec = ((uintptr_t)LU % 16 == 0) && ((lda * (long long)sizeof(TF)) % 16 == 0) &&
                   (n % (16 / (int)sizeof(TF)) == 0);
  for (int c0 = 0; c0 < nrhs; c0 += kRhsChunk) {
    const int cw = min(kRhsChunk, nrhs - c0);
    for (int tri = 0; tri < 2; ++tri) {
      int rc = launch_zero_words(rec, rec_words * 2, s);
      if (rc != LP_OK) return rc;
      if ((rc = launch_zero_words(ctl, 2, s)) != LP_OK) return rc;
#define LP_TRSV_P(LOWER, VEC)          \
      hipLaunchKernelGGL((trsv_persistent_kernel<TF, T, LOWER, VEC>), dim3(nblk), \
                         dim3(kPT), 0, s, n, LU, lda, B, ldb, c0, cw, rec, ctl, info)
      if (tri == 0) {
        if (vec) LP_TRSV_P(true, true); else LP_TRSV_P(true, false);
      } else {
        if (vec) LP_TRSV_P(false, true); else LP_TRSV_P(false, false);
      }
#undef LP_TRSV_P
      LP_LAUNCH_CHECK();
      if (status != nullptr) {
        hipLaunchKernelGGL(trsv_status_kernel, dim3(1), dim3(64), 0, s, ctl, status);
        LP_LAUNCH_CHECK();
      }
    }
  }
  return LP_OK;
}

template int launch_lu_solve_ws<double, double>(int, const double*, long long, const int32_t*,
                                                const int32_t*, double*, long long, int, int32_t*,
                                                void*, hipStream_t);
template int launch_lu_solve_ws<float, float>(int, const float*, long long, const int32_t*,
                                              const int32_t*, float*, long long, int, int32_t*,
                                              void*, hipStream_t);
template int launch_lu_solve_ws<float, double>(int, const float*, long long, const int32_t*,
                                               const int32_t*, double*, long long, int, int32_t*,
                                               void*, hipStream_t);

template int launch_lu_solve<double>(int, const double*, long long, const int32_t*,
                                     const int32_t*, double*, long long, int, int32_t*,
                                     hipStream_t);
template int launch_lu_solve<float>(int, const float*, long long, const int32_t*, const int32_t*,
                                    float*, long long, int, int32_t*, hipStream_t);

// Rv (optional): also writes r = B - A X (n x nrhs, ld ldr).
int launch_residual(int n, const double* A, long long lda, const double* X, long long ldx,
                    const double* B, long long ldb, int nrhs, double* out, hipStream_t s,
                    double* Rv, long long ldr) {
  if (nrhs <= 0) return LP_OK;
  for (int g0 = 0; g0 < nrhs; g0 += 64) {
    const int gw = min(64, nrhs - g0);
    int rc = launch_zero_words(out + 5 * g0, (size_t)10 * gw, s);
    if (rc != LP_OK) return rc;
    if (n > 0) {
      for (int c0 = 0; c0 < gw; c0 += kRhsChunk) {
        hipLaunchKernelGGL(residual_rows_kernel, dim3(n), dim3(256), 0, s, n, A, lda, X + g0, ldx,
                           B + g0, ldb, gw, c0, c0 == 0 ? 1 : 0,
                           reinterpret_cast<unsigned long long*>(out + 5 * g0),
                           Rv == nullptr ? nullptr : Rv + g0, ldr);
        LP_LAUNCH_CHECK();
      }
    }
    hipLaunchKernelGGL(residual_finalize_kernel, dim3(1), dim3(64), 0, s, n, gw, out + 5 * g0);
    LP_LAUNCH_CHECK();
  }
  return LP_OK;
}

}  // namespace lp

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

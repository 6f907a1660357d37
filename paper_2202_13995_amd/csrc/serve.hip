// Serving: a stream of independent solves of uneven size with continuous
// batching.
//
// Not in the paper (which times one large LINPACK run); this is the request
// loop built on the same method: each request is a dense system A X = B solved
// by Gaussian elimination with partial pivoting (section "High Performance
// Linpack") and checked with the benchmark's scaled residual.
//
// Runtime (host, poll-driven): lp_server_submit queues a request; every
// lp_server_poll call (1) retires finished work, (2) admits queued requests
// first-come-first-served while their device footprint fits the free part of
// the server's memory pool, and (3) hands them to the device: requests with
// n <= small_n_max are published into a ring of descriptors in pinned host
// memory, from which a persistent batched kernel pulls them (one workgroup per
// request, a workgroup takes the next published request as soon as it is free,
// so uneven sizes balance and every request completes on its own); larger ones
// run the blocked path (lu_factor / lu_solve_ir) on a stream of their own.
// Requests arriving while others are on the GPU start as soon as memory and a
// workgroup or slot are free.  A request's arithmetic depends only on its size
// and precision, never on what else is in flight.
//
// The ring protocol: the host writes a descriptor into slot (k mod capacity),
// then advances the published count with a release store; a workgroup claims
// index k only when k is below the published count (compare-and-swap on a
// device counter), so no claim ever waits for a request that does not exist.
// It reads the descriptor with system-scope loads, solves, writes the results
// with system-scope stores and then the slot's completion word (k + 1) with a
// release store, which the host polls.  The kernel exits when the host sets
// its stop word or after a spell without requests (so every launch drains);
// the host launches it again when a request is published and it is not
// running.  Requests are published only after the work their submitter's
// stream had queued has completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "common.h"
#include "device.h"

namespace lp {
namespace {

// ------------------------------------------------------ batched device work
struct SmallReq {
  const double* A;  // caller's matrix (n x n, lda), read only
  const double* B;  // caller's right-hand sides (n x nrhs, ldb), read only
  double* X;        // caller's output (n x nrhs, ldx)
  void* W;          // this request's workspace in the pool
  long long lda, ldb, ldx;
  int n, nrhs, prec, max_iter;
  double* result;   // device: {status, info, scaled residual, iterations, fell_back}
};

constexpr int kST = 256;  // threads per request

__device__ __forceinline__ double block_max_nonneg(double v, double* red) {
  // max of non-negative values (NaN wins) over the workgroup; all threads get it
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off);
    if (o > v || o != o) v = o;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
  for (int t = 1; t < kST / 64; ++t)
    if (red[t] > m || red[t] != red[t]) m = red[t];
  return m;
}

// In-place partial-pivoting LU of the n x n matrix W (ld n) by one workgroup;
// the same pivot rule as everywhere (largest |a|, lowest row, NaN below every
// number unless on the diagonal).  Returns info.
// perm (n ints) receives the final row order: position i holds original row perm[i].
template <typename T>
__device__ int wg_getrf(int n, T* W, int32_t* ipiv, int32_t* perm, double* rk, int* ri) {
  int info = 0;
  for (int i = threadIdx.x; i < n; i += kST) perm[i] = i;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double bk = -2.0;
    int bi = 0x7fffffff;
    for (int i = k + threadIdx.x; i < n; i += kST) {
      const T v = W[(long long)i * n + k];
      const double key = (v != v) ? -1.0 : fabs((double)v);
      if (key > bk || (key == bk && i < bi)) {
        bk = key;
        bi = i;
      }
    }
    {
      unsigned long long kb = (unsigned long long)__double_as_longlong(bk);
      wave_best(kb, bi, [](unsigned long long ka, int ia, unsigned long long kc, int ic) {
        return better(__longlong_as_double((long long)ka), ia,
                      __longlong_as_double((long long)kc), ic);
      });
      bk = __longlong_as_double((long long)kb);
    }
    if ((threadIdx.x & 63) == 0) {
      rk[threadIdx.x >> 6] = bk;
      ri[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    // every thread reduces the same four wave results in the same order, so
    // all agree on the pivot; row k itself is always a candidate, so bi < n
    bk = rk[0];
    bi = ri[0];
    for (int t = 1; t < kST / 64; ++t)
      if (rk[t] > bk || (rk[t] == bk && ri[t] < bi)) {
        bk = rk[t];
        bi = ri[t];
      }
    const T dkk = W[(long long)k * n + k];
    const int p = (dkk != dkk || bi >= n) ? k : bi;
    const T piv = W[(long long)p * n + k];
    __syncthreads();  // everyone has read rk/ri, the diagonal and the pivot before any swap
    if (threadIdx.x == 0) ipiv[k] = p;
    if (piv == T(0)) {
      if (info == 0) info = k + 1;
      continue;
    }
    if (p != k) {
      for (int j = threadIdx.x; j < n; j += kST) {
        const T t = W[(long long)k * n + j];
        W[(long long)k * n + j] = W[(long long)p * n + j];
        W[(long long)p * n + j] = t;
      }
      if (threadIdx.x == 0) {
        const int t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
      __syncthreads();
    }
    for (int i = k + 1 + threadIdx.x; i < n; i += kST) W[(long long)i * n + k] /= piv;
    __syncthreads();
    // rows over groups of 32 threads, columns over the threads of a group
    for (int i = k + 1 + (int)(threadIdx.x >> 5); i < n; i += kST / 32) {
      const T l = W[(long long)i * n + k];
      for (int j = k + 1 + (int)(threadIdx.x & 31); j < n; j += 32)
        W[(long long)i * n + j] -= l * W[(long long)k * n + j];
    }
    __syncthreads();
  }
  return info;
}

// Y := U^-1 L^-1 Y with the factors (Y n x nrhs, ld ldy, already in the
// pivoted row order), one workgroup.
template <typename T, typename V>
__device__ void wg_getrs(int n, const T* W, V* Y, long long ldy, int nrhs) {
  for (int k = 0; k < n; ++k) {  // forward, unit diagonal, column-oriented
    for (long long e = threadIdx.x; e < (long long)(n - k - 1) * nrhs; e += kST) {
      const int i = k + 1 + (int)(e / nrhs);
      const int c = (int)(e % nrhs);
      Y[(long long)i * ldy + c] -= (V)W[(long long)i * n + k] * Y[(long long)k * ldy + c];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {  // backward
    if (threadIdx.x < nrhs)
      Y[(long long)k * ldy + threadIdx.x] /= (V)W[(long long)k * n + k];
    __syncthreads();
    for (long long e = threadIdx.x; e < (long long)k * nrhs; e += kST) {
      const int i = (int)(e / nrhs);
      const int c = (int)(e % nrhs);
      Y[(long long)i * ldy + c] -= (V)W[(long long)i * n + k] * Y[(long long)k * ldy + c];
    }
    __syncthreads();
  }
}

// Scaled residual max_c s_c of X against the caller's A, B; optionally writes
// r = B - A X into Rv (n x nrhs, ld nrhs).
__device__ double wg_residual(int n, const double* A, long long lda, const double* X, long long ldx,
                              const double* B, long long ldb, int nrhs, double* Rv, double* red,
                              double anorm) {
  double worst = 0.0;
  for (int c = 0; c < nrhs; ++c) {
    double rn = 0.0, xn = 0.0, bn = 0.0;
    for (int i = threadIdx.x; i < n; i += kST) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += A[(long long)i * lda + j] * X[(long long)j * ldx + c];
      const double r = s - B[(long long)i * ldb + c];
      if (Rv) Rv[(long long)i * nrhs + c] = -r;
      const double ra = fabs(r), xa = fabs(X[(long long)i * ldx + c]),
                   ba = fabs(B[(long long)i * ldb + c]);
      if (ra > rn || ra != ra) rn = ra;
      if (xa > xn || xa != xa) xn = xa;
      if (ba > bn || ba != ba) bn = ba;
    }
    rn = block_max_nonneg(rn, red);
    xn = block_max_nonneg(xn, red);
    bn = block_max_nonneg(bn, red);
    const double sc = rn / (0x1.0p-53 * (anorm * xn + bn) * (double)n);
    if (sc > worst || sc != sc) worst = sc;
  }
  return worst;
}

__device__ double wg_anorm(int n, const double* A, long long lda, double* red) {
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kST) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += fabs(A[(long long)i * lda + j]);
    if (s > m || s != s) m = s;
  }
  return block_max_nonneg(m, red);
}

// Per-request workspace layout (bytes): factors (n x n of T), ipiv, R (n x nrhs
// double), D (n x nrhs float).
__host__ __device__ inline size_t small_ws_bytes(int n, int nrhs, int prec) {
  const size_t el = (prec == LP_FP64) ? 8 : 4;
  size_t off = el * (size_t)n * n;
  off = (off + 255) & ~(size_t)255;
  off += 8 * (size_t)n;  // ipiv and perm
  off = (off + 255) & ~(size_t)255;
  if (prec != LP_FP64) {
    off += 8 * (size_t)n * nrhs;
    off = (off + 255) & ~(size_t)255;
    off += 4 * (size_t)n * nrhs;
    off = (off + 255) & ~(size_t)255;
    off += 8 * (size_t)n * n;  // binary64 copy for the fallback
    off = (off + 255) & ~(size_t)255;
  }
  return off;
}

// One request, by the whole workgroup; res[0..4] = {status, info, scaled
// residual, iterations, fell_back} (res[5]: its device time, set by the caller).
constexpr int kResWords = 6;
// Systems of at most kLdsN rows are factored and solved with their factors
// held in the workgroup's LDS (128 KB for binary64), not in global memory.
constexpr int kLdsN = 128;
constexpr size_t kRingLdsBytes = sizeof(double) * kLdsN * kLdsN;
__device__ void solve_small(const SmallReq& q, double* res, double* red, int* redi, void* lds) {
  const int n = q.n, nrhs = q.nrhs;
  char* w = (char*)q.W;
  const size_t el = (q.prec == LP_FP64) ? 8 : 4;
  size_t off = (el * (size_t)n * n + 255) & ~(size_t)255;
  int32_t* ipiv = (int32_t*)(w + off);
  int32_t* perm = ipiv + n;
  off = (off + 8 * (size_t)n + 255) & ~(size_t)255;
  double status = 0.0, iters = 0.0, fell = 0.0, sres = 0.0;
  int info = 0;
  const double anorm = wg_anorm(n, q.A, q.lda, red);
  const bool in_lds = n <= kLdsN;
  if (q.prec == LP_FP64) {
    double* W = in_lds ? (double*)lds : (double*)w;
    for (long long e = threadIdx.x; e < (long long)n * n; e += kST)
      W[e] = q.A[(e / n) * q.lda + e % n];
    __syncthreads();
    info = wg_getrf<double>(n, W, ipiv, perm, red, redi);
    for (long long e = threadIdx.x; e < (long long)n * nrhs; e += kST)
      q.X[(e / nrhs) * q.ldx + e % nrhs] = q.B[(long long)perm[e / nrhs] * q.ldb + e % nrhs];
    __syncthreads();
    if (info == 0) {
      wg_getrs<double, double>(n, W, q.X, q.ldx, nrhs);
      sres = wg_residual(n, q.A, q.lda, q.X, q.ldx, q.B, q.ldb, nrhs, nullptr, red, anorm);
    } else {
      status = 1.0;
    }
  } else {
    // binary32 factors, binary64 refinement, binary64 fallback
    float* W = in_lds ? (float*)lds : (float*)w;
    double* Rv = (double*)(w + off);
    off = (off + 8 * (size_t)n * nrhs + 255) & ~(size_t)255;
    float* D = (float*)(w + off);
    off = (off + 4 * (size_t)n * nrhs + 255) & ~(size_t)255;
    double* W64 = (double*)(w + off);
    for (long long e = threadIdx.x; e < (long long)n * n; e += kST)
      W[e] = (float)q.A[(e / n) * q.lda + e % n];
    __syncthreads();
    info = wg_getrf<float>(n, W, ipiv, perm, red, redi);
    for (long long e = threadIdx.x; e < (long long)n * nrhs; e += kST)
      D[e] = (float)q.B[(long long)perm[e / nrhs] * q.ldb + e % nrhs];
    __syncthreads();
    bool ok = false;
    if (info == 0) {
      wg_getrs<float, float>(n, W, D, nrhs, nrhs);
      for (long long e = threadIdx.x; e < (long long)n * nrhs; e += kST)
        q.X[(e / nrhs) * q.ldx + e % nrhs] = (double)D[e];
      __syncthreads();
      double h[3] = {0, 0, 0};
      int hl = 0, k = 0;
      for (;;) {
        sres = wg_residual(n, q.A, q.lda, q.X, q.ldx, q.B, q.ldb, nrhs, Rv, red, anorm);
        h[0] = h[1];
        h[1] = h[2];
        h[2] = sres;
        ++hl;
        if (sres < 16.0) {
          ok = true;
          break;
        }
        if (sres != sres || sres > 1.7e308) break;
        if (hl >= 3 && h[2] > h[1] && h[1] > h[0]) break;
        if (k >= q.max_iter) break;
        for (long long e = threadIdx.x; e < (long long)n * nrhs; e += kST)
          D[e] = (float)Rv[(long long)perm[e / nrhs] * nrhs + e % nrhs];
        __syncthreads();
        wg_getrs<float, float>(n, W, D, nrhs, nrhs);
        for (long long e = threadIdx.x; e < (long long)n * nrhs; e += kST)
          q.X[(e / nrhs) * q.ldx + e % nrhs] += (double)D[e];
        __syncthreads();
        ++k;
      }
      iters = k;
    }
    if (!ok) {
      fell = 1.0;
      for (long long e = threadIdx.x; e < (long long)n * n; e += kST)
        W64[e] = q.A[(e / n) * q.lda + e % n];
      __syncthreads();
      const int info64 = wg_getrf<double>(n, W64, ipiv, perm, red, redi);
      for (long long e = threadIdx.x; e < (long long)n * nrhs; e += kST)
        q.X[(e / nrhs) * q.ldx + e % nrhs] = q.B[(long long)perm[e / nrhs] * q.ldb + e % nrhs];
      __syncthreads();
      if (info64 == 0) {
        wg_getrs<double, double>(n, W64, q.X, q.ldx, nrhs);
        sres = wg_residual(n, q.A, q.lda, q.X, q.ldx, q.B, q.ldb, nrhs, nullptr, red, anorm);
      } else {
        status = 1.0;
        info = info64;
      }
    }
  }
  res[0] = status;
  res[1] = (double)info;
  res[2] = sres;
  res[3] = iters;
  res[4] = fell;
}

// The ring of descriptors shared with the host (pinned, device-visible).
struct RingShared {
  unsigned long long published;  // requests written so far (host, release)
  unsigned long long stop;       // host: set to make the kernel exit
};

// A workgroup leaves after 2 ms (100 MHz clock) without a request, so an idle
// server holds no compute units; between looks at the host's counter it
// sleeps about 4 us, which keeps the polling traffic over PCIe small.
constexpr unsigned long long kIdleTicks = 200000ull;

__device__ __forceinline__ unsigned long long sys_load(const unsigned long long* p) {
  return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_ACQUIRE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(kST) void ring_solve_kernel(const SmallReq* __restrict__ ring,
                                                         double* __restrict__ results,
                                                         unsigned long long* __restrict__ done,
                                                         const RingShared* __restrict__ shared,
                                                         unsigned long long* __restrict__ head,
                                                         int capacity) {
  __shared__ double red[kST / 64];
  __shared__ int redi[kST / 64];
  __shared__ long long s_job;
  __shared__ unsigned long long s_desc[(sizeof(SmallReq) + 7) / 8];
  extern __shared__ __align__(16) unsigned char ring_lds[];  // kRingLdsBytes: small factors
  for (;;) {
    if (threadIdx.x == 0) {
      long long job = -1;
      unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      for (;;) {
        unsigned long long h =
            __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long pub = sys_load(&shared->published);
        if (h < pub) {
          if (__hip_atomic_compare_exchange_strong(head, &h, h + 1, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            job = (long long)h;
            break;
          }
          continue;  // another workgroup took it: look again at once
        }
        if (sys_load(&shared->stop) != 0ull) break;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kIdleTicks) break;
        __builtin_amdgcn_s_sleep(64);
      }
      if (job >= 0) {
        // the descriptor: system-scope loads after the acquire of `published`
        const unsigned long long* src =
            reinterpret_cast<const unsigned long long*>(ring + (job % capacity));
        for (int w = 0; w < (int)((sizeof(SmallReq) + 7) / 8); ++w)
          s_desc[w] = __hip_atomic_load(const_cast<unsigned long long*>(src + w), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_SYSTEM);
      }
      s_job = job;
    }
    __syncthreads();
    const long long job = s_job;
    if (job < 0) return;
    const SmallReq q = *reinterpret_cast<const SmallReq*>(s_desc);
    double res[kResWords];
    const unsigned long long t_start = __builtin_amdgcn_s_memrealtime();
    solve_small(q, res, red, redi, ring_lds);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int slot = (int)(job % capacity);
      // the request's own device time (100 MHz clock), apart from its wait
      res[5] = (double)(__builtin_amdgcn_s_memrealtime() - t_start) * 1e-5;
      for (int k = 0; k < kResWords; ++k)
        __hip_atomic_store(&results[kResWords * slot + k], res[k], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&done[slot], (unsigned long long)job + 1ull, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ host runtime
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Block {
  size_t off, size;
};

// First-fit allocator over one device buffer.
struct Pool {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  size_t used = 0;

  void init(char* b, size_t s) {
    base = b;
    size = s;
    free_.clear();
    free_[0] = s;
    used = 0;
  }
  bool alloc(size_t want, Block* out) {
    want = align256(std::max<size_t>(want, 256));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= want) {
        out->off = it->first;
        out->size = want;
        const size_t rest = it->second - want;
        const size_t roff = it->first + want;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used += want;
        return true;
      }
    }
    return false;
  }
  void release(const Block& b) {
    used -= b.size;
    auto it = free_.emplace(b.off, b.size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace lp

struct lp_server {
  lp_server_cfg cfg;
  void* dev = nullptr;  // the pool (one allocation at creation)
  lp::Pool pool;
  uint64_t next_ticket = 1;
  struct Pending {
    uint64_t ticket;
    lp_request req;
    size_t foot;
    double t_submit;
    hipEvent_t ready;  // recorded on the submitter's stream; the request's work waits on it
  };
  std::deque<Pending> queue;
  // the batched path: a ring of descriptors in pinned host memory and the
  // persistent kernel that pulls from it
  struct Ring {
    int capacity = 0;
    lp::SmallReq* desc = nullptr;       // pinned: capacity descriptors
    double* results = nullptr;          // pinned: kResWords per slot
    unsigned long long* done = nullptr; // pinned: completion word per slot (job + 1)
    lp::RingShared* shared = nullptr;   // pinned: published count, stop word
    unsigned long long* head = nullptr; // device (in the pool): claimed count
    unsigned long long published = 0;   // host copy
    hipStream_t s = nullptr;
    hipEvent_t exited = nullptr;        // recorded after each launch of the kernel
    bool launched = false;
    struct Slot {
      bool used = false;
      unsigned long long job = 0;
      Pending member;
      lp::Block ws;
    };
    std::vector<Slot> slots;
    int in_flight = 0;
  } ring;
  struct Large {
    hipStream_t s;
    hipEvent_t start, done;         // around the request's work on s (timing)
    bool busy = false;
    bool threaded = false;          // refinement runs on a worker thread
    std::thread worker;
    std::atomic<int> finished{0};
    Pending member;
    lp::Block ws;
    lp_ir_report rep;
    int32_t* info_host = nullptr;  // pinned
    double* res_host = nullptr;    // pinned: 5 * nrhs
    size_t res_cap = 0;
    int rc = 0;
  };
  std::vector<std::unique_ptr<Large>> larges;
  std::vector<lp_result> finished;
};

namespace {

using lp::Block;

size_t request_footprint(const lp_server_cfg& cfg, const lp_request& r) {
  if (r.n <= cfg.small_n_max) return lp::align256(lp::small_ws_bytes(r.n, r.nrhs, r.prec));
  if (r.prec == LP_FP64) {
    size_t f = lp::align256(sizeof(double) * (size_t)r.n * r.n);  // factors
    f += lp::align256(lu_workspace_bytes(r.n, r.nb, LP_FP64));
    f += lp::align256(4 * (size_t)r.n) + 256 + lp::align256(sizeof(double) * 5 * r.nrhs);
    f += lp::align256(lu_solve_workspace_bytes(r.n, LP_FP64, r.nrhs));
    return f;
  }
  return lp::align256(lu_solve_ir_workspace_bytes(r.n, r.nb, r.prec, r.nrhs));
}

int validate(const lp_request* r) {
  if (r == nullptr) return -2;
  if (r->n < 1 || r->n > 131072) return -2;
  if (r->nrhs < 1 || r->nrhs > 64) return -2;
  if (r->A == nullptr || r->B == nullptr || r->X == nullptr) return -2;
  if (r->lda < r->n || r->ldb < r->nrhs || r->ldx < r->nrhs) return -2;
  if (r->prec != LP_FP64 && r->prec != LP_FP32 && r->prec != LP_BF16 && r->prec != LP_FP16)
    return -2;
  if (r->nb < 1 || r->nb > 1024) return -2;
  return 0;
}

}  // namespace

// The ring's device counter lives in the first 256 bytes of the pool.
constexpr size_t kPoolReserve = 256;

extern "C" {

int lp_server_create(const lp_server_cfg* cfg, lp_server** out) {
  if (cfg == nullptr) return -1;
  if (out == nullptr) return -2;
  if (cfg->memory_bytes < (1u << 20) || cfg->batch_slots < 1 || cfg->batch_slots > 64 ||
      cfg->large_slots < 0 || cfg->large_slots > 64 || cfg->max_batch < 1 ||
      cfg->max_batch > 4096 || cfg->small_n_max < 0 || cfg->small_n_max > 2048 ||
      cfg->batch_workgroups < 1)
    return -1;
  lp_server* sv = new (std::nothrow) lp_server();
  if (sv == nullptr) return LP_ENOSPC;
  sv->cfg = *cfg;
  hipError_t e = hipMalloc(&sv->dev, cfg->memory_bytes);
  if (e != hipSuccess) {
    delete sv;
    return LP_EHIP_BASE - (int)e;
  }
  sv->pool.init((char*)sv->dev + kPoolReserve, cfg->memory_bytes - kPoolReserve);
  lp_server::Ring& rg = sv->ring;
  rg.capacity = cfg->max_batch;
  rg.slots.resize(rg.capacity);
  rg.head = (unsigned long long*)sv->dev;
  const unsigned mf = hipHostMallocMapped | hipHostMallocCoherent;
  if (hipHostMalloc((void**)&rg.desc, sizeof(lp::SmallReq) * rg.capacity, mf) != hipSuccess ||
      hipHostMalloc((void**)&rg.results, sizeof(double) * lp::kResWords * rg.capacity, mf) !=
          hipSuccess ||
      hipHostMalloc((void**)&rg.done, sizeof(unsigned long long) * rg.capacity, mf) !=
          hipSuccess ||
      hipHostMalloc((void**)&rg.shared, sizeof(lp::RingShared), mf) != hipSuccess ||
      hipStreamCreateWithFlags(&rg.s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&rg.exited, hipEventDisableTiming) != hipSuccess) {
    lp_server_destroy(sv);
    return LP_EHIP_BASE - (int)hipErrorOutOfMemory;
  }
  std::memset(rg.done, 0, sizeof(unsigned long long) * rg.capacity);
  rg.shared->published = 0;
  rg.shared->stop = 0;
  int rc = lp::launch_zero_words(rg.head, 2, rg.s);
  if (rc == LP_OK && hipStreamSynchronize(rg.s) != hipSuccess) rc = LP_EHIP_BASE;
  if (rc != LP_OK) {
    lp_server_destroy(sv);
    return rc;
  }
  for (int i = 0; i < cfg->large_slots; ++i) sv->larges.emplace_back(new lp_server::Large());
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (hipStreamCreateWithFlags(&l.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&l.start) != hipSuccess || hipEventCreate(&l.done) != hipSuccess ||
        hipHostMalloc((void**)&l.info_host, 16, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&l.res_host, sizeof(double) * 5 * 64, hipHostMallocDefault) !=
            hipSuccess) {
      lp_server_destroy(sv);
      return LP_EHIP_BASE - (int)hipErrorOutOfMemory;
    }
    l.res_cap = 64;
  }
  *out = sv;
  return LP_OK;
}

int lp_server_destroy(lp_server* sv) {
  if (sv == nullptr) return -1;
  lp_server::Ring& rg = sv->ring;
  // stop the persistent kernel and wait for the server's own streams only
  if (rg.shared) __atomic_store_n(&rg.shared->stop, 1ull, __ATOMIC_RELEASE);
  if (rg.s) (void)hipStreamSynchronize(rg.s);
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (l.threaded && l.worker.joinable()) l.worker.join();
    if (l.s) (void)hipStreamSynchronize(l.s);
  }
  if (rg.s) (void)hipStreamDestroy(rg.s);
  if (rg.exited) (void)hipEventDestroy(rg.exited);
  for (void* h : {(void*)rg.desc, (void*)rg.results, (void*)rg.done, (void*)rg.shared})
    if (h) (void)hipHostFree(h);
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (l.s) (void)hipStreamDestroy(l.s);
    if (l.start) (void)hipEventDestroy(l.start);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.info_host) (void)hipHostFree(l.info_host);
    if (l.res_host) (void)hipHostFree(l.res_host);
  }
  for (auto& p : sv->queue) (void)hipEventDestroy(p.ready);
  for (auto& sl : rg.slots)
    if (sl.used) (void)hipEventDestroy(sl.member.ready);
  if (sv->dev) (void)hipFree(sv->dev);
  delete sv;
  return LP_OK;
}

int lp_server_submit(lp_server* sv, const lp_request* req, uint64_t* ticket, void* stream) {
  if (sv == nullptr) return -1;
  const int v = validate(req);
  if (v != 0) return v;
  if (ticket == nullptr) return -3;
  if (req->n > sv->cfg.small_n_max && sv->cfg.large_slots == 0) return LP_ENOTSUP;
  const size_t foot = request_footprint(sv->cfg, *req);
  if (foot > sv->cfg.memory_bytes - kPoolReserve) return LP_ENOSPC;  // can never fit
  lp_server::Pending p;
  LP_HIP_TRY(hipEventCreateWithFlags(&p.ready, hipEventDisableTiming));
  const hipError_t e = hipEventRecord(p.ready, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(p.ready);
    return LP_EHIP_BASE - (int)e;
  }
  p.ticket = sv->next_ticket++;
  p.req = *req;
  p.foot = foot;
  p.t_submit = lp::now_ms();
  sv->queue.push_back(p);
  *ticket = p.ticket;
  return LP_OK;
}

static void finish(lp_server* sv, const lp_server::Pending& m, int status, int info, double sres,
                   int iters, int fell, int batched, double device_ms) {
  lp_result r;
  std::memset(&r, 0, sizeof(r));
  r.device_ms = device_ms;
  r.ticket = m.ticket;
  r.status = status;
  r.info = info;
  r.scaled_residual = sres;
  r.iterations = iters;
  r.fell_back = fell;
  r.batched = batched;
  r.latency_ms = lp::now_ms() - m.t_submit;
  sv->finished.push_back(r);
  (void)hipEventDestroy(m.ready);
}

static int retire(lp_server* sv) {
  lp_server::Ring& rg = sv->ring;
  for (int i = 0; i < rg.capacity && rg.in_flight > 0; ++i) {
    lp_server::Ring::Slot& sl = rg.slots[i];
    if (!sl.used) continue;
    if (__atomic_load_n(&rg.done[i], __ATOMIC_ACQUIRE) != sl.job + 1) continue;
    const double* rr = rg.results + lp::kResWords * i;
    finish(sv, sl.member, (int)rr[0], (int)rr[1], rr[2], (int)rr[3], (int)rr[4], 1, rr[5]);
    sv->pool.release(sl.ws);
    sl.used = false;
    --rg.in_flight;
  }
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (!l.busy) continue;
    if (!l.finished.load(std::memory_order_acquire)) continue;
    l.worker.join();
    l.threaded = false;
    if (l.member.req.prec == LP_FP64) {
      const int info = (l.rc == LP_OK) ? *l.info_host : 0;
      double m = 0.0;
      for (int c = 0; c < l.member.req.nrhs; ++c) {
        const double v = l.res_host[5 * c];
        if (!(v <= m)) m = v;
      }
      float ms = -1.0f;
      if (l.rc != LP_OK || hipEventElapsedTime(&ms, l.start, l.done) != hipSuccess) ms = -1.0f;
      if (l.rc != LP_OK) m = NAN;
      finish(sv, l.member, (l.rc != LP_OK || info != 0) ? 1 : 0, info, m, 0, 0, 0, ms);
    } else {
      finish(sv, l.member, (l.rc != LP_OK || !l.rep.converged) ? 1 : 0, l.rep.info,
             l.rep.scaled_residual, l.rep.iterations, l.rep.fell_back, 0, l.rep.t_total_ms);
    }
    sv->pool.release(l.ws);
    l.busy = false;
  }
  return LP_OK;
}

// The blocked-path work of one large request runs on a worker thread with the
// slot's stream (it issues many launches, and the refinement takes host
// decisions), so the poll loop keeps admitting and publishing other work.  A
// failure is reported as a failed request (status 1), never stranded; the
// request's memory returns to the pool at retirement either way.  The
// factorizations run without look-ahead: its internal streams per solve
// would multiply the streams sharing the device's few hardware queues, where
// a kernel at the head of a queue holds up every stream behind it.
static void run_large_fp64(lp_server::Large* l, const lp_request r, char* base,
                           hipEvent_t ready) {
  hipStream_t s = l->s;
  size_t off = 0;
  double* F = (double*)(base + off);
  off += lp::align256(sizeof(double) * (size_t)r.n * r.n);
  void* fw = base + off;
  const size_t fwb = lu_workspace_bytes(r.n, r.nb, LP_FP64);
  off += lp::align256(fwb);
  int32_t* ipiv = (int32_t*)(base + off);
  off += lp::align256(4 * (size_t)r.n);
  int32_t* info = (int32_t*)(base + off);
  off += 256;
  double* out = (double*)(base + off);
  off += lp::align256(sizeof(double) * 5 * r.nrhs);
  void* sw = base + off;
  const size_t swb = lu_solve_workspace_bytes(r.n, LP_FP64, r.nrhs);
  int rc = LP_OK;
  auto hip = [&](hipError_t e) {
    if (rc == LP_OK && e != hipSuccess) rc = LP_EHIP_BASE - (int)e;
  };
  hip(hipStreamWaitEvent(s, ready, 0));
  if (rc == LP_OK) hip(hipEventRecord(l->start, s));
  if (rc == LP_OK)
    hip(hipMemcpy2DAsync(F, sizeof(double) * r.n, r.A, sizeof(double) * r.lda,
                         sizeof(double) * r.n, r.n, hipMemcpyDeviceToDevice, s));
  if (rc == LP_OK)
    hip(hipMemcpy2DAsync(r.X, sizeof(double) * r.ldx, r.B, sizeof(double) * r.ldb,
                         sizeof(double) * r.nrhs, r.n, hipMemcpyDeviceToDevice, s));
  lp_factor_opts fo;
  fo.lookahead = 0;  // no internal streams (see above)
  fo.panel_cus = 0;
  fo.panel_rows = 0;
  fo.no_pivoting = 0;
  fo.panel_split_rows = 0;
  if (rc == LP_OK)
    rc = lu_factor_ex(r.n, r.nb, LP_FP64, F, r.n, ipiv, info, fw, fwb, &fo, nullptr, s);
  if (rc == LP_OK)
    rc = lu_solve_ex(r.n, LP_FP64, F, r.n, ipiv, info, r.X, r.ldx, r.nrhs, nullptr, sw, swb, s);
  if (rc == LP_OK) rc = residual_check(r.n, r.A, r.lda, r.X, r.ldx, r.B, r.ldb, r.nrhs, out, s);
  if (rc == LP_OK) hip(hipMemcpyAsync(l->info_host, info, 4, hipMemcpyDeviceToHost, s));
  if (rc == LP_OK)
    hip(hipMemcpyAsync(l->res_host, out, sizeof(double) * 5 * r.nrhs, hipMemcpyDeviceToHost, s));
  if (rc == LP_OK) hip(hipEventRecord(l->done, s));
  // whatever was queued runs to completion before the memory can be reused
  hip(hipStreamSynchronize(s));
  l->rc = rc;
}

static int launch_large(lp_server* sv, lp_server::Large& l, const lp_server::Pending& p,
                        const Block& ws) {
  const lp_request r = p.req;
  char* base = (char*)sv->dev + kPoolReserve + ws.off;
  l.member = p;
  l.ws = ws;
  l.rc = LP_OK;
  l.finished.store(0, std::memory_order_relaxed);
  l.threaded = true;
  l.busy = true;
  lp_server::Large* lpt = &l;
  const int maxit = r.max_iter > 0 ? r.max_iter : 30;
  const size_t wsb = ws.size;
  const hipEvent_t ready = p.ready;
  l.worker = std::thread([lpt, r, base, maxit, wsb, ready]() {
    if (r.prec == LP_FP64) {
      run_large_fp64(lpt, r, base, ready);
    } else {
      lp_ir_opts o;
      o.max_iter = maxit;
      o.gmres = 1;
      o.gmres_restart = 64;
      o.gmres_max_inner = 64;
      o.gmres_tol = 1e-10;
      o.no_lookahead = 1;  // no internal streams (see run_large_fp64)
      int rc = LP_EHIP_BASE;
      if (hipStreamWaitEvent(lpt->s, ready, 0) == hipSuccess)
        rc = lu_solve_ir_ex(r.n, r.nb, r.prec, r.A, r.lda, r.B, r.ldb, r.X, r.ldx, r.nrhs, &o,
                            base, wsb, &lpt->rep, lpt->s);
      lpt->rc = rc;
    }
    lpt->finished.store(1, std::memory_order_release);
  });
  return LP_OK;
}

// Make sure the persistent batched kernel is running (it exits after a spell
// without requests).
static int ensure_ring_kernel(lp_server* sv) {
  lp_server::Ring& rg = sv->ring;
  if (rg.launched) {
    const hipError_t q = hipEventQuery(rg.exited);
    if (q == hipErrorNotReady) return LP_OK;
    if (q != hipSuccess) return LP_EHIP_BASE - (int)q;
  }
  const int wgs = std::max(1, std::min(sv->cfg.batch_workgroups, 4 * lp::num_cus()));
  hipLaunchKernelGGL(lp::ring_solve_kernel, dim3(wgs), dim3(lp::kST), lp::kRingLdsBytes, rg.s,
                     (const lp::SmallReq*)rg.desc, rg.results, rg.done,
                     (const lp::RingShared*)rg.shared, rg.head, rg.capacity);
  LP_LAUNCH_CHECK();
  LP_HIP_TRY(hipEventRecord(rg.exited, rg.s));
  rg.launched = true;
  return LP_OK;
}

// Admission: walk the queue in arrival order.  A request whose submitter's
// work is still running, or that finds no free ring slot or large-path slot,
// is skipped (later ones may pass it); one that does not fit the free memory
// stops admission, so it is not starved by later arrivals.
static int admit_and_launch(lp_server* sv) {
  lp_server::Ring& rg = sv->ring;
  bool published = false;
  auto it = sv->queue.begin();
  while (it != sv->queue.end()) {
    const lp_request& r = it->req;
    const hipError_t q = hipEventQuery(it->ready);
    if (q == hipErrorNotReady && r.n <= sv->cfg.small_n_max) {
      ++it;  // the batched kernel cannot wait on a stream: publish once A, B are ready
      continue;
    }
    if (q != hipSuccess && q != hipErrorNotReady) return LP_EHIP_BASE - (int)q;
    if (r.n > sv->cfg.small_n_max) {
      lp_server::Large* slot = nullptr;
      for (auto& l : sv->larges)
        if (!l->busy) {
          slot = l.get();
          break;
        }
      if (slot == nullptr) {
        ++it;
        continue;
      }
      Block ws;
      if (!sv->pool.alloc(it->foot, &ws)) break;  // wait for memory in arrival order
      const lp_server::Pending p = *it;
      it = sv->queue.erase(it);
      int rc = launch_large(sv, *slot, p, ws);
      if (rc != LP_OK) return rc;
      continue;
    }
    if (rg.in_flight >= rg.capacity) {
      ++it;
      continue;
    }
    const int slot = (int)(rg.published % (unsigned long long)rg.capacity);
    if (rg.slots[slot].used) {  // the oldest request in the ring is still running
      ++it;
      continue;
    }
    Block ws;
    if (!sv->pool.alloc(it->foot, &ws)) break;
    lp::SmallReq d;
    d.A = r.A;
    d.B = r.B;
    d.X = r.X;
    d.W = (char*)sv->dev + kPoolReserve + ws.off;
    d.lda = r.lda;
    d.ldb = r.ldb;
    d.ldx = r.ldx;
    d.n = r.n;
    d.nrhs = r.nrhs;
    d.prec = r.prec;
    d.max_iter = r.max_iter > 0 ? r.max_iter : 30;
    d.result = nullptr;
    rg.desc[slot] = d;
    lp_server::Ring::Slot& sl = rg.slots[slot];
    sl.used = true;
    sl.job = rg.published;
    sl.member = *it;
    sl.ws = ws;
    ++rg.in_flight;
    ++rg.published;
    __atomic_store_n(&rg.shared->published, rg.published, __ATOMIC_RELEASE);
    published = true;
    it = sv->queue.erase(it);
  }
  if (published || rg.in_flight > 0) return ensure_ring_kernel(sv);
  return LP_OK;
}

int lp_server_poll(lp_server* sv, lp_result* done, int cap, int* count) {
  if (sv == nullptr) return -1;
  if (cap < 0 || (cap > 0 && done == nullptr)) return -3;
  if (count == nullptr) return -4;
  int rc = retire(sv);
  if (rc != LP_OK) return rc;
  rc = admit_and_launch(sv);
  if (rc != LP_OK) return rc;
  const int k = std::min<int>(cap, (int)sv->finished.size());
  for (int i = 0; i < k; ++i) done[i] = sv->finished[i];
  sv->finished.erase(sv->finished.begin(), sv->finished.begin() + k);
  *count = k;
  return LP_OK;
}

int lp_server_pending(const lp_server* sv, int* queued, int* running, size_t* pool_used) {
  if (sv == nullptr) return -1;
  int run = sv->ring.in_flight;
  for (auto& l : sv->larges) run += l->busy ? 1 : 0;
  if (queued) *queued = (int)sv->queue.size();
  if (running) *running = run;
  if (pool_used) *pool_used = sv->pool.used;
  return LP_OK;
}

size_t lp_request_footprint(const lp_server_cfg* cfg, const lp_request* req) {
  if (cfg == nullptr || validate(req) != 0) return 0;
  return request_footprint(*cfg, *req);
}

}  // extern "C"

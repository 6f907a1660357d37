// Serving: a stream of independent solves of uneven size with continuous
// batching.
//
// Not in the paper (which times one large LINPACK run); this is the request
// loop built on the same method: each request is a dense system A X = B solved
// by Gaussian elimination with partial pivoting (section "High Performance
// Linpack") and checked with the benchmark's scaled residual.
//
// Runtime (host, poll-driven): lp_server_submit queues a request; every
// lp_server_poll call (1) retires finished work (event queries), (2) admits
// queued requests first-come-first-served while their device footprint fits
// the free part of the server's memory pool and a launch slot is free, and
// (3) launches: requests with n <= small_n_max go into one batched launch
// (one workgroup per request, requests pulled through an atomic counter so
// uneven sizes balance), larger ones run the blocked path (lu_factor /
// lu_solve_ir) on a stream of their own.  Several batches and large requests
// run at once on different streams, so requests arriving while others are on
// the GPU start as soon as memory and a slot are free.  A request's arithmetic
// depends only on its size and precision, never on what it is batched with.
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
    const int m = n - k - 1;
    for (long long e = threadIdx.x; e < (long long)m * m; e += kST) {
      const int i = k + 1 + (int)(e / m);
      const int j = k + 1 + (int)(e % m);
      W[(long long)i * n + j] -= W[(long long)i * n + k] * W[(long long)k * n + j];
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

__global__ __launch_bounds__(kST) void batched_solve_kernel(const SmallReq* __restrict__ reqs,
                                                            int count,
                                                            unsigned* __restrict__ next) {
  __shared__ double red[kST / 64];
  __shared__ int redi[kST / 64];
  __shared__ int s_job;
  for (;;) {
    if (threadIdx.x == 0) s_job = (int)atomicAdd(next, 1u);
    __syncthreads();
    const int job = s_job;
    __syncthreads();
    if (job >= count) return;
    const SmallReq q = reqs[job];
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
    if (q.prec == LP_FP64) {
      double* W = (double*)w;
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
      float* W = (float*)w;
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
    if (threadIdx.x == 0) {
      q.result[0] = status;
      q.result[1] = (double)info;
      q.result[2] = sres;
      q.result[3] = iters;
      q.result[4] = fell;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ host runtime
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// One batched launch's block in the pool: max_batch descriptors, the job
// counter (own 256-byte line), then 5 result doubles per request.
struct DescLayout {
  size_t counter, results, total;
};
DescLayout desc_layout(int max_batch) {
  DescLayout d;
  d.counter = align256(sizeof(SmallReq) * (size_t)max_batch);
  d.results = d.counter + 256;
  d.total = d.results + align256(sizeof(double) * 5 * (size_t)max_batch);
  return d;
}

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
  struct Batch {
    hipStream_t s;
    hipEvent_t done;
    bool busy = false;
    lp::Block desc;  // descriptors + counter + results in the pool
    std::vector<Pending> members;
    std::vector<lp::Block> ws;
    lp::SmallReq* host_desc = nullptr;  // pinned staging for descriptors
    double* host_res = nullptr;         // pinned results
  };
  std::vector<Batch> batches;
  struct Large {
    hipStream_t s;
    hipEvent_t done;
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
  sv->pool.init((char*)sv->dev, cfg->memory_bytes);
  sv->batches.resize(cfg->batch_slots);
  for (auto& b : sv->batches) {
    if (hipStreamCreateWithFlags(&b.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&b.host_desc, sizeof(lp::SmallReq) * cfg->max_batch,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b.host_res, sizeof(double) * 5 * cfg->max_batch,
                      hipHostMallocDefault) != hipSuccess) {
      lp_server_destroy(sv);
      return LP_EHIP_BASE - (int)hipErrorOutOfMemory;
    }
  }
  for (int i = 0; i < cfg->large_slots; ++i) sv->larges.emplace_back(new lp_server::Large());
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (hipStreamCreateWithFlags(&l.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess ||
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
  (void)hipDeviceSynchronize();
  for (auto& b : sv->batches) {
    if (b.s) (void)hipStreamDestroy(b.s);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.host_desc) (void)hipHostFree(b.host_desc);
    if (b.host_res) (void)hipHostFree(b.host_res);
  }
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (l.threaded && l.worker.joinable()) l.worker.join();
    if (l.s) (void)hipStreamDestroy(l.s);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.info_host) (void)hipHostFree(l.info_host);
    if (l.res_host) (void)hipHostFree(l.res_host);
  }
  for (auto& p : sv->queue) (void)hipEventDestroy(p.ready);
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
  const size_t desc_reserve = lp::desc_layout(sv->cfg.max_batch).total;
  if (foot + desc_reserve > sv->cfg.memory_bytes) return LP_ENOSPC;  // can never fit
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

static int retire(lp_server* sv) {
  for (auto& b : sv->batches) {
    if (!b.busy) continue;
    const hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return LP_EHIP_BASE - (int)q;
    const double t = lp::now_ms();
    for (size_t i = 0; i < b.members.size(); ++i) {
      lp_result r;
      std::memset(&r, 0, sizeof(r));
      r.ticket = b.members[i].ticket;
      r.status = (int)b.host_res[5 * i + 0];
      r.info = (int)b.host_res[5 * i + 1];
      r.scaled_residual = b.host_res[5 * i + 2];
      r.iterations = (int)b.host_res[5 * i + 3];
      r.fell_back = (int)b.host_res[5 * i + 4];
      r.batched = 1;
      r.latency_ms = t - b.members[i].t_submit;
      sv->finished.push_back(r);
      sv->pool.release(b.ws[i]);
      (void)hipEventDestroy(b.members[i].ready);
    }
    sv->pool.release(b.desc);
    b.members.clear();
    b.ws.clear();
    b.busy = false;
  }
  for (auto& lp_ : sv->larges) {
    lp_server::Large& l = *lp_;
    if (!l.busy) continue;
    if (l.threaded) {
      if (!l.finished.load(std::memory_order_acquire)) continue;
      l.worker.join();
      l.threaded = false;
    } else {
      const hipError_t q = hipEventQuery(l.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return LP_EHIP_BASE - (int)q;
    }
    lp_result r;
    std::memset(&r, 0, sizeof(r));
    r.ticket = l.member.ticket;
    r.latency_ms = lp::now_ms() - l.member.t_submit;
    if (l.member.req.prec == LP_FP64) {
      r.info = *l.info_host;
      r.status = (l.rc != LP_OK || r.info != 0) ? 1 : 0;
      double m = 0.0;
      for (int c = 0; c < l.member.req.nrhs; ++c) {
        const double v = l.res_host[5 * c];
        if (!(v <= m)) m = v;
      }
      r.scaled_residual = m;
    } else {
      r.info = l.rep.info;
      r.status = (l.rc != LP_OK || !l.rep.converged) ? 1 : 0;
      r.scaled_residual = l.rep.scaled_residual;
      r.iterations = l.rep.iterations;
      r.fell_back = l.rep.fell_back;
    }
    sv->finished.push_back(r);
    sv->pool.release(l.ws);
    (void)hipEventDestroy(l.member.ready);
    l.busy = false;
  }
  return LP_OK;
}

static int launch_large(lp_server* sv, lp_server::Large& l, const lp_server::Pending& p,
                        const Block& ws) {
  const lp_request& r = p.req;
  char* base = (char*)sv->dev + ws.off;
  l.member = p;
  l.ws = ws;
  l.busy = true;
  l.rc = LP_OK;
  hipStream_t s = l.s;
  LP_HIP_TRY(hipStreamWaitEvent(s, p.ready, 0));
  if (r.prec == LP_FP64) {
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
    LP_HIP_TRY(hipMemcpy2DAsync(F, sizeof(double) * r.n, r.A, sizeof(double) * r.lda,
                                sizeof(double) * r.n, r.n, hipMemcpyDeviceToDevice, s));
    LP_HIP_TRY(hipMemcpy2DAsync(r.X, sizeof(double) * r.ldx, r.B, sizeof(double) * r.ldb,
                                sizeof(double) * r.nrhs, r.n, hipMemcpyDeviceToDevice, s));
    int rc = lu_factor(r.n, r.nb, LP_FP64, F, r.n, ipiv, info, fw, fwb, s);
    if (rc == LP_OK) rc = lu_solve(r.n, LP_FP64, F, r.n, ipiv, info, r.X, r.ldx, r.nrhs, nullptr, s);
    if (rc == LP_OK)
      rc = residual_check(r.n, r.A, r.lda, r.X, r.ldx, r.B, r.ldb, r.nrhs, out, s);
    l.rc = rc;
    LP_HIP_TRY(hipMemcpyAsync(l.info_host, info, 4, hipMemcpyDeviceToHost, s));
    LP_HIP_TRY(hipMemcpyAsync(l.res_host, out, sizeof(double) * 5 * r.nrhs,
                              hipMemcpyDeviceToHost, s));
    LP_HIP_TRY(hipEventRecord(l.done, s));
  } else {
    // refinement takes host decisions (it synchronizes its own stream), so it
    // runs on a worker thread and the poll loop keeps admitting other work
    l.finished.store(0, std::memory_order_relaxed);
    l.threaded = true;
    lp_server::Large* lpt = &l;
    const int maxit = r.max_iter > 0 ? r.max_iter : 30;
    const size_t wsb = ws.size;
    l.worker = std::thread([lpt, r, base, maxit, wsb]() {
      lpt->rc = lu_solve_ir(r.n, r.nb, r.prec, r.A, r.lda, r.B, r.ldb, r.X, r.ldx, r.nrhs, maxit,
                            base, wsb, &lpt->rep, lpt->s);
      lpt->finished.store(1, std::memory_order_release);
    });
  }
  return LP_OK;
}

// Admission: walk the queue in arrival order.  A large request that has no
// free slot is skipped (small ones may pass it); one that does not fit the
// free memory stops admission, so it is not starved by later arrivals.  Small
// requests fill batches (as many batches as slots are free).
static int launch_batch(lp_server* sv, lp_server::Batch& b, std::vector<lp::SmallReq>& descs,
                        const Block& dblk) {
  char* dbase = (char*)sv->dev + dblk.off;
  const int cnt = (int)descs.size();
  const lp::DescLayout dl = lp::desc_layout(sv->cfg.max_batch);
  if (cnt < 1 || cnt > sv->cfg.max_batch || dblk.size < dl.total) return LP_ENOSPC;
  double* res_dev = (double*)(dbase + dl.results);
  unsigned* counter = (unsigned*)(dbase + dl.counter);
  for (int i = 0; i < cnt; ++i) {
    descs[i].result = res_dev + 5 * i;
    b.host_desc[i] = descs[i];
  }
  b.desc = dblk;
  b.busy = true;
  hipStream_t s = b.s;
  for (const auto& m : b.members) LP_HIP_TRY(hipStreamWaitEvent(s, m.ready, 0));
  LP_HIP_TRY(hipMemcpyAsync(dbase, b.host_desc, sizeof(lp::SmallReq) * cnt, hipMemcpyHostToDevice,
                            s));
  int rc = lp::launch_zero_words(counter, 1, s);
  if (rc != LP_OK) return rc;
  const int wgs = std::min(cnt, sv->cfg.batch_workgroups);
  hipLaunchKernelGGL(lp::batched_solve_kernel, dim3(wgs), dim3(lp::kST), 0, s,
                     (const lp::SmallReq*)dbase, cnt, counter);
  LP_LAUNCH_CHECK();
  LP_HIP_TRY(hipMemcpyAsync(b.host_res, res_dev, sizeof(double) * 5 * cnt, hipMemcpyDeviceToHost,
                            s));
  LP_HIP_TRY(hipEventRecord(b.done, s));
  return LP_OK;
}

static int admit_and_launch(lp_server* sv) {
  const size_t desc_bytes = lp::desc_layout(sv->cfg.max_batch).total;
  lp_server::Batch* batch = nullptr;
  std::vector<lp::SmallReq> descs;
  Block dblk{0, 0};
  auto flush = [&]() -> int {
    int rc = LP_OK;
    if (batch != nullptr) {
      if (!descs.empty())
        rc = launch_batch(sv, *batch, descs, dblk);
      else
        sv->pool.release(dblk);
    }
    batch = nullptr;
    descs.clear();
    return rc;
  };
  auto it = sv->queue.begin();
  while (it != sv->queue.end()) {
    const lp_request& r = it->req;
    if (r.n > sv->cfg.small_n_max) {
      lp_server::Large* slot = nullptr;
      for (auto& l : sv->larges)
        if (!l->busy) {
          slot = l.get();
          break;
        }
      if (slot == nullptr) {
        ++it;  // no slot: later small requests may go first
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
    if (batch != nullptr && (int)batch->members.size() >= sv->cfg.max_batch) {
      int rc = flush();
      if (rc != LP_OK) return rc;
    }
    if (batch == nullptr) {
      for (auto& b : sv->batches)
        if (!b.busy) {
          batch = &b;
          break;
        }
      if (batch == nullptr) break;  // every batch slot is busy
      if (!sv->pool.alloc(desc_bytes, &dblk)) {
        batch = nullptr;
        break;
      }
    }
    Block ws;
    if (!sv->pool.alloc(it->foot, &ws)) break;
    lp::SmallReq q;
    q.A = r.A;
    q.B = r.B;
    q.X = r.X;
    q.W = (char*)sv->dev + ws.off;
    q.lda = r.lda;
    q.ldb = r.ldb;
    q.ldx = r.ldx;
    q.n = r.n;
    q.nrhs = r.nrhs;
    q.prec = r.prec;
    q.max_iter = r.max_iter > 0 ? r.max_iter : 30;
    q.result = nullptr;
    descs.push_back(q);
    batch->members.push_back(*it);
    batch->ws.push_back(ws);
    it = sv->queue.erase(it);
  }
  return flush();
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
  int run = 0;
  for (auto& b : sv->batches) run += b.busy ? (int)b.members.size() : 0;
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

// Host driver and C ABI of liblp.so.
//
// lu_factor runs the blocked right-looking LU of the paper's "Base
// Implementation" (section "High Performance Linpack", figure fig:lu_iteration)
// one block column of width nb at a time:
//   1. factor the column panel (diagonal block plus the "left" blocks below it)
//      with partial pivoting -- recursively: split the panel in two, factor the
//      left half, exchange rows / solve / update the right half, factor the
//      right half, exchange rows in the left half; the narrow leaves (<= 32
//      columns) run as one kernel with a grid barrier per column;
//   2. apply the panel's row exchanges to every column outside the panel;
//   3. solve the "top" blocks with the panel's unit lower triangle;
//   4. update the "inner" blocks with one matrix multiplication.
// With look-ahead (figure fig:lu_execution_schedule_pcie: the communication
// phase of the next iteration overlaps the update phase), step 4 first updates
// only the next panel's columns, the next panel is factored on a second stream
// while the rest of the multiplication runs, and step 2/3 of the next
// iteration wait for both.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace lp {

template <typename T>
int launch_lu_solve(int n, const T* LU, long long lda, const int32_t* ipiv, const int32_t* info,
                    T* B, long long ldb, int nrhs, int32_t* status, hipStream_t s);
int launch_residual(int n, const double* A, long long lda, const double* X, long long ldx,
                    const double* B, long long ldb, int nrhs, double* out, hipStream_t s);

int num_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < 64) {
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (dev >= 0 && dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

namespace {

constexpr int kMaxN = 131072;
constexpr int kMaxNb = 1024;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Workspace layout of lu_factor (offsets in bytes).
struct FactorLayout {
  size_t barriers, n_barriers, slots, plan_panel, plan_trail, total;
};

FactorLayout factor_layout(int n, int nb) {
  (void)nb;
  FactorLayout L;
  size_t off = 0;
  L.barriers = off;
  L.n_barriers = (size_t)n + 64;
  off = align_up(off + 4 * L.n_barriers, 256);
  L.slots = off;
  off = align_up(off + leaf_slots_bytes(n, kLeafMax), 256);
  L.plan_panel = off;
  off = align_up(off + swap_plan_bytes(kMaxNb), 256);
  L.plan_trail = off;
  off = align_up(off + swap_plan_bytes(kMaxNb), 256);
  L.total = off;
  return L;
}

bool valid_prec(int p) { return p == LP_FP64 || p == LP_FP32 || p == LP_BF16 || p == LP_FP16; }

template <typename T>
struct Factor {
  int m;  // rows
  T* A;
  long long lda;
  int32_t* ipiv;
  int32_t* info;
  int prec;
  char* slots;
  unsigned* barriers;
  int n_barriers;
  int next_barrier;
  void* plan_panel;
  hipStream_t s;

  T* at(long long i, long long j) const { return A + i * lda + j; }

  int leaf(int j0, int w) {
    if (next_barrier >= n_barriers) return LP_ENOTSUP;
    unsigned* bar = barriers + next_barrier++;
    return launch_panel_leaf<T>(m, j0, w, A, lda, ipiv, info, 0, slots, bar, s);
  }

  // exchange rows per ipiv[k1..k2) over columns [c0, c1)
  int swaps(int k1, int k2, int c0, int c1) {
    if (k2 <= k1 || c1 <= c0) return LP_OK;
    int rc = launch_swap_plan(ipiv, k1, k2, plan_panel, s);
    if (rc != LP_OK) return rc;
    return launch_swap_apply<T>(A, lda, c0, c1, c1, c1, k2 - k1, plan_panel, s);
  }

  // factor columns [j0, j0 + w) over rows [j0, m)
  int panel(int j0, int w) {
    if (w <= kLeafMax) return leaf(j0, w);
    int w1 = w / 2;
    w1 = std::max(kLeafMax, (w1 / kLeafMax) * kLeafMax);
    const int w2 = w - w1;
    int rc = panel(j0, w1);
    if (rc != LP_OK) return rc;
    if ((rc = swaps(j0, j0 + w1, j0 + w1, j0 + w)) != LP_OK) return rc;
    if ((rc = launch_trsm_lower_unit<T>(w1, w2, at(j0, j0), lda, at(j0, j0 + w1), lda, s)) !=
        LP_OK)
      return rc;
    const int mrest = m - j0 - w1;
    if (mrest > 0) {
      if ((rc = launch_gemm_update(prec_for_gemm(), mrest, w2, w1, at(j0 + w1, j0), lda,
                                   at(j0, j0 + w1), lda, at(j0 + w1, j0 + w1), lda, s)) != LP_OK)
        return rc;
    }
    if ((rc = panel(j0 + w1, w2)) != LP_OK) return rc;
    return swaps(j0 + w1, j0 + w, j0, j0 + w1);
  }

  // The panel's own multiplications stay in the storage precision.
  int prec_for_gemm() const { return sizeof(T) == 8 ? LP_FP64 : LP_FP32; }
};

template <typename T>
int factor_impl(int n, int nb, int prec, T* A, long long lda, int32_t* ipiv, int32_t* info,
                char* work, hipStream_t s) {
  const FactorLayout L = factor_layout(n, nb);
  int rc = launch_zero_words(info, 1, s);
  if (rc != LP_OK) return rc;
  if (n == 0) return LP_OK;
  if ((rc = launch_zero_words(work + L.barriers, L.n_barriers, s)) != LP_OK) return rc;
  Factor<T> f{n,       A,    lda,   ipiv, info, prec, work + L.slots, (unsigned*)(work + L.barriers),
              (int)L.n_barriers, 0, work + L.plan_panel, s};
  void* plan_trail = work + L.plan_trail;
  for (int j0 = 0; j0 < n; j0 += nb) {
    const int w = std::min(nb, n - j0);
    if ((rc = f.panel(j0, w)) != LP_OK) return rc;
    const int j1 = j0 + w;
    if (j0 > 0 || j1 < n) {
      if ((rc = launch_swap_plan(ipiv, j0, j1, plan_trail, s)) != LP_OK) return rc;
      if ((rc = launch_swap_apply<T>(A, lda, j1, n, 0, j0, w, plan_trail, s)) != LP_OK) return rc;
    }
    if (j1 < n) {
      if ((rc = launch_trsm_lower_unit<T>(w, n - j1, f.at(j0, j0), lda, f.at(j0, j1), lda, s)) !=
          LP_OK)
        return rc;
      if ((rc = launch_gemm_update(prec, n - j1, n - j1, w, f.at(j1, j0), lda, f.at(j0, j1), lda,
                                   f.at(j1, j1), lda, s)) != LP_OK)
        return rc;
    }
  }
  return LP_OK;
}

}  // namespace
}  // namespace lp

using namespace lp;

extern "C" {

int lp_version(void) { return 100; }

const char* lp_strerror(int code) {
  if (code == LP_OK) return "success";
  if (code == LP_ENOSPC) return "workspace too small";
  if (code == LP_ENOTSUP) return "size or precision not supported by the kernels";
  if (code <= LP_EHIP_BASE) {
    const hipError_t e = (hipError_t)(LP_EHIP_BASE - code);
    return hipGetErrorString(e);
  }
  if (code < 0) return "illegal argument";
  return "unknown status";
}

size_t lu_workspace_bytes(int n, int nb, int prec) {
  if (n < 0 || n > kMaxN || nb < 1 || nb > kMaxNb || !valid_prec(prec)) return 0;
  return factor_layout(n, nb).total;
}

int lu_factor(int n, int nb, int prec, void* A, int lda, int32_t* ipiv, int32_t* info, void* work,
              size_t work_bytes, void* stream) {
  if (n < 0) return -1;
  if (n > kMaxN) return LP_ENOTSUP;
  if (nb < 1 || nb > kMaxNb) return -2;
  if (!valid_prec(prec)) return -3;
  if (A == nullptr && n > 0) return -4;
  if (lda < std::max(1, n)) return -5;
  if (ipiv == nullptr && n > 0) return -6;
  if (info == nullptr) return -7;
  if (work == nullptr) return -8;
  if (work_bytes < lu_workspace_bytes(n, nb, prec)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (prec == LP_FP64)
    return factor_impl<double>(n, nb, prec, (double*)A, lda, ipiv, info, (char*)work, s);
  return factor_impl<float>(n, nb, prec, (float*)A, lda, ipiv, info, (char*)work, s);
}

int lu_solve(int n, int storage, const void* LU, int lda, const int32_t* ipiv,
             const int32_t* info, void* B, int ldb, int nrhs, int32_t* solve_status,
             void* stream) {
  if (n < 0) return -1;
  if (storage != LP_FP64 && storage != LP_FP32) return -2;
  if (LU == nullptr && n > 0) return -3;
  if (lda < std::max(1, n)) return -4;
  if (ipiv == nullptr && n > 0) return -5;
  if (B == nullptr && n > 0 && nrhs > 0) return -7;
  if (nrhs < 0) return -9;
  if (ldb < std::max(1, nrhs)) return -8;
  hipStream_t s = (hipStream_t)stream;
  if (storage == LP_FP64)
    return launch_lu_solve<double>(n, (const double*)LU, lda, ipiv, info, (double*)B, ldb, nrhs,
                                   solve_status, s);
  return launch_lu_solve<float>(n, (const float*)LU, lda, ipiv, info, (float*)B, ldb, nrhs,
                                solve_status, s);
}

int residual_check(int n, const double* A, int lda, const double* X, int ldx, const double* B,
                   int ldb, int nrhs, double* out, void* stream) {
  if (n < 0) return -1;
  if (A == nullptr && n > 0) return -2;
  if (lda < std::max(1, n)) return -3;
  if (X == nullptr && n > 0) return -4;
  if (ldx < std::max(1, nrhs)) return -5;
  if (B == nullptr && n > 0) return -6;
  if (ldb < std::max(1, nrhs)) return -7;
  if (nrhs < 0) return -8;
  if (out == nullptr && nrhs > 0) return -9;
  return launch_residual(n, A, lda, X, ldx, B, ldb, nrhs, out, (hipStream_t)stream);
}

int lp_panel_factor(int m, int w, int prec, void* A, int lda, int32_t* ipiv, int32_t* info,
                    void* work, size_t work_bytes, void* stream) {
  if (m < 0 || m > kMaxN) return -1;
  if (w < 0 || w > m || w > kMaxNb) return -2;
  if (!valid_prec(prec)) return -3;
  if (A == nullptr && m > 0) return -4;
  if (lda < std::max(1, w)) return -5;
  if (ipiv == nullptr && w > 0) return -6;
  if (info == nullptr) return -7;
  if (work == nullptr) return -8;
  if (work_bytes < lu_workspace_bytes(m, std::max(1, w), prec)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  const FactorLayout L = factor_layout(m, std::max(1, w));
  int rc = launch_zero_words(info, 1, s);
  if (rc != LP_OK || w == 0) return rc;
  if ((rc = launch_zero_words((char*)work + L.barriers, L.n_barriers, s)) != LP_OK) return rc;
  char* wk = (char*)work;
  if (prec == LP_FP64) {
    Factor<double> f{m, (double*)A, lda, ipiv, info, prec, wk + L.slots, (unsigned*)(wk + L.barriers),
                     (int)L.n_barriers, 0, wk + L.plan_panel, s};
    return f.panel(0, w);
  }
  Factor<float> f{m, (float*)A, lda, ipiv, info, prec, wk + L.slots, (unsigned*)(wk + L.barriers),
                  (int)L.n_barriers, 0, wk + L.plan_panel, s};
  return f.panel(0, w);
}

size_t lp_laswp_workspace_bytes(int nswaps) {
  if (nswaps < 0 || nswaps > kMaxNb) return 0;
  return swap_plan_bytes(nswaps);
}

int lp_laswp(int prec, void* A, int lda, int c0, int c1, int k1, int k2, const int32_t* ipiv,
             void* work, size_t work_bytes, void* stream) {
  if (!valid_prec(prec)) return -1;
  if (lda < 1) return -3;
  if (c0 < 0 || c0 > lda) return -4;
  if (c1 < c0 || c1 > lda) return -5;
  if (k1 < 0) return -6;
  if (k2 < k1 || k2 - k1 > kMaxNb) return -7;
  if (ipiv == nullptr && k2 > k1) return -8;
  if (A == nullptr && k2 > k1 && c1 > c0) return -2;
  if (work == nullptr) return -9;
  if (work_bytes < lp_laswp_workspace_bytes(k2 - k1)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (k2 == k1 || c1 == c0) return LP_OK;
  int rc = launch_swap_plan(ipiv, k1, k2, work, s);
  if (rc != LP_OK) return rc;
  if (prec == LP_FP64)
    return launch_swap_apply<double>((double*)A, lda, c0, c1, c1, c1, k2 - k1, work, s);
  return launch_swap_apply<float>((float*)A, lda, c0, c1, c1, c1, k2 - k1, work, s);
}

int lp_trsm_lower_unit(int prec, int m, int ncols, const void* L, int ldl, void* B, int ldb,
                       void* stream) {
  if (!valid_prec(prec)) return -1;
  if (m < 0) return -2;
  if (ncols < 0) return -3;
  if (L == nullptr && m > 0) return -4;
  if (ldl < std::max(1, m)) return -5;
  if (B == nullptr && m > 0 && ncols > 0) return -6;
  if (ldb < std::max(1, ncols)) return -7;
  hipStream_t s = (hipStream_t)stream;
  if (prec == LP_FP64)
    return launch_trsm_lower_unit<double>(m, ncols, (const double*)L, ldl, (double*)B, ldb, s);
  return launch_trsm_lower_unit<float>(m, ncols, (const float*)L, ldl, (float*)B, ldb, s);
}

int lp_gemm_update(int prec, int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                   void* C, int ldc, void* stream) {
  if (!valid_prec(prec)) return -1;
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (K < 0) return -4;
  if (A == nullptr && M > 0 && K > 0) return -5;
  if (lda < std::max(1, K)) return -6;
  if (B == nullptr && K > 0 && N > 0) return -7;
  if (ldb < std::max(1, N)) return -8;
  if (C == nullptr && M > 0 && N > 0) return -9;
  if (ldc < std::max(1, N)) return -10;
  return launch_gemm_update(prec, M, N, K, A, lda, B, ldb, C, ldc, (hipStream_t)stream);
}

int lp_convert(int to_f32, int rows, int cols, const void* src, int lds, void* dst, int ldd,
               void* stream) {
  if (rows < 0) return -2;
  if (cols < 0) return -3;
  if (src == nullptr && rows > 0 && cols > 0) return -4;
  if (lds < std::max(1, cols)) return -5;
  if (dst == nullptr && rows > 0 && cols > 0) return -6;
  if (ldd < std::max(1, cols)) return -7;
  return launch_convert(to_f32, rows, cols, src, lds, dst, ldd, (hipStream_t)stream);
}

size_t lu_solve_ir_workspace_bytes(int n, int nb, int prec, int nrhs) {
  (void)n;
  (void)nb;
  (void)prec;
  (void)nrhs;
  return 0;
}

int lu_solve_ir(int n, int nb, int prec, const double* A, int lda, const double* B, int ldb,
                double* X, int ldx, int nrhs, int max_iter, void* work, size_t work_bytes,
                lp_ir_report* rep, void* stream) {
  (void)n; (void)nb; (void)prec; (void)A; (void)lda; (void)B; (void)ldb; (void)X; (void)ldx;
  (void)nrhs; (void)max_iter; (void)work; (void)work_bytes; (void)rep; (void)stream;
  return LP_ENOTSUP;
}

}  // extern "C"

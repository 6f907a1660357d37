// Mixed-precision solve with binary64 iterative refinement.
//
// The paper lets its LINPACK kernels run in single precision and, because the
// benchmark only times the device, does not refine the result (section "High
// Performance Linpack").  Here the low-precision factorization is the fast
// part, and binary64 accuracy is won back by classical iterative refinement:
// factor a binary32 copy of A (trailing-update operands in binary32, bfloat16
// or half), solve for x0 with those factors, then repeat
//     r = b - A x        (binary64, original A; the same pass yields the
//                         benchmark's scaled residual)
//     d = solve(LU32, r) (binary32 factors and solve)
//     x = x + d          (binary64)
// until the scaled residual is below 16.  If it does not get there (too many
// steps, a non-finite residual, or growth two steps in a row) the matrix is
// factored in binary64 and solved directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace lp {
namespace {

__global__ void copy_f64_kernel(int rows, int cols, const double* __restrict__ src, long long lds,
                                double* __restrict__ dst, long long ldd) {
  const long long total = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / cols, c = e - r * cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

// X (double) += D (float)
__global__ void add_f32_to_f64_kernel(int rows, int cols, const float* __restrict__ D, long long ldd,
                                      double* __restrict__ X, long long ldx) {
  const long long total = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / cols, c = e - r * cols;
    X[r * ldx + c] += (double)D[r * ldd + c];
  }
}

unsigned blocks_for(long long total) {
  long long b = (total + 255) / 256;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct IRLayout {
  size_t big, fwork, ipiv, info, R, D, out, swork, total;
};

IRLayout ir_layout(int n, int nb, int prec, int nrhs) {
  IRLayout L;
  size_t off = 0;
  L.big = off;  // binary32 copy of A; reused for the binary64 copy of the fallback
  off = align_up(off + sizeof(double) * (size_t)n * n, 256);
  L.fwork = off;
  // the low-precision factorization and the binary64 fallback share it
  off = align_up(off + std::max(lu_workspace_bytes(n, nb, prec), lu_workspace_bytes(n, nb, LP_FP64)),
                 256);
  L.ipiv = off;
  off = align_up(off + sizeof(int32_t) * (size_t)std::max(n, 1), 256);
  L.info = off;
  off = align_up(off + 16, 256);
  L.R = off;
  off = align_up(off + sizeof(double) * (size_t)n * nrhs, 256);
  L.D = off;
  off = align_up(off + sizeof(float) * (size_t)n * nrhs, 256);
  L.out = off;
  off = align_up(off + sizeof(double) * 5 * (size_t)std::max(nrhs, 1), 256);
  L.swork = off;  // the one-launch triangular solves (binary64 size covers binary32)
  off = align_up(off + lu_solve_workspace_bytes_t(n, 8), 256);
  L.total = off;
  return L;
}

struct Events {
  std::vector<hipEvent_t> ev;
  ~Events() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  int record(hipStream_t s, hipEvent_t* out) {
    hipEvent_t e;
    LP_HIP_TRY(hipEventCreate(&e));
    ev.push_back(e);
    LP_HIP_TRY(hipEventRecord(e, s));
    *out = e;
    return LP_OK;
  }
};

double ms_between(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (a && b && hipEventElapsedTime(&ms, a, b) == hipSuccess) return ms;
  return 0.0;
}

}  // namespace
}  // namespace lp

using namespace lp;

extern "C" {

// Refinement decision from the scaled-residual history h[0..len) (h[0] after x0,
// h[k] after the k-th correction): 1 = converged (last < 16), 2 = give up
// (last not finite, last two steps both grew, or corrections == max_iter),
// 0 = apply another correction.
int lp_ir_decide(const double* h, int len, int corrections, int max_iter) {
  if (h == nullptr || len <= 0) return 0;
  const double s = h[len - 1];
  if (!std::isfinite(s)) return 2;
  if (s < 16.0) return 1;
  if (len >= 3 && h[len - 1] > h[len - 2] && h[len - 2] > h[len - 3]) return 2;
  if (corrections >= max_iter) return 2;
  return 0;
}

size_t lu_solve_ir_workspace_bytes(int n, int nb, int prec, int nrhs) {
  if (n < 0 || nrhs < 0 || lu_workspace_bytes(n, nb, prec) == 0) return 0;
  return ir_layout(n, nb, prec, nrhs).total;
}

int lu_solve_ir(int n, int nb, int prec, const double* A, int lda, const double* B, int ldb,
                double* X, int ldx, int nrhs, int max_iter, void* work, size_t work_bytes,
                lp_ir_report* rep, void* stream) {
  if (n < 0) return -1;
  if (nb < 1) return -2;
  if (prec != LP_FP64 && prec != LP_FP32 && prec != LP_BF16 && prec != LP_FP16) return -3;
  if (A == nullptr && n > 0) return -4;
  if (lda < std::max(1, n)) return -5;
  if (B == nullptr && n > 0 && nrhs > 0) return -6;
  if (ldb < std::max(1, nrhs)) return -7;
  if (X == nullptr && n > 0 && nrhs > 0) return -8;
  if (ldx < std::max(1, nrhs)) return -9;
  if (nrhs < 0) return -10;
  if (max_iter < 0 || max_iter > 62) return -11;
  if (work == nullptr) return -12;
  if (rep == nullptr) return -14;
  const size_t need = lu_solve_ir_workspace_bytes(n, nb, prec, nrhs);
  if (need == 0) return LP_ENOTSUP;
  if (work_bytes < need) return LP_ENOSPC;
  std::memset(rep, 0, sizeof(*rep));
  hipStream_t s = (hipStream_t)stream;
  if (n == 0 || nrhs == 0) {
    rep->converged = 1;
    return LP_OK;
  }
  const IRLayout L = ir_layout(n, nb, prec, nrhs);
  char* w = (char*)work;
  int32_t* ipiv = (int32_t*)(w + L.ipiv);
  int32_t* info = (int32_t*)(w + L.info);
  double* R = (double*)(w + L.R);
  float* D = (float*)(w + L.D);
  double* out_d = (double*)(w + L.out);
  void* swork = w + L.swork;
  const long long nn = (long long)n;
  Events evs;
  hipEvent_t e0, e_conv = nullptr, e_fact = nullptr, e_solve0 = nullptr, e_ref = nullptr,
                 e_fb0 = nullptr, e_end = nullptr;
  int rc;
  if ((rc = evs.record(s, &e0)) != LP_OK) return rc;

  std::vector<double> host_out(5 * (size_t)nrhs);
  auto scaled_residual = [&](double* smax) -> int {
    int r = launch_residual(n, A, lda, X, ldx, B, ldb, nrhs, out_d, s, R, nrhs);
    if (r != LP_OK) return r;
    LP_HIP_TRY(hipMemcpyAsync(host_out.data(), out_d, sizeof(double) * 5 * nrhs,
                              hipMemcpyDeviceToHost, s));
    LP_HIP_TRY(hipStreamSynchronize(s));
    double m = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const double v = host_out[5 * c];
      if (!(v <= m)) m = v;  // NaN propagates
    }
    *smax = m;
    return LP_OK;
  };
  auto direct_fp64 = [&]() -> int {
    double* A64 = (double*)(w + L.big);
    hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks_for(nn * nn)), dim3(256), 0, s, n, n, A, lda,
                       A64, nn);
    LP_LAUNCH_CHECK();
    int r = lu_factor(n, nb, LP_FP64, A64, n, ipiv, info, w + L.fwork,
                      lu_workspace_bytes(n, nb, LP_FP64), s);
    if (r != LP_OK) return r;
    hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks_for(nn * nrhs)), dim3(256), 0, s, n, nrhs, B,
                       ldb, X, ldx);
    LP_LAUNCH_CHECK();
    return launch_lu_solve_ws<double, double>(n, A64, nn, ipiv, info, X, ldx, nrhs, nullptr,
                                              swork, s);
  };

  bool need_fallback = (prec == LP_FP64);
  if (prec != LP_FP64) {
    // low-precision factorization and the first solve
    float* A32 = (float*)(w + L.big);
    if ((rc = launch_convert(1, n, n, A, lda, A32, nn, s)) != LP_OK) return rc;
    if ((rc = evs.record(s, &e_conv)) != LP_OK) return rc;
    if ((rc = lu_factor(n, nb, prec, A32, n, ipiv, info, w + L.fwork,
                        lu_workspace_bytes(n, nb, prec), s)) != LP_OK)
      return rc;
    if ((rc = evs.record(s, &e_fact)) != LP_OK) return rc;
    if ((rc = launch_convert(1, n, nrhs, B, ldb, D, nrhs, s)) != LP_OK) return rc;
    if ((rc = launch_lu_solve_ws<float, float>(n, A32, nn, ipiv, info, D, nrhs, nrhs, nullptr,
                                                swork, s)) != LP_OK)
      return rc;
    if ((rc = launch_convert(0, n, nrhs, D, nrhs, X, ldx, s)) != LP_OK) return rc;
    if ((rc = evs.record(s, &e_solve0)) != LP_OK) return rc;
    int32_t info_h = 0;
    LP_HIP_TRY(hipMemcpyAsync(&info_h, info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    double sres = 0.0;
    if ((rc = scaled_residual(&sres)) != LP_OK) return rc;  // synchronizes
    rep->info = info_h;
    rep->history[rep->history_len++] = sres;
    if (info_h != 0) {
      need_fallback = true;
    } else {
      for (;;) {
        const int d = lp_ir_decide(rep->history, rep->history_len, rep->iterations, max_iter);
        if (d == 1) break;
        if (d == 2) {
          need_fallback = true;
          break;
        }
        // d = solve(LU32, r); x += d
        if ((rc = launch_convert(1, n, nrhs, R, nrhs, D, nrhs, s)) != LP_OK) return rc;
        if ((rc = launch_lu_solve_ws<float, float>(n, A32, nn, ipiv, info, D, nrhs, nrhs,
                                                    nullptr, swork, s)) != LP_OK)
          return rc;
        hipLaunchKernelGGL(add_f32_to_f64_kernel, dim3(blocks_for(nn * nrhs)), dim3(256), 0, s,
                           n, nrhs, D, (long long)nrhs, X, (long long)ldx);
        LP_LAUNCH_CHECK();
        rep->iterations++;
        if ((rc = scaled_residual(&sres)) != LP_OK) return rc;
        rep->history[rep->history_len++] = sres;
        if (rep->history_len >= 64) {
          need_fallback = lp_ir_decide(rep->history, rep->history_len, rep->iterations,
                                       max_iter) != 1;
          break;
        }
      }
    }
    if ((rc = evs.record(s, &e_ref)) != LP_OK) return rc;
    rep->scaled_residual = rep->history[rep->history_len - 1];
  }
  if (need_fallback) {
    if ((rc = evs.record(s, &e_fb0)) != LP_OK) return rc;
    if ((rc = direct_fp64()) != LP_OK) return rc;
    int32_t info_h = 0;
    LP_HIP_TRY(hipMemcpyAsync(&info_h, info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    double sres = 0.0;
    if ((rc = scaled_residual(&sres)) != LP_OK) return rc;
    rep->fell_back = (prec != LP_FP64) ? 1 : 0;
    rep->fallback_info = info_h;
    rep->scaled_residual = sres;
    if (prec == LP_FP64) {
      rep->info = info_h;
      rep->history[rep->history_len++] = sres;
    }
  }
  if ((rc = evs.record(s, &e_end)) != LP_OK) return rc;
  LP_HIP_TRY(hipEventSynchronize(e_end));
  rep->converged = (rep->scaled_residual < 16.0) ? 1 : 0;
  rep->t_convert_ms = ms_between(e0, e_conv);
  rep->t_factor_ms = ms_between(e_conv, e_fact);
  rep->t_solve0_ms = ms_between(e_fact, e_solve0);
  rep->t_refine_ms = ms_between(e_solve0, e_ref);
  rep->t_fallback_ms = ms_between(e_fb0, e_end);
  rep->t_total_ms = ms_between(e0, e_end);
  return LP_OK;
}

}  // extern "C"

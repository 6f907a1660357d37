// Shared helpers for the gfx950 kernels and the host driver of liblp.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/lp.h"

#define LP_HIP_TRY(expr)                              \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return LP_EHIP_BASE - (int)e_; \
  } while (0)

#define LP_LAUNCH_CHECK()                                  \
  do {                                                     \
    hipError_t e_ = hipGetLastError();                     \
    if (e_ != hipSuccess) return LP_EHIP_BASE - (int)e_;   \
  } while (0)

namespace lp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

__host__ __device__ inline long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

// Number of compute units of the current device (cached per device id).
int num_cus();

// ---------------------------------------------------------------- kernels
// All launchers return LP_OK or LP_EHIP_BASE - hipError.  Arguments are
// assumed valid (checked by the C ABI layer).

// C := C - A B (row-major, prec as lp_prec).  kind selects the kernel name
// (trailing update or update inside a panel); the arithmetic is the same.
constexpr int kGemmTrailing = 0;
constexpr int kGemmPanel = 1;
int launch_gemm_update(int prec, int M, int N, int K, const void* A, long long lda,
                       const void* B, long long ldb, void* C, long long ldc, hipStream_t s,
                       int kind = kGemmTrailing);

// binary32 storage: C := C - A B with operands on FP32, BF16 or FP16 MFMA.
int launch_gemm_update_lp(int prec, int M, int N, int K, const float* A, long long lda,
                          const float* B, long long ldb, float* C, long long ldc, hipStream_t s);
// The same update for bfloat16 / half through operands packed into pa (-A,
// gemm_lp_packed_bytes(M, K) bytes; written only when pack_a) and pb (B^T,
// gemm_lp_packed_bytes(N, K) bytes), 16-byte aligned.  Pays off when
// gemm_lp_packed_pays (enough 256 x 256 tiles to fill the device).
size_t gemm_lp_packed_bytes(int rows, int K);
bool gemm_lp_packed_pays(int prec, int M, int N, int K);
int launch_gemm_update_lp_packed(int prec, int M, int N, int K, const float* A, long long lda,
                                 const float* B, long long ldb, float* C, long long ldc,
                                 void* pa, void* pb, bool pack_a, hipStream_t s);

// B := L^-1 B, L unit lower m x m; work: trsm_workspace_bytes(m), which first
// receives the inverses of L's 16 x 16 diagonal blocks.  With inverses_ready
// the caller has already written them there (launch_diag_block_inverse, on a
// stream ordered before this one), so several column ranges can share them.
size_t trsm_workspace_bytes(int m);
template <typename T>
int launch_diag_block_inverse(int m, const T* L, long long ldl, void* work, hipStream_t s);
template <typename T>
int launch_trsm_lower_unit(int m, int ncols, const T* L, long long ldl, T* B, long long ldb,
                           void* work, hipStream_t s, bool inverses_ready = false);

// Swap plan for interchanges k1..k2-1 (device ipiv, absolute rows): writes a
// gather list (dst, src) into plan; see panel.hip.
size_t swap_plan_bytes(int nswaps);
int launch_swap_plan(const int32_t* ipiv, int k1, int k2, void* plan, hipStream_t s);
// Interchanges k1..k2-1 (k2 - k1 <= 1024) applied to columns [c0, c1) in one
// launch, each workgroup building the plan itself.
template <typename T>
int launch_swap_fused(T* A, long long lda, int c0, int c1, const int32_t* ipiv, int k1, int k2,
                      hipStream_t s);
// Apply a plan to columns [c0, c1) and [c2, c3) of A.
template <typename T>
int launch_swap_apply(T* A, long long lda, int c0, int c1, int c2, int c3, int nswaps,
                      const void* plan, hipStream_t s);

// Panel factorization in one launch: columns [c0, c0+W) over rows [c0, m)
// (absolute indices), W <= 1024.  slots: leaf_slots_bytes(); barrier: one
// zeroed 32-bit counter; staging: panel_staging_bytes(W).
constexpr int kLeafMax = 32;
size_t leaf_slots_bytes(int m, int w);
size_t panel_staging_bytes(int W);
// keys: this launch's zeroed key buffer; keys_next: the buffer of the next
// panel launch on the same stream, which this launch zeroes.
// max_wgs > 0: the launch runs on a stream restricted to that many compute
// units, so it uses at most max_wgs workgroups (up to 1024 rows each) and
// returns LP_ENOTSUP when the rows do not fit.
// nopiv: no pivot search, the diagonal row is every column's pivot (ipiv[j] =
// j); only for at most 1024 rows (one workgroup), else LP_ENOTSUP.
size_t panel_keys_bytes();
constexpr int kPanelRowsPerWg = 1024;
// next_w: the widest later launch that uses keys_next (its key slots are
// cleared by this launch); the launch's own width when 0.
template <typename T>
int launch_panel_fused(int m, int c0, int W, T* A, long long lda, int32_t* ipiv, int32_t* info,
                       void* slots, unsigned* barrier, void* staging, void* keys,
                       void* keys_next, hipStream_t s, int max_wgs = 0, bool nopiv = false,
                       int next_w = 0);

// X U = B for X, U upper triangular (non-unit) w x w, B m x w (ld ldb), in
// place: B := B U^-1 (the "left blocks" of the no-pivot LU).  work:
// trsm_workspace_bytes(min(w, 128)) bytes.
template <typename T>
int launch_trsm_right_upper(int m, int w, const T* U, long long ldu, T* B, long long ldb,
                            void* work, hipStream_t s);

// Factorization / solve / residual (driver.hip, solve.hip), used by the IR driver.
template <typename T>
int launch_lu_solve(int n, const T* LU, long long lda, const int32_t* ipiv, const int32_t* info,
                    T* B, long long ldb, int nrhs, int32_t* status, hipStream_t s);
// The same solve as one persistent launch per triangle (and per 8
// right-hand sides) with a workspace of lu_solve_workspace_bytes_t(n,
// sizeof(T)) bytes; TF is the factors' storage, T the right-hand sides'
// type and the arithmetic (float factors may be applied in double).
size_t lu_solve_workspace_bytes_t(int n, int elem_bytes);
template <typename TF, typename T>
int launch_lu_solve_ws(int n, const TF* LU, long long lda, const int32_t* ipiv,
                       const int32_t* info, T* B, long long ldb, int nrhs, int32_t* status,
                       void* work, hipStream_t s);
int launch_residual(int n, const double* A, long long lda, const double* X, long long ldx,
                    const double* B, long long ldb, int nrhs, double* out, hipStream_t s,
                    double* Rv, long long ldr);

// C := B + A^T (n x n, prec LP_FP64 or LP_FP32); C may be B, must not overlap A.
int launch_ptrans(int prec, int n, const void* A, long long lda, const void* B, long long ldb,
                  void* C, long long ldc, hipStream_t s);

// Timing-enabled HIP events from a process-wide pool (per device): an event
// is handed out again only after it has completed.
hipError_t acquire_timing_event(hipEvent_t* out);
void release_timing_event(hipEvent_t e);

// Zero a range of 32-bit words (a kernel, not a memset node).
int launch_zero_words(void* p, size_t nwords, hipStream_t s);

// Element-wise precision conversion.
int launch_convert(int to_f32, int rows, int cols, const void* src, long long lds, void* dst,
                   long long ldd, hipStream_t s);

}  // namespace lp

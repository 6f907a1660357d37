// Device side of the seeded input generator (no solver arithmetic here).
//
// Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): for a given
// (seed, stream) the state starts at key = mix64(seed) ^ (stream << 60) and the
// idx-th word is mix64(key + (idx + 1) * 0x9E3779B97F4A7C15); the value is
// (word >> 11) * 2^-53 - 0.5 in [-0.5, 0.5).  Element (i, j) of a logical
// rows x logical_cols matrix uses idx = i * logical_cols + j, so any block of
// rows can be produced on its own.  An optional diagonal shift adds `shift` to
// element (i, i) in round-to-nearest binary64 (then narrows to float for the
// float32 output form).  The host generator in inputs/__init__.py is the same
// definition; the two are compared bitwise by the tests.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

template <typename T>
__global__ void gen_uniform_kernel(T* __restrict__ out, int rows, int cols, long long ld,
                                   long long row0, long long logical_cols, uint64_t key,
                                   double shift) {
  const long long total = (long long)rows * cols;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const long long r = e / cols;
    const long long c = e - r * cols;
    const long long gi = row0 + r;
    const uint64_t idx = (uint64_t)gi * (uint64_t)logical_cols + (uint64_t)c;
    const uint64_t w = mix64(key + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
    double v = (double)(w >> 11) * 0x1.0p-53 - 0.5;
    if (shift != 0.0 && gi == c) v = v + shift;
    out[r * ld + c] = (T)v;
  }
}

uint64_t host_mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

}  // namespace

// Fill rows [row0, row0+rows) x columns [0, cols) of the logical matrix into
// `out` (row-major, leading dimension ld >= cols, device memory owned by the
// caller).  is_f32 selects float output, else double.  Returns 0, -k for an
// illegal k-th argument, or -1000 - hipError for a launch failure.
extern "C" int lp_gen_uniform(void* out, int rows, int cols, int ld, long long row0,
                              long long logical_cols, int is_f32, int reserved,
                              uint64_t seed, int stream, double shift, hipStream_t s) {
  (void)reserved;
  if (rows < 0) return -2;
  if (cols < 0) return -3;
  if (ld < (cols > 1 ? cols : 1)) return -4;
  if (row0 < 0) return -5;
  if (logical_cols < cols) return -6;
  if (stream < 0 || stream > 15) return -10;
  if (rows == 0 || cols == 0) return 0;
  if (out == nullptr) return -1;
  const uint64_t key = host_mix64(seed) ^ ((uint64_t)stream << 60);
  const long long total = (long long)rows * cols;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (is_f32) {
    hipLaunchKernelGGL(gen_uniform_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (float*)out, rows, cols, (long long)ld, row0, logical_cols, key, shift);
  } else {
    hipLaunchKernelGGL(gen_uniform_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (double*)out, rows, cols, (long long)ld, row0, logical_cols, key, shift);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -1000 - (int)e;
}

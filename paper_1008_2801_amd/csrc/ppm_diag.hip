// The arithmetic diagnostics (ppm_diag.h): the step kernels' FP64 quotient
// and square roots (ppm_math.h) and their zone-index division
// (ppm_internal.h) evaluated for caller-given arguments.
#include <hip/hip_runtime.h>

#include "ppm_diag.h"
#include "ppm_internal.h"
#include "ppm_math.h"

namespace {

// Values of the kernels' FP64 quotient for a list of operand pairs (grid-stride).
__global__ void __launch_bounds__(256) k_quotient(const double* __restrict__ a, const double* __restrict__ b,
                                                  double* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    out[i] = ppm::qdiv(a[i], b[i]);
}

// Values of the kernels' roots for a list of arguments (grid-stride): form
// 0 the FP64 wave-speed root, 1 the FP64 sound-speed root, 2 the FP32
// wave-speed root of (float) x, widened back to double.
__global__ void __launch_bounds__(256) k_sqrt_form(const double* __restrict__ x, double* __restrict__ out,
                                                   long long n, int form) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    out[i] = form == 0 ? ppm::sqrt_wave(x[i])
                       : (form == 1 ? ppm::sqrt_phys(x[i]) : (double)ppm::sqrt_wave((float)x[i]));
}

// The kernels' zone-index division by an invariant divisor (grid-stride).
__global__ void __launch_bounds__(256) k_div31(const uint32_t* __restrict__ n, ppm::Div31 q,
                                               uint32_t* __restrict__ out, long long count) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long long)gridDim.x * 256)
    out[i] = ppm::div31(n[i], q);
}

unsigned grid_of(long long n) {
  const long long blocks = (n + 255) / 256;
  return blocks < 4096 ? (unsigned)blocks : 4096u;
}

}  // namespace

extern "C" int ppm_diag_sqrt_values(const double* x, double* out, int64_t n, int32_t form, void* stream) {
  if (n < 0 || (n > 0 && (!x || !out)) || form < 0 || form > 2) return 1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_sqrt_form, dim3(grid_of(n)), dim3(256), 0, (hipStream_t)stream, x, out, (long long)n, form);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int ppm_diag_quotient_values(const double* a, const double* b, double* out, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!a || !b || !out))) return 1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_quotient, dim3(grid_of(n)), dim3(256), 0, (hipStream_t)stream, a, b, out, (long long)n);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int ppm_diag_div31_params(uint32_t d, uint32_t* m, int32_t* s) {
  if (d < 2 || d > 0x7fffffffu || !m || !s) return 1;
  const ppm::Div31 q = ppm::make_div31(d);
  *m = q.m;
  *s = q.s;
  return 0;
}

extern "C" int ppm_diag_div31_values(const uint32_t* n, uint32_t d, uint32_t* out, int64_t count, void* stream) {
  if (count < 0 || (count > 0 && (!n || !out)) || d < 2 || d > 0x7fffffffu) return 1;
  if (count == 0) return 0;
  hipLaunchKernelGGL(k_div31, dim3(grid_of(count)), dim3(256), 0, (hipStream_t)stream, n, ppm::make_div31(d), out,
                     (long long)count);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

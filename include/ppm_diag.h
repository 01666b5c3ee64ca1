/*
 * ppm_diag.h -- C ABI of the arithmetic diagnostics of the PPM step's
 * kernels (libppm_diag.so, a library of its own beside libppm.so).
 *
 * The step's Riemann solver (the two-shock solver of the compressible
 * code's explicit advance, paper Sec. 1), its corrected states, tracing and
 * flattening divide and take square roots with the core of the compiler's
 * correctly rounded sequences, without the operand scaling that their
 * magnitudes never need.  These entry points run exactly those sequences on
 * the device for caller-given arguments, so that a caller (the test suite)
 * can compare them with IEEE results on the host; likewise the integer
 * division the kernels decode zone indices with.  They are not part of the
 * step.
 *
 * All pointers are HIP device memory owned by the caller; calls are
 * asynchronous on the given stream (a hipStream_t passed as void*, 0 = the
 * null stream).  Return 0 on success, 1 for invalid arguments (nothing
 * enqueued), 2 for a HIP launch error.
 */
#ifndef PPM_DIAG_H
#define PPM_DIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out[i] = one of the FP64 square roots the Riemann solver takes, for n
 * arguments x[i].  form 0: the root of the wave-speed factor
 * 1 + beta (p/p_s - 1) (>= 1 - beta > 0; the Lagrangian shock speed of
 * Colella-Glaz 1985 is C_s times it); form 1: the root of gamma p rho (the
 * Lagrangian sound speed C_s) and of the star state's gamma p / rho; form 2:
 * the FP32 root of the wave-speed factor, taken of (float) x[i] and returned
 * widened to double.  The IEEE root for every finite argument >= 2^-767
 * (form 2: >= 2^-96; form 1: also for 0, +inf, negative and NaN
 * arguments).  Invalid: n < 0, null pointers with n > 0, another form. */
int ppm_diag_sqrt_values(const double* x, double* out, int64_t n, int32_t form, void* stream);

/* out[i] = a[i] / b[i] as the kernels divide in FP64, for n operand pairs:
 * the IEEE quotient when the exponents of a and b lie in [-900, 900] and
 * differ by at most 700, and for zero, infinite and NaN operands (the step
 * raises PPM_FLAG_RANGE, ppm.h, for input states whose quantities could
 * leave that range).  Invalid: n < 0 or null pointers with n > 0. */
int ppm_diag_quotient_values(const double* a, const double* b, double* out, int64_t n, void* stream);

/* The division by an invariant divisor d (2 <= d < 2^31) with which every
 * kernel decodes a linear zone index into coordinates (the row lengths of a
 * box's grids and of its bricks), for dividends below 2^31: with
 * l = ceil(log2 d), m = ceil(2^(31+l) / d) (below 2^32) and s = l - 1,
 * floor(n / d) = ((n m) >> 32) >> s (Granlund and Montgomery 1994).
 * ppm_diag_div31_params returns m and s as the library forms them (host
 * only); ppm_diag_div31_values computes out[i] = floor(n[i] / d) on the
 * device exactly as the kernels do (n[i] < 2^31; device pointers).
 * Invalid: d outside [2, 2^31), null pointers, count < 0. */
int ppm_diag_div31_params(uint32_t d, uint32_t* m, int32_t* s);
int ppm_diag_div31_values(const uint32_t* n, uint32_t d, uint32_t* out, int64_t count, void* stream);

#ifdef __cplusplus
}
#endif

#endif

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
 * can compare them with IEEE results on the host.  They are not part of the
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

#ifdef __cplusplus
}
#endif

#endif

// Pointwise arithmetic of the step, shared by the forward and adjoint
// kernels and compilable for the host (for CPU checks of the derivatives).
// Every formula is a C expression evaluated left to right; built without
// FP contraction, the results are those of IEEE double/float arithmetic.
//
// The formulas are algebraically those of the method, arranged to divide
// less often: the Newton step of the two-shock solver works with 1/p_s,
// 1/W_s and 1/Z_s = (1 + (C_s/W_s)^2)/(2 W_s) (in FP64 both 1/W_s of a step
// from one division, 1/(W_L W_R)); the star sound speed uses 1/rho* from
// the Hugoniot instead of dividing by rho*; the outer sound speed is
// C_s/rho_s; a corrected state's three velocities share one 1/rho; the
// tracing's wave amplitudes multiply by 1/c^2.  They round differently
// from the plain definition (which the CPU reference evaluates), so the
// two agree to rounding, not bit for bit.
#pragma once

#include "ppm.h"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define PPM_HD __host__ __device__ __forceinline__
#else
#define PPM_HD inline
#endif

namespace ppm {

// Gas and scheme constants in the reconstruction scalar, formed on the host
// in FP64 from gamma and the floors, rounded once to S.
template <class S> struct Gas {
  S gamma, gm1, gm1inv, beta, small_dens, small_pres, ismall_dens;
  int limiter, flattening, iters, grav;
};


// ------------------------------------------------------------ helpers ------
template <class S> PPM_HD S smax(S a, S b) { return (a < b) ? b : a; }
template <class S> PPM_HD S smin(S a, S b) { return (b < a) ? b : a; }
// |a| (the sign bit cleared: one instruction, or free as an operand modifier)
PPM_HD double sabs(double a) { return __builtin_fabs(a); }
PPM_HD float sabs(float a) { return __builtin_fabsf(a); }
// min and max of two values that are not NaN (the hardware min and max)
PPM_HD double fmin2(double a, double b) { return __builtin_fmin(a, b); }
PPM_HD float fmin2(float a, float b) { return __builtin_fminf(a, b); }
// x with its sign flipped where s is negative (sign bit set)
PPM_HD double flipsign(double x, double s) {
  return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, x) ^
                                        (__builtin_bit_cast(unsigned long long, s) & 0x8000000000000000ull));
}
PPM_HD float flipsign(float x, float s) {
  return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, x) ^ (__builtin_bit_cast(unsigned, s) & 0x80000000u));
}
PPM_HD double ssqrt(double x) { return __builtin_sqrt(x); }
PPM_HD float ssqrt(float x) { return __builtin_sqrtf(x); }
// a / b.  FP64 on the device: the correctly rounded division hipcc emits
// (hardware reciprocal of b, two Newton-Raphson steps on it, the quotient,
// one residual correction, the fix-up of signs and special values) without
// its operand scaling: 9 instructions instead of 11.  The scaling only acts
// near the ends of the exponent range; when the exponents of a and b lie in
// [-900, 900] and differ by at most 700 the two give the same bits, the
// IEEE quotient (measured on the device over random operands of that range
// and tested against the host's quotient); zero, infinite and NaN operands
// go through the fix-up as before.  The kernels divide only
// quantities of a physical state (densities, pressures, sound and wave
// speeds, their sums and differences), far inside that range.  Elsewhere
// the library division.
PPM_HD double qdiv(double a, double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double q = a * r;
  e = __builtin_fma(-b, q, a);
  return __builtin_amdgcn_div_fixup(__builtin_fma(e, r, q), b, a);
#else
  return a / b;
#endif
}
PPM_HD float qdiv(float a, float b) { return a / b; }

// Square root of the two-shock wave-speed factor 1 + beta (p/p_s - 1),
// which is at least 1 - beta > 0.  FP64 on the device: the core of the
// correctly rounded square root hipcc emits (hardware reciprocal square
// root, one Newton-Raphson step on the root and the half reciprocal, two
// residual corrections of the root), without the rescaling of arguments
// below 2^-767 and the fix-up of 0 and +inf that surround it.  For every
// finite argument >= 2^-767 the two are the same instructions and give the
// same bits: 10 instructions instead of 18.  Elsewhere the library root.
PPM_HD double sqrt_wave(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r;
  double h = r * 0.5;
  const double e = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, e, g);
  h = __builtin_fma(h, e, h);
  double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  d = __builtin_fma(-g, g, x);
  return __builtin_fma(d, h, g);
#else
  return __builtin_sqrt(x);
#endif
}
// FP32 on the device: hipcc's correctly rounded FP32 root (hardware root,
// then a one-ulp correction either way from two residuals) without its
// rescaling of arguments below 2^-96 and its fix-up of 0 and +inf: 8
// instructions instead of 17, the same bits for every finite argument
// >= 2^-96.
PPM_HD float sqrt_wave(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float s = __builtin_amdgcn_sqrtf(x);
  const int si = __float_as_int(s);
  const float sm = __int_as_float(si - 1), sp = __int_as_float(si + 1);
  const float rm = __builtin_fmaf(-sm, s, x);
  const float rp = __builtin_fmaf(-sp, s, x);
  const float t = (rm <= 0.0f) ? sm : s;
  return (rp > 0.0f) ? sp : t;
#else
  return __builtin_sqrtf(x);
#endif
}
// Square root of a product of a density, a pressure and gamma (a squared
// Lagrangian sound speed or the star sound speed).  FP64 on the device: the
// same core as sqrt_wave followed by hipcc's fix-up of 0 and +inf (the root
// is x there), without the rescaling of positive arguments below 2^-767:
// 13 instructions instead of 18, the IEEE root for every argument except
// positive ones below 2^-767 (a density-pressure product below 1e-231).
PPM_HD double sqrt_phys(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double g = sqrt_wave(x);
  return __builtin_amdgcn_class(x, 0x260) ? x : g;  // +0, -0, +inf
#else
  return __builtin_sqrt(x);
#endif
}
PPM_HD float sqrt_phys(float x) { return __builtin_sqrtf(x); }
PPM_HD double scopysign(double m, double s) { return __builtin_copysign(m, s); }
PPM_HD float scopysign(float m, float s) { return __builtin_copysignf(m, s); }
// 2^-120 <= x <= 2^120 for a state's density, pressure and sound speed,
// |u| <= 2^120 for its velocity components (no quotient divides by a
// velocity): the magnitudes for which every quotient and root the step
// forms from them keeps the operand exponents where qdiv, sqrt_wave and
// sqrt_phys are the IEEE results (products of up to five such quantities
// and their differences stay within 2^-800 .. 2^600).
template <class S> PPM_HD bool in_range(S x) { return x >= S(0x1p-120) && x <= S(0x1p120); }
template <class S> PPM_HD bool speed_in_range(S u) { return sabs(u) <= S(0x1p120); }
// The sound speed sqrt(gamma p / rho) of a zone's primitives (IEEE division
// and root).  The conversion forms it, and every stage that needs it forms
// it again from the stored density and pressure, by this one expression, so
// all of them hold the same bits.
template <class S> PPM_HD S sound_speed(S r, S p, const Gas<S>& G) { return ssqrt(G.gamma * p / r); }
// a b > 0: the MC slope and the CW84 limiter test the sign of a product of
// two differences of one field.
template <class S> PPM_HD bool same_sign(S a, S b) { return a * b > S(0); }

// 1/a and 1/b of the two wave speeds W_L, W_R.  FP64: from one division,
// 1/a = b/(a b).  FP32: two divisions, which keep the FP32 range of a
// single wave speed.
template <class S> PPM_HD void pair_recip(S a, S b, S& ia, S& ib) {
  if constexpr (sizeof(S) == 4) {
    ia = S(1) / a;
    ib = S(1) / b;
  } else {
    const S iab = qdiv(S(1), a * b);
    ia = b * iab;
    ib = a * iab;
  }
}

#define HALF S(0.5)
#define ONE S(1.0)
#define TWO S(2.0)
#define THREE S(3.0)
#define SIX S(6.0)
#define SIXTH S(1.0 / 6.0)
#define TWO3 S(2.0 / 3.0)
#define C033 S(0.33)
#define TEN S(10.0)
#define C075 S(0.75)

// The CW84 overshoot tests dq m > dq^2/6 (hi) and dq m < -dq^2/6 (lo),
// m = a0 - (aL + aR)/2.
template <class S> PPM_HD void cw_overshoot(S dq, S m, bool& hi, bool& lo) {
  const S t = dq * m;
  const S d2 = dq * dq * SIXTH;
  hi = t > d2;
  lo = -d2 > t;
}

// ------------------------------------------------------- O6: Riemann -------
// Fan sampling on the left side of the contact for (rho, u, p) with the
// normal velocity oriented so that the side is the left one.  The right
// side is the mirror image: the caller negates u, u* on entry and u on exit
// (exact in IEEE arithmetic).
template <class S>
PPM_HD void sample_side(S ro, S uo, S po, S C, S W, S iW, S us, S p, const Gas<S>& G,
                                            S& r_, S& u_, S& p_, int& fl) {
  const S irho = qdiv(ONE, ro);
  const S vstar = irho - (p - po) * (iW * iW);
  S rs = qdiv(ONE, vstar), ivs = vstar;  // ivs = 1/rho* (floored with it)
  if (!(vstar > S(0)) || rs < G.small_dens) { fl |= PPM_FLAG_FLOOR; rs = G.small_dens; ivs = G.ismall_dens; }
  const S cst = sqrt_phys(G.gamma * p * ivs);
  const S co = C * irho;
  r_ = ro; u_ = uo; p_ = po;
  if (p > po) {
    const S sh = uo - W * irho;
    if (!(sh >= S(0))) { r_ = rs; u_ = us; p_ = p; }
  } else {
    const S hd = uo - co, tl = us - cst;
    if (hd >= S(0)) {
    } else if (tl <= S(0)) {
      r_ = rs; u_ = us; p_ = p;
    } else {
      const S w = qdiv(-hd, tl - hd);
      r_ = (ONE - w) * ro + w * rs;
      u_ = (ONE - w) * uo + w * us;
      p_ = (ONE - w) * po + w * p;
    }
  }
}

// Two-shock Riemann solver: flux F (xyz component order) at a face normal
// to d from primitive states L and R (rho, u, v, w, p).
template <int d, class S>
PPM_HD void riemann(const S L[5], const S R[5], const Gas<S>& G, S F[5], int& fl) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const S rl = L[0], ul = L[1 + d], pl = L[4];
  const S rr = R[0], ur = R[1 + d], pr = R[4];
  const S cl = sqrt_phys(G.gamma * pl * rl);
  const S cr = sqrt_phys(G.gamma * pr * rr);
  S p = qdiv((cr * pl + cl * pr) + (cl * cr) * (ul - ur), cl + cr);
  if (p < G.small_pres) fl |= PPM_FLAG_FLOOR;
  p = smax(p, G.small_pres);
  const S ipl = qdiv(ONE, pl), ipr = qdiv(ONE, pr);
  for (int it = 0; it < G.iters; ++it) {
    const S wl = cl * sqrt_wave(ONE + G.beta * (p * ipl - ONE));
    const S wr = cr * sqrt_wave(ONE + G.beta * (p * ipr - ONE));
    S iwl, iwr;
    pair_recip(wl, wr, iwl, iwr);
    const S xl = cl * iwl, xr = cr * iwr;
    const S izl = HALF * iwl * (ONE + xl * xl);
    const S izr = HALF * iwr * (ONE + xr * xr);
    const S usl = ul - (p - pl) * iwl;
    const S usr = ur + (p - pr) * iwr;
    p = p - qdiv(usr - usl, izl + izr);
    if (p < G.small_pres) fl |= PPM_FLAG_FLOOR;
    p = smax(p, G.small_pres);
  }
  const S wl = cl * sqrt_wave(ONE + G.beta * (p * ipl - ONE));
  const S wr = cr * sqrt_wave(ONE + G.beta * (p * ipr - ONE));
  S iwl, iwr;
  pair_recip(wl, wr, iwl, iwr);
  const S us = qdiv((wl * ul + wr * ur) + (pl - pr), wl + wr);

  S g0, g1, g2, g3, g4;
  if (us != S(0)) {
    const bool left = us > S(0);
    const S ro = left ? rl : rr;
    const S uo = left ? ul : -ur;
    const S po = left ? pl : pr;
    const S C = left ? cl : cr;
    const S W = left ? wl : wr;
    const S iW = left ? iwl : iwr;
    const S uss = left ? us : -us;
    S r_, u_, p_;
    sample_side(ro, uo, po, C, W, iW, uss, p, G, r_, u_, p_, fl);
    g0 = r_;
    g1 = left ? u_ : -u_;
    g2 = p_;
    g3 = left ? L[1 + t1] : R[1 + t1];
    g4 = left ? L[1 + t2] : R[1 + t2];
  } else {  // u* == 0: both sides averaged
    S ra, ua, pa, rb, ub, pb;
    sample_side(rl, ul, pl, cl, wl, iwl, us, p, G, ra, ua, pa, fl);
    sample_side(rr, -ur, pr, cr, wr, iwr, -us, p, G, rb, ub, pb, fl);
    ub = -ub;
    g0 = HALF * (ra + rb);
    g1 = HALF * (ua + ub);
    g2 = HALF * (pa + pb);
    g3 = HALF * (L[1 + t1] + R[1 + t1]);
    g4 = HALF * (L[1 + t2] + R[1 + t2]);
  }
  const S m = g0 * g1;
  const S e = g2 * G.gm1inv + HALF * g0 * ((g1 * g1 + g3 * g3) + g4 * g4);
  F[0] = m;
  F[1 + d] = m * g1 + g2;
  F[1 + t1] = m * g3;
  F[1 + t2] = m * g4;
  F[4] = g1 * (e + g2);
}

// ------------------------------------------------------------ O4: PPM ------
template <class S>
PPM_HD S ppm_slope(S am, S a0, S ap, int limiter) {
  const S dc = HALF * (ap - am);
  if (!limiter) return dc;
  const S dl = a0 - am, dr = ap - a0;
  // dl dr > 0 makes dc, dl and dr nonzero and finite (or infinite), so the
  // hardware min and the sign copy give the plain definition's value
  if (same_sign(dl, dr)) return scopysign(fmin2(fmin2(sabs(dc), TWO * sabs(dl)), TWO * sabs(dr)), dc);
  return S(0);
}

template <class S>
PPM_HD void ppm_parabola(S am2, S am1, S a0, S ap1, S ap2, S phi, const Gas<S>& G,
                                             S& aL, S& aR, S& a6) {
  const S sm = ppm_slope(am2, am1, a0, G.limiter);
  const S s0 = ppm_slope(am1, a0, ap1, G.limiter);
  const S sp = ppm_slope(a0, ap1, ap2, G.limiter);
  aL = HALF * (am1 + a0) - (s0 - sm) * SIXTH;
  aR = HALF * (a0 + ap1) - (sp - s0) * SIXTH;
  if (G.limiter) {
    if (G.flattening) {
      const S omp = ONE - phi;
      aL = phi * aL + omp * a0;
      aR = phi * aR + omp * a0;
    }
    if (!same_sign(aR - a0, a0 - aL)) {  // a0 is an extremum
      aL = a0;
      aR = a0;
    } else {
      bool hi, lo;
      cw_overshoot(aR - aL, a0 - HALF * (aL + aR), hi, lo);
      if (hi) {
        aL = THREE * a0 - TWO * aR;
      } else if (lo) {
        aR = THREE * a0 - TWO * aL;
      }
    }
  }
  a6 = SIX * a0 - THREE * (aL + aR);
}

template <class S> PPM_HD S ppm_ip(S aR, S da, S a6, S sg) {
  return aR - HALF * sg * (da - (ONE - TWO3 * sg) * a6);
}
template <class S> PPM_HD S ppm_im(S aL, S da, S a6, S sg) {
  return aL + HALF * sg * (da + (ONE - TWO3 * sg) * a6);
}

// ---------------------------------------------------------- O5: tracing ----
template <class S>
PPM_HD void trace_edge(const S ref[5], S a1, S a2, S a3, S at1, S at2, S cor, S c2,
                                           int mn, int m1, int m2, const Gas<S>& G, const S* hdtg,
                                           S q[5], int& fl) {
  q[0] = ref[0] - ((a1 + a3) + a2);
  q[mn] = ref[mn] + cor * (a1 - a3);
  q[4] = ref[4] - c2 * (a1 + a3);
  q[m1] = ref[m1] - at1;
  q[m2] = ref[m2] - at2;
  if (G.grav) {
    q[1] = q[1] + hdtg[0];
    q[2] = q[2] + hdtg[1];
    q[3] = q[3] + hdtg[2];
  }
  if (q[0] < G.small_dens) fl |= PPM_FLAG_FLOOR;
  if (q[4] < G.small_pres) fl |= PPM_FLAG_FLOOR;
  q[0] = smax(q[0], G.small_dens);
  q[4] = smax(q[4], G.small_pres);
}

template <int d, class S>
PPM_HD void trace_zone(const S aL[5], const S aR[5], const S a6[5], S r, S un, S c,
                                           S dtdx, const Gas<S>& G, const S* hdtg, S qp[5],
                                           S qm[5], int& fl) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  constexpr int mn = 1 + d, m1 = 1 + t1, m2 = 1 + t2;
  S da[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) da[m] = aR[m] - aL[m];
  const S rc = r * c, c2 = c * c, ic2 = qdiv(ONE, c2), hic2 = HALF * ic2, cor = qdiv(c, r);
  const S l1 = un - c, l2 = un, l3 = un + c;
  const S zero = S(0);
  {
    const S s1 = smax(l1, zero) * dtdx, s2 = smax(l2, zero) * dtdx, s3 = smax(l3, zero) * dtdx;
    S ref[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) ref[m] = ppm_ip(aR[m], da[m], a6[m], s3);
    S a1 = zero, a2 = zero, a3 = zero, at1 = zero, at2 = zero;
    if (l1 > zero) {
      const S dp = ref[4] - ppm_ip(aR[4], da[4], a6[4], s1);
      const S du = ref[mn] - ppm_ip(aR[mn], da[mn], a6[mn], s1);
      a1 = (dp - rc * du) * hic2;
    }
    if (l2 > zero) {
      const S dr = ref[0] - ppm_ip(aR[0], da[0], a6[0], s2);
      const S dp = ref[4] - ppm_ip(aR[4], da[4], a6[4], s2);
      a2 = dr - dp * ic2;
      at1 = ref[m1] - ppm_ip(aR[m1], da[m1], a6[m1], s2);
      at2 = ref[m2] - ppm_ip(aR[m2], da[m2], a6[m2], s2);
    }
    if (l3 > zero) {
      const S dp = ref[4] - ppm_ip(aR[4], da[4], a6[4], s3);
      const S du = ref[mn] - ppm_ip(aR[mn], da[mn], a6[mn], s3);
      a3 = (dp + rc * du) * hic2;
    }
    trace_edge(ref, a1, a2, a3, at1, at2, cor, c2, mn, m1, m2, G, hdtg, qp, fl);
  }
  {
    const S s1 = smax(-l1, zero) * dtdx, s2 = smax(-l2, zero) * dtdx, s3 = smax(-l3, zero) * dtdx;
    S ref[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) ref[m] = ppm_im(aL[m], da[m], a6[m], s1);
    S a1 = zero, a2 = zero, a3 = zero, at1 = zero, at2 = zero;
    if (l1 < zero) {
      const S dp = ref[4] - ppm_im(aL[4], da[4], a6[4], s1);
      const S du = ref[mn] - ppm_im(aL[mn], da[mn], a6[mn], s1);
      a1 = (dp - rc * du) * hic2;
    }
    if (l2 < zero) {
      const S dr = ref[0] - ppm_im(aL[0], da[0], a6[0], s2);
      const S dp = ref[4] - ppm_im(aL[4], da[4], a6[4], s2);
      a2 = dr - dp * ic2;
      at1 = ref[m1] - ppm_im(aL[m1], da[m1], a6[m1], s2);
      at2 = ref[m2] - ppm_im(aL[m2], da[m2], a6[m2], s2);
    }
    if (l3 < zero) {
      const S dp = ref[4] - ppm_im(aL[4], da[4], a6[4], s3);
      const S du = ref[mn] - ppm_im(aL[mn], da[mn], a6[mn], s3);
      a3 = (dp + rc * du) * hic2;
    }
    trace_edge(ref, a1, a2, a3, at1, at2, cor, c2, mn, m1, m2, G, hdtg, qm, fl);
  }
}

// ------------------------------------------------ conversions (O2, O8) -----
template <class S>
PPM_HD void prim_to_cons(const S q[5], const Gas<S>& G, S U[5]) {
  U[0] = q[0];
  U[1] = q[0] * q[1];
  U[2] = q[0] * q[2];
  U[3] = q[0] * q[3];
  U[4] = q[4] * G.gm1inv + HALF * q[0] * ((q[1] * q[1] + q[2] * q[2]) + q[3] * q[3]);
}

template <class S>
PPM_HD void cons_to_prim_floor(const S U[5], const Gas<S>& G, S q[5], int& fl) {
  if (U[0] < G.small_dens) fl |= PPM_FLAG_FLOOR;
  const S r = smax(U[0], G.small_dens);
  const S ir = qdiv(ONE, r);  // one division for the three velocities
  const S u = U[1] * ir, v = U[2] * ir, w = U[3] * ir;
  const S ke = HALF * r * ((u * u + v * v) + w * w);
  S p = G.gm1 * (U[4] - ke);
  if (p < G.small_pres) fl |= PPM_FLAG_FLOOR;
  p = smax(p, G.small_pres);
  q[0] = r; q[1] = u; q[2] = v; q[3] = w; q[4] = p;
}

}  // namespace ppm

/*
 * TEST INFRASTRUCTURE -- the oracle.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load this library; the product path never
 * does, and this file shares no code with the HIP path.
 *
 * Plain, serial CPU reference of one explicit unsplit Godunov step of the 3-D
 * gamma-law Euler equations on the rectangular boxes (FABs) of one level:
 * the compressible code's explicit update of a hyperbolic system of
 * conservation laws (paper Sec. 1), on the MultiFAB / FAB data model with
 * ghost cells filled from intersecting grids (paper Sec. 2).
 *
 * The paper names the advance but not its discretisation.  The reading used
 * here (stated step by step next to each function) is the classical one:
 *   O1  ghost fill: periodic images, outflow, reflecting walls
 *   O2  conserved -> primitive (rho, u, v, w, p), sound speed c
 *   O3  Colella-Woodward shock flattening (eps 0.33, omega1 0.75, omega2 10)
 *   O4  PPM parabolas, MC-limited slopes, CW84 monotonicity limiter
 *   O5  characteristic tracing with a reference state (fastest wave)
 *   O6  two-shock Riemann solver, fixed number of Newton iterations
 *   O7-O9  12-solve 3-D corner-transport-upwind: normal predictor,
 *       6 single-transverse corrections (dt/3h), 3 double corrections (dt/2h)
 *   O10 conservative flux-divergence update (+ Heun constant-gravity source)
 *   O11 CFL time step from the per-axis maximum signal speed
 *   S1-S3 passive species (optional): each mass fraction X = (rho X)/rho is
 *       reconstructed like a primitive variable, traced across the entropy
 *       wave only (as a transverse velocity), carried through the three
 *       stages by the stage's mass flux from the side the mass comes from,
 *       corrected transversely like the density, and rho X updated
 *       conservatively in FP64.  The paper does not describe species; this
 *       is the usual passive-scalar extension of the same advance.
 * Every formula is the method's definition written out as it stands: each
 * quotient is a division, each root a square root, no reciprocal is shared
 * between formulas.  The order of evaluation is the one C defines (left to
 * right, no contraction, IEEE division and sqrt).  The GPU kernels evaluate
 * algebraically equal forms with fewer divisions, so the two agree to
 * rounding.
 *
 * Pins that tie this file to the method rather than to itself are in the
 * test suite: exact solutions (Sod, two-shock collisions, uniform flow,
 * uniform acceleration), invariants (conservation, mirror and axis
 * symmetries, planar data), convergence rates, hand-computed flattening
 * coefficients and CFL speeds, and hand counts of the operations of one
 * Riemann solve and one state conversion.
 *
 * The arithmetic is templated on the scalar type:
 *   double   - the FP64 reference
 *   float    - the FP32-reconstruction mode: O2..O9 in float, O10/O11 double
 *   Dual     - forward-mode tangent (exact Jacobian-vector product with the
 *              branch decisions taken on the primal values)
 *   DualF    - the same for the FP32-reconstruction mode: float primal
 *              (rounded exactly as the float mode), FP64 tangent
 *   Counted  - a double that counts its own floating-point operations
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <type_traits>

namespace {

// ------------------------------------------------------------------ scalars --
// Operation counters for the Counted scalar, one row per stage of the step.
enum { OP_ADD = 0, OP_MUL, OP_DIV, OP_SQRT, OP_CMP, OP_NKIND };
enum { ST_PRIM = 0, ST_FLAT, ST_TRACE, ST_RIEM1, ST_TRANS1, ST_RIEM2, ST_TRANS2,
       ST_RIEM3, ST_UPDATE, ST_NSTAGE };
uint64_t g_ops[ST_NSTAGE][OP_NKIND];
int g_stage = 0;

struct Counted {
  double v;
  Counted() : v(0) {}
  Counted(double x) : v(x) {}
};
inline Counted operator+(Counted a, Counted b) { g_ops[g_stage][OP_ADD]++; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { g_ops[g_stage][OP_ADD]++; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { g_ops[g_stage][OP_MUL]++; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { g_ops[g_stage][OP_DIV]++; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }

struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double t) : v(x), d(t) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }

// Primal in float, tangent in double: the derivative of the FP32 mode's
// piecewise-smooth step with its own (float) branch decisions.
struct DualF {
  float v;
  double d;
  DualF() : v(0), d(0) {}
  DualF(double x) : v((float)x), d(0) {}
  DualF(float x, double t) : v(x), d(t) {}
};
inline DualF operator+(DualF a, DualF b) { return DualF(a.v + b.v, a.d + b.d); }
inline DualF operator-(DualF a, DualF b) { return DualF(a.v - b.v, a.d - b.d); }
inline DualF operator*(DualF a, DualF b) { return DualF(a.v * b.v, a.d * (double)b.v + (double)a.v * b.d); }
inline DualF operator/(DualF a, DualF b) {
  const float q = a.v / b.v;
  return DualF(q, (a.d - (double)q * b.d) / (double)b.v);
}
inline DualF operator-(DualF a) { return DualF(-a.v, -a.d); }

inline double V(double x) { return x; }
inline double V(float x) { return x; }
inline double V(const Counted& x) { return x.v; }
inline double V(const Dual& x) { return x.v; }
inline double V(const DualF& x) { return (double)x.v; }

// max/min select an operand by value; the derivative follows the selection.
template <class S> inline S smax(S a, S b) {
  if (std::is_same<S, Counted>::value) g_ops[g_stage][OP_CMP]++;
  return (V(a) < V(b)) ? b : a;
}
template <class S> inline S smin(S a, S b) {
  if (std::is_same<S, Counted>::value) g_ops[g_stage][OP_CMP]++;
  return (V(b) < V(a)) ? b : a;
}
template <class S> inline S sabs(S a) { return (V(a) < 0) ? -a : a; }
// |m| carrying the sign of s (m >= 0 on every call site).
template <class S> inline S scopysign(S m, S s) { return std::signbit(V(s)) ? -m : m; }


inline double ssqrt(double x) { return std::sqrt(x); }
inline float ssqrt(float x) { return std::sqrt(x); }
inline Counted ssqrt(Counted x) { g_ops[g_stage][OP_SQRT]++; return Counted(std::sqrt(x.v)); }
inline Dual ssqrt(Dual x) {
  double r = std::sqrt(x.v);
  return Dual(r, x.d / (2.0 * r));
}
inline DualF ssqrt(DualF x) {
  const float r = std::sqrt(x.v);
  return DualF(r, x.d / (2.0 * (double)r));
}

// Conversion of the FP64 state into the reconstruction scalar and back.
template <class S, class A> inline S to_s(const A& a);
template <> inline double to_s<double, double>(const double& a) { return a; }
template <> inline float to_s<float, double>(const double& a) { return (float)a; }
template <> inline Counted to_s<Counted, Counted>(const Counted& a) { return a; }
template <> inline Dual to_s<Dual, Dual>(const Dual& a) { return a; }
template <> inline DualF to_s<DualF, Dual>(const Dual& a) { return DualF((float)a.v, a.d); }
template <class A, class S> inline A to_a(const S& s);
template <> inline double to_a<double, double>(const double& s) { return s; }
template <> inline double to_a<double, float>(const float& s) { return (double)s; }
template <> inline Counted to_a<Counted, Counted>(const Counted& s) { return s; }
template <> inline Dual to_a<Dual, Dual>(const Dual& s) { return s; }
template <> inline Dual to_a<Dual, DualF>(const DualF& s) { return Dual((double)s.v, s.d); }

// ------------------------------------------------------------- parameters --
struct OParams {
  double gamma, cfl, small_dens, small_pres;
  double grav[3];
  int limiter;        // 1: MC slopes + CW84 limiter (+ flattening); 0: unlimited
  int flattening;     // 1: shock flattening (only with limiter = 1)
  int riemann_iters;  // fixed number of Newton iterations in O6
  int precision;      // 0: FP64; 1: FP32 reconstruction / FP64 update
};

enum { FLAG_NONPHYS = 1, FLAG_FLOOR = 2 };
// BC_COARSE_FINE: the face borders a coarser level; ghost zones beyond it
// are filled by interpolation from that level, not by the level's own fill.
// BC_INFLOW: ghost zones beyond the face hold a prescribed state (inflow).
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_COARSE_FINE = 3, BC_INFLOW = 4 };
const int NG = 4;  // ghost width: flattening reaches 3 zones past a traced zone

// a b > 0: the sign tests of the MC slope and the CW84 limiter compare a
// product of two differences of one field with zero.
template <class S> inline bool pos_product(S a, S b) { return V(a * b) > 0; }

// Per-step constants in the reconstruction scalar.  They are formed in FP64
// from gamma, dt and h, then rounded to S once.
template <class S> struct Consts {
  S gamma, gm1, beta, small_dens, small_pres;
  S dtdx[3], dt2h[3], dt3h[3], hdtg[3];
  S half, one, two, three, six, two3, c033, ten, c075;
  bool grav;
  int limiter, flattening, iters;
};
template <class S>
Consts<S> make_consts(const OParams& P, double dt, const double h[3]) {
  Consts<S> K;
  K.gamma = S(P.gamma);
  K.gm1 = S(P.gamma - 1.0);
  K.beta = S((P.gamma + 1.0) / (2.0 * P.gamma));
  K.small_dens = S(P.small_dens);
  K.small_pres = S(P.small_pres);
  for (int d = 0; d < 3; ++d) {
    K.dtdx[d] = S(dt / h[d]);
    K.dt2h[d] = S(dt / (2.0 * h[d]));
    K.dt3h[d] = S(dt / (3.0 * h[d]));
    K.hdtg[d] = S(0.5 * dt * P.grav[d]);
  }
  K.half = S(0.5); K.one = S(1.0); K.two = S(2.0); K.three = S(3.0); K.six = S(6.0);
  K.two3 = S(2.0 / 3.0); K.c033 = S(0.33); K.ten = S(10.0);
  K.c075 = S(0.75);
  K.grav = (P.grav[0] != 0.0 || P.grav[1] != 0.0 || P.grav[2] != 0.0);
  K.limiter = P.limiter;
  K.flattening = P.flattening && P.limiter;
  K.iters = P.riemann_iters;
  return K;
}

// ------------------------------------------------- O6: two-shock Riemann ----
// Godunov flux at a face normal to axis d from the left state L and the right
// state R (primitive, xyz order: rho, u, v, w, p).
//
// Two-shock approximation (Colella-Woodward 1984 Sec. 2, Colella-Glaz 1985):
// both nonlinear waves follow the shock Hugoniot.  With the Lagrangian sound
// speed C_s = sqrt(gamma p_s rho_s) of side s, a wave of post-wave pressure p
// moves with the Lagrangian speed
//   W_s(p) = C_s sqrt(1 + beta (p/p_s - 1)),   beta = (gamma + 1)/(2 gamma),
// and leaves the velocity u*_L = u_L - (p - p_L)/W_L behind it on the left,
// u*_R = u_R + (p - p_R)/W_R on the right.  The star pressure makes the two
// agree; it is found by a fixed number of Newton steps from the acoustic
// guess, each branch's slope |dp/du*_s| taken as Z_s = 2 W_s^3/(W_s^2 + C_s^2).
// Each quantity below is that formula written out as it stands.
template <class S>
void riemann(const S L[5], const S R[5], int d, const Consts<S>& K, S F[5], int& flags) {
  const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const S rl = L[0], ul = L[1 + d], pl = L[4], vl1 = L[1 + t1], vl2 = L[1 + t2];
  const S rr = R[0], ur = R[1 + d], pr = R[4], vr1 = R[1 + t1], vr2 = R[1 + t2];

  const S cl = ssqrt(K.gamma * pl * rl);
  const S cr = ssqrt(K.gamma * pr * rr);
  // acoustic (linearised) guess
  S p = ((cr * pl + cl * pr) + (cl * cr) * (ul - ur)) / (cl + cr);
  if (V(p) < V(K.small_pres)) flags |= FLAG_FLOOR;
  p = smax(p, K.small_pres);
  auto wave_speed = [&](S c, S ps) { return c * ssqrt(K.one + K.beta * (p / ps - K.one)); };
  for (int it = 0; it < K.iters; ++it) {
    const S wl = wave_speed(cl, pl);
    const S wr = wave_speed(cr, pr);
    const S zl = K.two * wl * wl * wl / (wl * wl + cl * cl);
    const S zr = K.two * wr * wr * wr / (wr * wr + cr * cr);
    const S usl = ul - (p - pl) / wl;
    const S usr = ur + (p - pr) / wr;
    p = p - zl * zr * (usr - usl) / (zl + zr);
    if (V(p) < V(K.small_pres)) flags |= FLAG_FLOOR;
    p = smax(p, K.small_pres);
  }
  const S wl = wave_speed(cl, pl);
  const S wr = wave_speed(cr, pr);
  const S us = ((wl * ul + wr * ur) + (pl - pr)) / (wl + wr);

  // Sample the wave fan at x/t = 0 on one side of the contact.  Outer state:
  // the side's input; star state: (rho*_s, u*, p*) with rho* from the Hugoniot
  // 1/rho* = 1/rho_s - (p* - p_s)/W_s^2 (floored at small_dens, also when the
  // right-hand side is not positive).  A shock is a single jump at speed
  // u_s -/+ W_s/rho_s; a rarefaction is a linear fan between its head
  // (u_s -/+ c_s, c_s = sqrt(gamma p_s/rho_s)) and tail (u* -/+ c*_s,
  // c*_s = sqrt(gamma p*/rho*_s)).
  auto star_density = [&](S rs_, S ps, S ws) {
    const S vstar = K.one / rs_ - (p - ps) / (ws * ws);
    S rs = K.one / vstar;
    if (!(V(vstar) > 0) || V(rs) < V(K.small_dens)) { flags |= FLAG_FLOOR; rs = K.small_dens; }
    return rs;
  };
  auto sample_left = [&](S st[5]) {
    const S rs = star_density(rl, pl, wl);
    const S cst = ssqrt(K.gamma * p / rs);
    const S co = ssqrt(K.gamma * pl / rl);
    S r_ = rl, u_ = ul, p_ = pl;  // outer
    if (V(p) > V(pl)) {
      const S sh = ul - wl / rl;
      if (!(V(sh) >= 0)) { r_ = rs; u_ = us; p_ = p; }
    } else {
      const S hd = ul - co, tl = us - cst;
      if (V(hd) >= 0) {
      } else if (V(tl) <= 0) {
        r_ = rs; u_ = us; p_ = p;
      } else {
        const S w = -hd / (tl - hd);
        r_ = (K.one - w) * rl + w * rs;
        u_ = (K.one - w) * ul + w * us;
        p_ = (K.one - w) * pl + w * p;
      }
    }
    st[0] = r_; st[1] = u_; st[2] = p_; st[3] = vl1; st[4] = vl2;
  };
  auto sample_right = [&](S st[5]) {
    const S rs = star_density(rr, pr, wr);
    const S cst = ssqrt(K.gamma * p / rs);
    const S co = ssqrt(K.gamma * pr / rr);
    S r_ = rr, u_ = ur, p_ = pr;
    if (V(p) > V(pr)) {
      const S sh = ur + wr / rr;
      if (!(V(sh) <= 0)) { r_ = rs; u_ = us; p_ = p; }
    } else {
      const S hd = ur + co, tl = us + cst;
      if (V(hd) <= 0) {
      } else if (V(tl) >= 0) {
        r_ = rs; u_ = us; p_ = p;
      } else {
        const S w = hd / (hd - tl);
        r_ = (K.one - w) * rr + w * rs;
        u_ = (K.one - w) * ur + w * us;
        p_ = (K.one - w) * pr + w * p;
      }
    }
    st[0] = r_; st[1] = u_; st[2] = p_; st[3] = vr1; st[4] = vr2;
  };
  S g[5];  // Godunov state in the rotated frame: rho, u_n, p, u_t1, u_t2
  if (V(us) > 0) {
    sample_left(g);
  } else if (V(us) < 0) {
    sample_right(g);
  } else {  // u* == 0: both sides, averaged (keeps exact mirror symmetry)
    S a[5], b[5];
    sample_left(a);
    sample_right(b);
    for (int m = 0; m < 5; ++m) g[m] = K.half * (a[m] + b[m]);
  }
  // Euler flux of the Godunov state, rotated back to xyz component order.
  const S m = g[0] * g[1];
  const S e = g[2] / K.gm1 + K.half * g[0] * ((g[1] * g[1] + g[3] * g[3]) + g[4] * g[4]);
  F[0] = m;
  F[1 + d] = m * g[1] + g[2];
  F[1 + t1] = m * g[3];
  F[1 + t2] = m * g[4];
  F[4] = g[1] * (e + g[2]);
}

// -------------------------------------------------- O4: PPM parabola -------
// Slope of a at zone i from a[i-1], a[i], a[i+1]: the centred difference,
// limited by twice the one-sided differences (van Leer / MC; CW84 eq. 1.8),
// zero at an extremum.
template <class S>
S ppm_slope(S am, S a0, S ap, const Consts<S>& K) {
  const S dc = K.half * (ap - am);
  if (!K.limiter) return dc;
  const S dl = a0 - am, dr = ap - a0;
  if (pos_product(dl, dr)) return scopysign(smin(smin(sabs(dc), K.two * sabs(dl)), K.two * sabs(dr)), dc);
  return S(0.0);
}

// Parabola in zone i from a[i-2..i+2] (CW84 Sec. 1): edge values
//   a_{i+1/2} = (a_i + a_{i+1})/2 - (delta_{i+1} - delta_i)/6,
// blended toward the cell value by the flattening coefficient phi, then
// the CW84 monotonicity limiter; returns (aL, aR, a6).
template <class S>
void ppm_parabola(const S a[5], S phi, const Consts<S>& K, S& aL, S& aR, S& a6) {
  const S sm = ppm_slope(a[0], a[1], a[2], K);
  const S s0 = ppm_slope(a[1], a[2], a[3], K);
  const S sp = ppm_slope(a[2], a[3], a[4], K);
  const S a0 = a[2];
  aL = K.half * (a[1] + a0) - (s0 - sm) / K.six;
  aR = K.half * (a0 + a[3]) - (sp - s0) / K.six;
  if (K.limiter) {
    if (K.flattening) {
      const S omp = K.one - phi;
      aL = phi * aL + omp * a0;
      aR = phi * aR + omp * a0;
    }
    // a0 is an extremum when (aR - a0)(a0 - aL) <= 0; otherwise the
    // parabola overshoots an edge when dq (a0 - mid) > dq^2/6 (or
    // < -dq^2/6), dq = aR - aL, mid = (aL + aR)/2.
    if (!pos_product(aR - a0, a0 - aL)) {
      aL = a0;
      aR = a0;
    } else {
      const S dq = aR - aL;
      const S m = a0 - K.half * (aL + aR);
      const S t = dq * m;
      const S d2 = dq * dq / K.six;
      if (V(t) > V(d2)) {
        aL = K.three * a0 - K.two * aR;
      } else if (V(-d2) > V(t)) {
        aR = K.three * a0 - K.two * aL;
      }
    }
  }
  a6 = K.six * a0 - K.three * (aL + aR);
}

// Averages of the parabola over the domain of dependence of the high face
// (I+) and the low face (I-) for a Courant number sigma >= 0.
template <class S> inline S ppm_ip(S aR, S da, S a6, S sigma, const Consts<S>& K) {
  return aR - K.half * sigma * (da - (K.one - K.two3 * sigma) * a6);
}
template <class S> inline S ppm_im(S aL, S da, S a6, S sigma, const Consts<S>& K) {
  return aL + K.half * sigma * (da + (K.one - K.two3 * sigma) * a6);
}

// ---------------------------------------------- O5: characteristic tracing --
// Time-centred states on the high face (qp) and low face (qm) of a zone along
// axis d.  Reference state: the parabola average swept by the fastest wave
// moving toward the face; every other wave that reaches the face removes its
// projection of (reference - its own average) with the primitive left
// eigenvectors at the cell centre (rho, c, u_n).  Waves moving away add nothing.
template <class S>
void trace_zone(const S aL[5], const S aR[5], const S a6[5], const S cell[6], int d,
                const Consts<S>& K, S qp[5], S qm[5], int& flags) {
  const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const int mn = 1 + d, m1 = 1 + t1, m2 = 1 + t2;
  S da[5];
  for (int m = 0; m < 5; ++m) da[m] = aR[m] - aL[m];
  const S r = cell[0], un = cell[1 + d], c = cell[5];
  const S rc = r * c, c2 = c * c;
  const S lam[3] = {un - c, un, un + c};
  const S zero(0.0);

  auto edge = [&](const S ref[5], S a1, S a2, S a3, S at1, S at2, S q[5]) {
    q[0] = ref[0] - ((a1 + a3) + a2);
    q[mn] = ref[mn] + c / r * (a1 - a3);
    q[4] = ref[4] - c2 * (a1 + a3);
    q[m1] = ref[m1] - at1;
    q[m2] = ref[m2] - at2;
    if (K.grav)
      for (int k = 0; k < 3; ++k) q[1 + k] = q[1 + k] + K.hdtg[k];
    if (V(q[0]) < V(K.small_dens)) flags |= FLAG_FLOOR;
    if (V(q[4]) < V(K.small_pres)) flags |= FLAG_FLOOR;
    q[0] = smax(q[0], K.small_dens);
    q[4] = smax(q[4], K.small_pres);
  };

  {  // high face: waves with lambda > 0
    S sg[3];
    for (int k = 0; k < 3; ++k) sg[k] = smax(lam[k], zero) * K.dtdx[d];
    S ref[5];
    for (int m = 0; m < 5; ++m) ref[m] = ppm_ip(aR[m], da[m], a6[m], sg[2], K);
    S a1 = zero, a2 = zero, a3 = zero, at1 = zero, at2 = zero;
    if (V(lam[0]) > 0) {
      const S dp = ref[4] - ppm_ip(aR[4], da[4], a6[4], sg[0], K);
      const S du = ref[mn] - ppm_ip(aR[mn], da[mn], a6[mn], sg[0], K);
      a1 = (dp - rc * du) / (K.two * c2);
    }
    if (V(lam[1]) > 0) {
      const S dr = ref[0] - ppm_ip(aR[0], da[0], a6[0], sg[1], K);
      const S dp = ref[4] - ppm_ip(aR[4], da[4], a6[4], sg[1], K);
      a2 = dr - dp / c2;
      at1 = ref[m1] - ppm_ip(aR[m1], da[m1], a6[m1], sg[1], K);
      at2 = ref[m2] - ppm_ip(aR[m2], da[m2], a6[m2], sg[1], K);
    }
    if (V(lam[2]) > 0) {
      const S dp = ref[4] - ppm_ip(aR[4], da[4], a6[4], sg[2], K);
      const S du = ref[mn] - ppm_ip(aR[mn], da[mn], a6[mn], sg[2], K);
      a3 = (dp + rc * du) / (K.two * c2);
    }
    edge(ref, a1, a2, a3, at1, at2, qp);
  }
  {  // low face: waves with lambda < 0
    S sg[3];
    for (int k = 0; k < 3; ++k) sg[k] = smax(-lam[k], zero) * K.dtdx[d];
    S ref[5];
    for (int m = 0; m < 5; ++m) ref[m] = ppm_im(aL[m], da[m], a6[m], sg[0], K);
    S a1 = zero, a2 = zero, a3 = zero, at1 = zero, at2 = zero;
    if (V(lam[0]) < 0) {
      const S dp = ref[4] - ppm_im(aL[4], da[4], a6[4], sg[0], K);
      const S du = ref[mn] - ppm_im(aL[mn], da[mn], a6[mn], sg[0], K);
      a1 = (dp - rc * du) / (K.two * c2);
    }
    if (V(lam[1]) < 0) {
      const S dr = ref[0] - ppm_im(aL[0], da[0], a6[0], sg[1], K);
      const S dp = ref[4] - ppm_im(aL[4], da[4], a6[4], sg[1], K);
      a2 = dr - dp / c2;
      at1 = ref[m1] - ppm_im(aL[m1], da[m1], a6[m1], sg[1], K);
      at2 = ref[m2] - ppm_im(aL[m2], da[m2], a6[m2], sg[1], K);
    }
    if (V(lam[2]) < 0) {
      const S dp = ref[4] - ppm_im(aL[4], da[4], a6[4], sg[2], K);
      const S du = ref[mn] - ppm_im(aL[mn], da[mn], a6[mn], sg[2], K);
      a3 = (dp + rc * du) / (K.two * c2);
    }
    edge(ref, a1, a2, a3, at1, at2, qm);
  }
}

// ----------------------------------------------------------- O2 and cons ---
// Conserved (rho, rho u, rho v, rho w, rho E) -> primitive (rho, u, v, w, p)
// and c = sqrt(gamma p / rho) for the gamma law p = (gamma-1)(rho E - rho|u|^2/2).
template <class S>
void cons_to_prim_cell(const S U[5], const Consts<S>& K, S q[6], int& flags) {
  const S r = U[0];
  const S u = U[1] / r, v = U[2] / r, w = U[3] / r;
  const S ke = K.half * r * ((u * u + v * v) + w * w);
  S p = K.gm1 * (U[4] - ke);
  bool fin = true;
  for (int m = 0; m < 5; ++m) fin = fin && std::isfinite(V(U[m]));
  if (!fin || !(V(r) > 0) || !(V(p) > 0)) flags |= FLAG_NONPHYS;
  if (V(p) < V(K.small_pres)) flags |= FLAG_FLOOR;
  p = smax(p, K.small_pres);
  q[0] = r; q[1] = u; q[2] = v; q[3] = w; q[4] = p;
  q[5] = ssqrt(K.gamma * p / r);
}

// Primitive from a corrected conserved state (O8/O9) with density and
// pressure floors.
template <class S>
void cons_to_prim_floor(const S U[5], const Consts<S>& K, S q[5], int& flags) {
  if (V(U[0]) < V(K.small_dens)) flags |= FLAG_FLOOR;
  const S r = smax(U[0], K.small_dens);
  const S u = U[1] / r, v = U[2] / r, w = U[3] / r;
  const S ke = K.half * r * ((u * u + v * v) + w * w);
  S p = K.gm1 * (U[4] - ke);
  if (V(p) < V(K.small_pres)) flags |= FLAG_FLOOR;
  p = smax(p, K.small_pres);
  q[0] = r; q[1] = u; q[2] = v; q[3] = w; q[4] = p;
}

template <class S>
void prim_to_cons(const S q[5], const Consts<S>& K, S U[5]) {
  U[0] = q[0];
  U[1] = q[0] * q[1];
  U[2] = q[0] * q[2];
  U[3] = q[0] * q[3];
  U[4] = q[4] / K.gm1 + K.half * q[0] * ((q[1] * q[1] + q[2] * q[2]) + q[3] * q[3]);
}

// ------------------------------------------------------------ 3-D arrays ---
template <class T> struct Grid {
  int lo[3] = {0, 0, 0}, n[3] = {0, 0, 0};
  std::vector<T> a;
  void init(const int l[3], const int h[3]) {
    size_t tot = 1;
    for (int d = 0; d < 3; ++d) { lo[d] = l[d]; n[d] = h[d] - l[d] + 1; tot *= (size_t)n[d]; }
    a.assign(tot, T(0.0));
  }
  T& at(const int x[3]) {
    return a[((size_t)(x[2] - lo[2]) * n[1] + (size_t)(x[1] - lo[1])) * n[0] + (size_t)(x[0] - lo[0])];
  }
};

// Calls f(x) for every zone x in [lo, hi] (inclusive), x fastest.
template <class Fn> void for_region(const int lo[3], const int hi[3], Fn f) {
  int x[3];
  for (x[2] = lo[2]; x[2] <= hi[2]; ++x[2])
    for (x[1] = lo[1]; x[1] <= hi[1]; ++x[1])
      for (x[0] = lo[0]; x[0] <= hi[0]; ++x[0]) f(x);
}

// ------------------------------------------------------- the step (O2-O10) --
// One box: U holds the 5 conserved fields with 4 ghost zones on each side,
// ghosts already filled (O1), layout [comp][k][j][i] over (n+8)^3.  The new
// state is produced on the window [wlo, whi] of valid zones (the whole box
// for a full step; a sub-window reproduces exactly the same values there,
// since every intermediate is recomputed from the input on the window's
// domain of dependence).
template <class S, class A>
struct Step {
  const A* U;
  int n[3], N[3];
  const OParams* P;
  double dt, h[3];
  Consts<S> K;
  int flags = 0;
  // faces of the box on a reflecting domain boundary: wall[2d] low, [2d+1] high
  int wall[6] = {0, 0, 0, 0, 0, 0};
  // passive species: ns partial densities rho X_s, layout [s][k][j][i] over
  // the stored grid like U; null / 0: none
  const A* RX = nullptr;
  int ns = 0;
  A* RXnew = nullptr;
  // non-null: stop after O3 and write the flattening coefficient of the
  // traced zones of the window here
  double* phi_out = nullptr;

  const A& rx_at(int s, const int x[3]) const {
    return RX[(((size_t)s * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)];
  }

  // S2: passive scalar carried by a face's mass flux: it takes the mass
  // fraction of the side the mass comes from (a zero flux carries nothing,
  // whichever side is taken; on a wall face the mirror states make the mass
  // flux exactly zero, so no species crosses a wall).
  static S carried(S frho, S xl, S xr) { return (V(frho) > 0) ? frho * xl : frho * xr; }

  // Riemann problem on a reflecting wall (R14): the state outside the wall
  // is the mirror image of the state inside it (normal velocity negated), so
  // the solve gives u* = 0 — no mass or energy crosses the wall, only the
  // pressure acts on it — whatever the traced ghost states hold (the gravity
  // shift of the traced velocities is not mirror-symmetric).
  void wall_states(int d, const int x[3], S L[5], S R[5]) const {
    if (wall[2 * d] && x[d] == 0) {
      for (int m = 0; m < 5; ++m) L[m] = R[m];
      L[1 + d] = -R[1 + d];
    } else if (wall[2 * d + 1] && x[d] == n[d]) {
      for (int m = 0; m < 5; ++m) R[m] = L[m];
      R[1 + d] = -L[1 + d];
    }
  }

  const A& u_at(int c, const int x[3]) const {
    return U[(((size_t)c * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)];
  }

  int run(const int wlo[3], const int whi[3], A* Unew, A* Fout[3], bool counting) {
    auto stage = [&](int s) { if (counting) g_stage = s; };
    int glo[3], ghi[3], plo[3], phi_[3];
    for (int d = 0; d < 3; ++d) {
      glo[d] = wlo[d] - 1; ghi[d] = whi[d] + 1;   // traced zones
      plo[d] = wlo[d] - NG; phi_[d] = whi[d] + NG; // primitive zones
    }
    // O2: primitive variables on the whole domain of dependence
    stage(ST_PRIM);
    Grid<S> q[6];
    for (int m = 0; m < 6; ++m) q[m].init(plo, phi_);
    for_region(plo, phi_, [&](const int x[3]) {
      S uc[5], qc[6];
      for (int c = 0; c < 5; ++c) uc[c] = to_s<S, A>(u_at(c, x));
      cons_to_prim_cell(uc, K, qc, flags);
      for (int m = 0; m < 6; ++m) q[m].at(x) = qc[m];
    });

    // O3: flattening coefficient on the traced zones
    stage(ST_FLAT);
    Grid<S> flat;
    flat.init(glo, ghi);
    for_region(glo, ghi, [&](const int x[3]) {
      S phi = K.one;
      if (K.flattening) {
        for (int d = 0; d < 3; ++d) {
          auto Q = [&](int m, int o) {
            int y[3] = {x[0], x[1], x[2]};
            y[d] += o;
            return q[m].at(y);
          };
          // shock-detector coefficient at offset o along d
          auto chit = [&](int o) {
            const S dp1 = Q(4, o + 1) - Q(4, o - 1);
            const S dp2 = Q(4, o + 2) - Q(4, o - 2);
            const S zeta = sabs(dp1) / smax(sabs(dp2), K.small_pres);
            const S z = smin(smax(K.ten * (zeta - K.c075), S(0.0)), K.one);
            const bool compress = V(Q(1 + d, o - 1) - Q(1 + d, o + 1)) > 0;
            const bool strong = V(sabs(dp1)) > V(K.c033 * smin(Q(4, o + 1), Q(4, o - 1)));
            return (compress && strong) ? z : S(0.0);
          };
          const S dp1 = Q(4, 1) - Q(4, -1);
          S chi;
          if (V(dp1) > 0) chi = smax(chit(0), chit(-1));
          else if (V(dp1) < 0) chi = smax(chit(0), chit(1));
          else chi = smax(smax(chit(-1), chit(0)), chit(1));
          phi = (d == 0) ? (K.one - chi) : smin(phi, K.one - chi);
        }
      }
      flat.at(x) = phi;
    });
    if (phi_out) {  // O3 alone: the coefficient over the traced zones, x fastest
      size_t i = 0;
      for_region(glo, ghi, [&](const int x[3]) { phi_out[i++] = V(flat.at(x)); });
      return flags;
    }

    // O4 + O5: parabolas and traced edge states on the traced zones
    stage(ST_TRACE);
    Grid<S> tp[3][5], tm[3][5];  // tp: high-face state, tm: low-face state
    for (int d = 0; d < 3; ++d)
      for (int m = 0; m < 5; ++m) { tp[d][m].init(glo, ghi); tm[d][m].init(glo, ghi); }
    for_region(glo, ghi, [&](const int x[3]) {
      S cell[6];
      for (int m = 0; m < 6; ++m) cell[m] = q[m].at(x);
      for (int d = 0; d < 3; ++d) {
        S aL[5], aR[5], a6[5];
        for (int m = 0; m < 5; ++m) {
          S st[5];
          for (int o = -2; o <= 2; ++o) {
            int y[3] = {x[0], x[1], x[2]};
            y[d] += o;
            st[o + 2] = q[m].at(y);
          }
          ppm_parabola(st, flat.at(x), K, aL[m], aR[m], a6[m]);
        }
        S qp[5], qm[5];
        trace_zone(aL, aR, a6, cell, d, K, qp, qm, flags);
        for (int m = 0; m < 5; ++m) { tp[d][m].at(x) = qp[m]; tm[d][m].at(x) = qm[m]; }
      }
    });

    // Face slot convention: slot x along d holds the face between zones
    // x - e_d and x.  Face ranges below are the domain of dependence of the
    // window.
    auto shifted = [](const int x[3], int d, int o, int y[3]) {
      y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; y[d] += o;
    };

    // O7: normal predictor fluxes F^d on d-faces with both transverse indices
    // on the traced range.
    stage(ST_RIEM1);
    Grid<S> f1[3][5];
    for (int d = 0; d < 3; ++d) {
      for (int m = 0; m < 5; ++m) f1[d][m].init(glo, ghi);
      int lo[3] = {glo[0], glo[1], glo[2]}, hi[3] = {ghi[0], ghi[1], ghi[2]};
      lo[d] = wlo[d]; hi[d] = whi[d] + 1;
      for_region(lo, hi, [&](const int x[3]) {
        int y[3];
        shifted(x, d, -1, y);
        S L[5], R[5], F[5];
        for (int m = 0; m < 5; ++m) { L[m] = tp[d][m].at(y); R[m] = tm[d][m].at(x); }
        wall_states(d, x, L, R);
        riemann(L, R, d, K, F, flags);
        for (int m = 0; m < 5; ++m) f1[d][m].at(x) = F[m];
      });
    }

    // O8: edge states of axis d corrected by the transverse flux difference
    // along t (factor dt/3h_t, conserved form), then the fluxes F^{d|t}.
    Grid<S> f2[3][3][5];
    for (int d = 0; d < 3; ++d)
      for (int t = 0; t < 3; ++t) {
        if (t == d) continue;
        const int r = 3 - d - t;
        for (int m = 0; m < 5; ++m) f2[d][t][m].init(glo, ghi);
        auto corrected = [&](Grid<S>* tr, const int z[3], S qo[5]) {
          S qe[5], ue[5];
          for (int m = 0; m < 5; ++m) qe[m] = tr[m].at(z);
          prim_to_cons(qe, K, ue);
          int zp[3];
          shifted(z, t, 1, zp);
          for (int m = 0; m < 5; ++m)
            ue[m] = ue[m] - K.dt3h[t] * (f1[t][m].at(zp) - f1[t][m].at(z));
          cons_to_prim_floor(ue, K, qo, flags);
        };
        int lo[3], hi[3];
        lo[d] = wlo[d]; hi[d] = whi[d] + 1;
        lo[t] = wlo[t]; hi[t] = whi[t];
        lo[r] = glo[r]; hi[r] = ghi[r];
        for_region(lo, hi, [&](const int x[3]) {
          int y[3];
          shifted(x, d, -1, y);
          S L[5], R[5], F[5];
          stage(ST_TRANS1);
          corrected(tp[d], y, L);
          corrected(tm[d], x, R);
          wall_states(d, x, L, R);
          stage(ST_RIEM2);
          riemann(L, R, d, K, F, flags);
          for (int m = 0; m < 5; ++m) f2[d][t][m].at(x) = F[m];
        });
      }

    // O9: edge states of axis d corrected by both transverse fluxes of the
    // second stage (factor dt/2h), then the final fluxes F^{d,n+1/2}.
    Grid<S> f3[3][5];
    for (int d = 0; d < 3; ++d) {
      const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
      for (int m = 0; m < 5; ++m) f3[d][m].init(glo, ghi);
      auto corrected = [&](Grid<S>* tr, const int z[3], S qo[5]) {
        S qe[5], ue[5];
        for (int m = 0; m < 5; ++m) qe[m] = tr[m].at(z);
        prim_to_cons(qe, K, ue);
        int z1[3], z2[3];
        shifted(z, t1, 1, z1);
        shifted(z, t2, 1, z2);
        for (int m = 0; m < 5; ++m)
          ue[m] = ue[m] - K.dt2h[t1] * (f2[t1][t2][m].at(z1) - f2[t1][t2][m].at(z))
                        - K.dt2h[t2] * (f2[t2][t1][m].at(z2) - f2[t2][t1][m].at(z));
        cons_to_prim_floor(ue, K, qo, flags);
      };
      int lo[3] = {wlo[0], wlo[1], wlo[2]}, hi[3] = {whi[0], whi[1], whi[2]};
      hi[d] = whi[d] + 1;
      for_region(lo, hi, [&](const int x[3]) {
        int y[3];
        shifted(x, d, -1, y);
        S L[5], R[5], F[5];
        stage(ST_TRANS2);
        corrected(tp[d], y, L);
        corrected(tm[d], x, R);
        wall_states(d, x, L, R);
        stage(ST_RIEM3);
        riemann(L, R, d, K, F, flags);
        for (int m = 0; m < 5; ++m) f3[d][m].at(x) = F[m];
      });
      // optional face-centred flux output, extents (n_d + 1) along d
      if (Fout && Fout[d]) {
        int fe[3] = {n[0], n[1], n[2]};
        fe[d] += 1;
        for_region(lo, hi, [&](const int x[3]) {
          for (int m = 0; m < 5; ++m)
            Fout[d][(((size_t)m * fe[2] + x[2]) * fe[1] + x[1]) * fe[0] + x[0]] =
                to_a<A, S>(f3[d][m].at(x));
        });
      }
    }

    // S1-S3, passive species (ns > 0): the same CTU sequence for each mass
    // fraction X = rho X / rho, carried by the mass fluxes of the three
    // stages.
    if (ns > 0) {
      // mass fractions on the primitive zones
      std::vector<Grid<S>> xq(ns);
      for (int sp = 0; sp < ns; ++sp) {
        xq[sp].init(plo, phi_);
        for_region(plo, phi_, [&](const int x[3]) { xq[sp].at(x) = to_s<S, A>(rx_at(sp, x)) / q[0].at(x); });
      }
      // traced mass fractions: PPM parabola (same limiter and flattening),
      // reference state of the fastest wave toward the face, corrected by
      // the entropy wave when it moves toward the face (as the transverse
      // velocities)
      std::vector<Grid<S>> xp(3 * ns), xm(3 * ns);
      for (int i = 0; i < 3 * ns; ++i) { xp[i].init(glo, ghi); xm[i].init(glo, ghi); }
      for_region(glo, ghi, [&](const int x[3]) {
        const S c = q[5].at(x);
        for (int d = 0; d < 3; ++d) {
          const S un = q[1 + d].at(x);
          const S lam[3] = {un - c, un, un + c};
          const S zero(0.0);
          S sgp[3], sgm[3];
          for (int k = 0; k < 3; ++k) {
            sgp[k] = smax(lam[k], zero) * K.dtdx[d];
            sgm[k] = smax(-lam[k], zero) * K.dtdx[d];
          }
          for (int sp = 0; sp < ns; ++sp) {
            S st[5], aL, aR, a6;
            for (int o = -2; o <= 2; ++o) {
              int y[3] = {x[0], x[1], x[2]};
              y[d] += o;
              st[o + 2] = xq[sp].at(y);
            }
            ppm_parabola(st, flat.at(x), K, aL, aR, a6);
            const S da = aR - aL;
            {
              const S ref = ppm_ip(aR, da, a6, sgp[2], K);
              const S at = (V(lam[1]) > 0) ? ref - ppm_ip(aR, da, a6, sgp[1], K) : zero;
              xp[d * ns + sp].at(x) = ref - at;
            }
            {
              const S ref = ppm_im(aL, da, a6, sgm[0], K);
              const S at = (V(lam[1]) < 0) ? ref - ppm_im(aL, da, a6, sgm[1], K) : zero;
              xm[d * ns + sp].at(x) = ref - at;
            }
          }
        }
      });
      // S2, stage 1: species fluxes of the normal predictor
      std::vector<Grid<S>> g1(3 * ns);
      for (int d = 0; d < 3; ++d) {
        int lo[3] = {glo[0], glo[1], glo[2]}, hi[3] = {ghi[0], ghi[1], ghi[2]};
        lo[d] = wlo[d]; hi[d] = whi[d] + 1;
        for (int sp = 0; sp < ns; ++sp) {
          g1[d * ns + sp].init(glo, ghi);
          for_region(lo, hi, [&](const int x[3]) {
            int y[3];
            shifted(x, d, -1, y);
            const S xl = xp[d * ns + sp].at(y), xr = xm[d * ns + sp].at(x);
            g1[d * ns + sp].at(x) = carried(f1[d][0].at(x), xl, xr);
          });
        }
      }
      // S2, stage 2: pair (d, t); corrected X = (rho X)/rho of the corrected
      // conserved pair, the density floored as in O8
      std::vector<Grid<S>> g2(9 * ns);
      for (int d = 0; d < 3; ++d)
        for (int t = 0; t < 3; ++t) {
          if (t == d) continue;
          const int r = 3 - d - t;
          int lo[3], hi[3];
          lo[d] = wlo[d]; hi[d] = whi[d] + 1;
          lo[t] = wlo[t]; hi[t] = whi[t];
          lo[r] = glo[r]; hi[r] = ghi[r];
          for (int sp = 0; sp < ns; ++sp) {
            Grid<S>& G2 = g2[(d * 3 + t) * ns + sp];
            G2.init(glo, ghi);
            auto corrected = [&](Grid<S>& rt, Grid<S>& xt, const int z[3]) {
              int zp[3];
              shifted(z, t, 1, zp);
              const S rho = smax(rt.at(z) - K.dt3h[t] * (f1[t][0].at(zp) - f1[t][0].at(z)), K.small_dens);
              const S rx = rt.at(z) * xt.at(z) - K.dt3h[t] * (g1[t * ns + sp].at(zp) - g1[t * ns + sp].at(z));
              return rx / rho;
            };
            for_region(lo, hi, [&](const int x[3]) {
              int y[3];
              shifted(x, d, -1, y);
              const S xl = corrected(tp[d][0], xp[d * ns + sp], y), xr = corrected(tm[d][0], xm[d * ns + sp], x);
                G2.at(x) = carried(f2[d][t][0].at(x), xl, xr);
            });
          }
        }
      // S2, stage 3, and S3: the update of rho X (FP64, x + y + z in that order)
      std::vector<Grid<S>> g3(3 * ns);
      for (int d = 0; d < 3; ++d) {
        const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
        int lo[3] = {wlo[0], wlo[1], wlo[2]}, hi[3] = {whi[0], whi[1], whi[2]};
        hi[d] = whi[d] + 1;
        for (int sp = 0; sp < ns; ++sp) {
          g3[d * ns + sp].init(glo, ghi);
          auto corrected = [&](Grid<S>& rt, Grid<S>& xt, const int z[3]) {
            int z1[3], z2[3];
            shifted(z, t1, 1, z1);
            shifted(z, t2, 1, z2);
            const S rho = smax(rt.at(z) - K.dt2h[t1] * (f2[t1][t2][0].at(z1) - f2[t1][t2][0].at(z))
                                        - K.dt2h[t2] * (f2[t2][t1][0].at(z2) - f2[t2][t1][0].at(z)),
                               K.small_dens);
            Grid<S>& a = g2[(t1 * 3 + t2) * ns + sp];
            Grid<S>& b = g2[(t2 * 3 + t1) * ns + sp];
            const S rx = rt.at(z) * xt.at(z) - K.dt2h[t1] * (a.at(z1) - a.at(z)) - K.dt2h[t2] * (b.at(z2) - b.at(z));
            return rx / rho;
          };
          for_region(lo, hi, [&](const int x[3]) {
            int y[3];
            shifted(x, d, -1, y);
            const S xl = corrected(tp[d][0], xp[d * ns + sp], y), xr = corrected(tm[d][0], xm[d * ns + sp], x);
            g3[d * ns + sp].at(x) = carried(f3[d][0].at(x), xl, xr);
          });
        }
      }
      const A dtdxs[3] = {A(dt / h[0]), A(dt / h[1]), A(dt / h[2])};
      for (int sp = 0; sp < ns; ++sp)
        for_region(wlo, whi, [&](const int x[3]) {
          int xp1[3], yp1[3], zp1[3];
          shifted(x, 0, 1, xp1);
          shifted(x, 1, 1, yp1);
          shifted(x, 2, 1, zp1);
          const A fx = to_a<A, S>(g3[0 * ns + sp].at(xp1)) - to_a<A, S>(g3[0 * ns + sp].at(x));
          const A fy = to_a<A, S>(g3[1 * ns + sp].at(yp1)) - to_a<A, S>(g3[1 * ns + sp].at(x));
          const A fz = to_a<A, S>(g3[2 * ns + sp].at(zp1)) - to_a<A, S>(g3[2 * ns + sp].at(x));
          RXnew[(((size_t)sp * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)] =
              rx_at(sp, x) - ((dtdxs[0] * fx + dtdxs[1] * fy) + dtdxs[2] * fz);
        });
    }

    // O10: conservative update, FP64, x + y + z in that order; then the
    // Heun constant-gravity source S(U) = (0, rho g, (rho u).g).
    stage(ST_UPDATE);
    const A dtdx[3] = {A(dt / h[0]), A(dt / h[1]), A(dt / h[2])};
    const bool grav = K.grav;
    const A g[3] = {A(P->grav[0]), A(P->grav[1]), A(P->grav[2])};
    const A adt(dt), hdt(0.5 * dt);
    for_region(wlo, whi, [&](const int x[3]) {
      int xp[3], yp[3], zp[3];
      shifted(x, 0, 1, xp);
      shifted(x, 1, 1, yp);
      shifted(x, 2, 1, zp);
      A un[5], uo[5];
      for (int m = 0; m < 5; ++m) {
        const A fx = to_a<A, S>(f3[0][m].at(xp)) - to_a<A, S>(f3[0][m].at(x));
        const A fy = to_a<A, S>(f3[1][m].at(yp)) - to_a<A, S>(f3[1][m].at(x));
        const A fz = to_a<A, S>(f3[2][m].at(zp)) - to_a<A, S>(f3[2][m].at(x));
        uo[m] = u_at(m, x);
        un[m] = uo[m] - ((dtdx[0] * fx + dtdx[1] * fy) + dtdx[2] * fz);
      }
      if (grav) {
        A s0[5], s1[5];
        auto src = [&](const A u[5], A s[5]) {
          s[0] = A(0.0);
          s[1] = u[0] * g[0];
          s[2] = u[0] * g[1];
          s[3] = u[0] * g[2];
          s[4] = (u[1] * g[0] + u[2] * g[1]) + u[3] * g[2];
        };
        src(uo, s0);
        for (int m = 1; m < 5; ++m) un[m] = un[m] + adt * s0[m];
        src(un, s1);
        for (int m = 1; m < 5; ++m) un[m] = un[m] + hdt * (s1[m] - s0[m]);
      }
      for (int m = 0; m < 5; ++m)
        Unew[(((size_t)m * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)] = un[m];
    });
    return flags;
  }
};

template <class S, class A>
int run_step(const A* U, const int n[3], const int wlo[3], const int whi[3], double dt,
             const double h[3], const OParams* P, const int* walls, A* Unew, A* F[3], bool counting,
             const A* RX = nullptr, int ns = 0, A* RXnew = nullptr) {
  Step<S, A> st;
  st.U = U;
  st.RX = RX;
  st.ns = ns;
  st.RXnew = RXnew;
  if (walls)
    for (int f = 0; f < 6; ++f) st.wall[f] = walls[f] != 0;
  for (int d = 0; d < 3; ++d) { st.n[d] = n[d]; st.N[d] = n[d] + 2 * NG; st.h[d] = h[d]; }
  st.P = P;
  st.dt = dt;
  st.K = make_consts<S>(*P, dt, h);
  return st.run(wlo, whi, Unew, F, counting);
}

bool window_ok(const int n[3], const int wlo[3], const int whi[3]) {
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || wlo[d] < 0 || whi[d] >= n[d] || wlo[d] > whi[d]) return false;
  return true;
}

}  // namespace

// ================================================================= C API ====
extern "C" {

// One step of one box on a window of valid zones (see Step).  precision 0:
// FP64; 1: FP32 reconstruction with FP64 update.  walls: null or six flags
// (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi) marking the box faces that lie on a
// reflecting domain boundary.  F may be null (no flux output) or point to
// three face-centred arrays, any of which may be null.  Returns the status
// flags (1: non-physical input, 2: a floor bound) or -1 for invalid
// arguments.
int oracle_step(const double* U, const int n[3], const int wlo[3], const int whi[3], double dt,
                const double h[3], const OParams* P, const int* walls, double* Unew, double** F) {
  if (!U || !Unew || !P || !window_ok(n, wlo, whi) || !(dt > 0) || !(P->gamma > 1.0)) return -1;
  if (P->precision == 1)
    return run_step<float, double>(U, n, wlo, whi, dt, h, P, walls, Unew, F, false);
  return run_step<double, double>(U, n, wlo, whi, dt, h, P, walls, Unew, F, false);
}

// The step with ns passive species: RX holds the partial densities rho X_s
// of the box (layout [s][k][j][i] over the stored grid, ghosts filled like
// U); RXnew receives the window's new values (other entries untouched).
// Returns the status flags or -1.
int oracle_step_species(const double* U, const double* RX, int ns, const int n[3], const int wlo[3],
                        const int whi[3], double dt, const double h[3], const OParams* P, const int* walls,
                        double* Unew, double* RXnew) {
  if (!U || !Unew || !P || !RX || !RXnew || ns < 1 || !window_ok(n, wlo, whi) || !(dt > 0) ||
      !(P->gamma > 1.0))
    return -1;
  if (P->precision == 1)
    return run_step<float, double>(U, n, wlo, whi, dt, h, P, walls, Unew, nullptr, false, RX, ns, RXnew);
  return run_step<double, double>(U, n, wlo, whi, dt, h, P, walls, Unew, nullptr, false, RX, ns, RXnew);
}

// Same step with the Counted scalar; counts[stage][kind] receives the number
// of floating-point operations per stage (kinds: add/sub, mul, div, sqrt,
// min/max).  FP64 mode only.
int oracle_step_count(const double* U, const int n[3], const int wlo[3], const int whi[3],
                      double dt, const double h[3], const OParams* P, const int* walls, double* Unew,
                      unsigned long long* counts) {
  if (!U || !Unew || !P || !window_ok(n, wlo, whi)) return -1;
  const int N[3] = {n[0] + 2 * NG, n[1] + 2 * NG, n[2] + 2 * NG};
  const size_t tot = (size_t)5 * N[0] * N[1] * N[2];
  std::vector<Counted> uc(tot), un(tot);
  for (size_t i = 0; i < tot; ++i) { uc[i] = Counted(U[i]); un[i] = Counted(Unew[i]); }
  std::memset(g_ops, 0, sizeof(g_ops));
  Counted* none[3] = {nullptr, nullptr, nullptr};
  int fl = run_step<Counted, Counted>(uc.data(), n, wlo, whi, dt, h, P, walls, un.data(), none, true);
  g_stage = 0;
  for (size_t i = 0; i < tot; ++i) Unew[i] = un[i].v;
  for (int s = 0; s < ST_NSTAGE; ++s)
    for (int k = 0; k < OP_NKIND; ++k) counts[s * OP_NKIND + k] = g_ops[s][k];
  return fl;
}

// Jacobian-vector product of the step: (Unew, dUnew) = (step(U), J(U) dU)
// with dt frozen and every branch decided on the primal values.  precision
// 0: FP64; 1: the FP32-reconstruction step (float primal, double tangent).
int oracle_step_jvp(const double* U, const double* dU, const int n[3], const int wlo[3],
                    const int whi[3], double dt, const double h[3], const OParams* P, const int* walls,
                    double* Unew, double* dUnew) {
  if (!U || !dU || !Unew || !dUnew || !P || !window_ok(n, wlo, whi)) return -1;
  const int N[3] = {n[0] + 2 * NG, n[1] + 2 * NG, n[2] + 2 * NG};
  const size_t tot = (size_t)5 * N[0] * N[1] * N[2];
  std::vector<Dual> ud(tot), un(tot);
  for (size_t i = 0; i < tot; ++i) { ud[i] = Dual(U[i], dU[i]); un[i] = Dual(Unew[i], dUnew[i]); }
  Dual* none[3] = {nullptr, nullptr, nullptr};
  const int fl = (P->precision == 1)
                     ? run_step<DualF, Dual>(ud.data(), n, wlo, whi, dt, h, P, walls, un.data(), none, false)
                     : run_step<Dual, Dual>(ud.data(), n, wlo, whi, dt, h, P, walls, un.data(), none, false);
  for (size_t i = 0; i < tot; ++i) { Unew[i] = un[i].v; dUnew[i] = un[i].d; }
  return fl;
}

// The same with the flux outputs and their tangents: F[d], dF[d] (any may be
// null) receive the face-centred fluxes F^{n+1/2} of axis d (extents n + e_d,
// order [c][k][j][i]) and their tangents along dU.
int oracle_step_jvp_flux(const double* U, const double* dU, const int n[3], const int wlo[3], const int whi[3],
                         double dt, const double h[3], const OParams* P, const int* walls, double* Unew,
                         double* dUnew, double** F, double** dF) {
  if (!U || !dU || !Unew || !dUnew || !P || !F || !dF || !window_ok(n, wlo, whi) || P->precision != 0) return -1;
  const int N[3] = {n[0] + 2 * NG, n[1] + 2 * NG, n[2] + 2 * NG};
  const size_t tot = (size_t)5 * N[0] * N[1] * N[2];
  std::vector<Dual> ud(tot), un(tot);
  for (size_t i = 0; i < tot; ++i) { ud[i] = Dual(U[i], dU[i]); un[i] = Dual(Unew[i], dUnew[i]); }
  std::vector<Dual> fd[3];
  Dual* fp[3] = {nullptr, nullptr, nullptr};
  size_t fn[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    if (!F[d] || !dF[d]) continue;
    size_t e = 5;
    for (int a = 0; a < 3; ++a) e *= (size_t)(n[a] + (a == d ? 1 : 0));
    fd[d].assign(e, Dual(0.0));
    fp[d] = fd[d].data();
    fn[d] = e;
  }
  const int fl = run_step<Dual, Dual>(ud.data(), n, wlo, whi, dt, h, P, walls, un.data(), fp, false);
  for (size_t i = 0; i < tot; ++i) { Unew[i] = un[i].v; dUnew[i] = un[i].d; }
  for (int d = 0; d < 3; ++d)
    for (size_t i = 0; i < fn[d]; ++i) { F[d][i] = fd[d][i].v; dF[d][i] = fd[d][i].d; }
  return fl;
}

// O11: largest signal speed over valid zones and axes, max_d (|u_d| + c)/h_d,
// from the FP64 primitive state; dt = cfl / s.  Sets *flags like the step.
double oracle_max_wavespeed(const double* U, const int n[3], const double h[3], const OParams* P,
                            int* flags) {
  OParams Q = *P;
  Q.precision = 0;
  Consts<double> K = make_consts<double>(Q, 1.0, h);
  const int N[3] = {n[0] + 2 * NG, n[1] + 2 * NG, n[2] + 2 * NG};
  int fl = 0;
  double s = 0.0;
  const int lo[3] = {0, 0, 0}, hi[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
  for_region(lo, hi, [&](const int x[3]) {
    double uc[5], qc[6];
    for (int c = 0; c < 5; ++c)
      uc[c] = U[(((size_t)c * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)];
    cons_to_prim_cell(uc, K, qc, fl);
    for (int d = 0; d < 3; ++d) {
      const double sd = (std::fabs(qc[1 + d]) + qc[5]) / h[d];
      s = std::max(s, sd);
    }
  });
  if (flags) *flags = fl;
  return s;
}

// O6 alone, for tests: flux at a d-face from primitive states L, R.
int oracle_riemann(const double L[5], const double R[5], int d, const OParams* P, double F[5]) {
  const double h[3] = {1.0, 1.0, 1.0};
  Consts<double> K = make_consts<double>(*P, 1.0, h);
  int fl = 0;
  riemann(L, R, d, K, F, fl);
  return fl;
}

// O3 alone, for tests: after O2 on the stored zones of one box (ghosts of U
// as given), the flattening coefficient phi of every traced zone [-1, n]^3,
// written to phi ((n+2)^3 values, x fastest).  Returns the status flags or -1.
int oracle_flatten(const double* U, const int n[3], const OParams* P, double* phi) {
  const int wlo[3] = {0, 0, 0}, whi[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
  if (!U || !phi || !P || !window_ok(n, wlo, whi)) return -1;
  Step<double, double> st;
  st.U = U;
  for (int d = 0; d < 3; ++d) { st.n[d] = n[d]; st.N[d] = n[d] + 2 * NG; st.h[d] = 1.0; }
  st.P = P;
  st.dt = 1.0;
  const double h[3] = {1.0, 1.0, 1.0};
  st.K = make_consts<double>(*P, 1.0, h);
  st.phi_out = phi;
  return st.run(wlo, whi, nullptr, nullptr, false);
}

// Operation counts of single pieces of the method with the Counted scalar,
// for the op-count pins.  what = 0: one Riemann solve (O6) of the face normal
// to x, in = L[5] then R[5], out = the flux F[5].  what = 1: one conversion
// of a corrected state as in O8/O9 without the correction, primitive ->
// conserved -> primitive with floors, in = q[5], out = the primitive state.
// counts[kind] (add/sub, mul, div, sqrt, min/max) receives the counts.
// Returns the status flags or -1.
int oracle_count_ops(int what, const double* in, const OParams* P, double* out, unsigned long long counts[5]) {
  if (!in || !out || !P || !counts || what < 0 || what > 1) return -1;
  const double h[3] = {1.0, 1.0, 1.0};
  Consts<Counted> K = make_consts<Counted>(*P, 1.0, h);
  std::memset(g_ops, 0, sizeof(g_ops));
  g_stage = 0;
  int fl = 0;
  if (what == 0) {
    Counted L[5], R[5], F[5];
    for (int m = 0; m < 5; ++m) { L[m] = Counted(in[m]); R[m] = Counted(in[5 + m]); }
    riemann(L, R, 0, K, F, fl);
    for (int m = 0; m < 5; ++m) out[m] = F[m].v;
  } else {
    Counted q[5], u[5], qo[5];
    for (int m = 0; m < 5; ++m) q[m] = Counted(in[m]);
    prim_to_cons(q, K, u);
    cons_to_prim_floor(u, K, qo, fl);
    for (int m = 0; m < 5; ++m) out[m] = qo[m].v;
  }
  for (int k = 0; k < OP_NKIND; ++k) counts[k] = g_ops[0][k];
  return fl;
}

// O4 alone, for tests: parabolas (aL, aR, a6) of a 1-D line a[0..m-1] at
// zones 2..m-3 (outputs at the same indices; others untouched).  phi may be
// null (phi = 1).
int oracle_ppm_line(const double* a, int m, const double* phi, const OParams* P, double* aL,
                    double* aR, double* a6) {
  const double h[3] = {1.0, 1.0, 1.0};
  Consts<double> K = make_consts<double>(*P, 1.0, h);
  for (int i = 2; i < m - 2; ++i) ppm_parabola(a + i - 2, phi ? phi[i] : 1.0, K, aL[i], aR[i], a6[i]);
  return 0;
}

// O4 integrals: I+(sigma) and I-(sigma) of a parabola (aL, aR, a6).
void oracle_ppm_integrals(double aL, double aR, double a6, double sigma, double* ip, double* im) {
  const double h[3] = {1.0, 1.0, 1.0};
  OParams P{};
  P.gamma = 1.4;
  Consts<double> K = make_consts<double>(P, 1.0, h);
  *ip = ppm_ip(aR, aR - aL, a6, sigma, K);
  *im = ppm_im(aL, aR - aL, a6, sigma, K);
}

// O5 alone, for tests: traced states of one zone along d from its
// parabolas and cell primitive state (rho, u, v, w, p, c), Courant factor
// dtdx = dt/h_d.
int oracle_trace(const double aL[5], const double aR[5], const double a6[5], const double cell[6],
                 int d, double dtdx, const OParams* P, double qp[5], double qm[5]) {
  double h[3] = {1.0, 1.0, 1.0};
  h[d] = 1.0 / dtdx;
  Consts<double> K = make_consts<double>(*P, 1.0, h);
  int fl = 0;
  trace_zone(aL, aR, a6, cell, d, K, qp, qm, fl);
  return fl;
}

// O1: ghost fill of every box of a level.  Boxes are inclusive [lo, hi]
// triples in a global index space and tile the domain [dlo, dhi] exactly.
// bc[2d], bc[2d+1]: low/high face of axis d (0 periodic, 1 outflow, 2
// reflect, 3 coarse-fine).  Box b's data start at arena + off[b], layout
// [comp][k][j][i] over (n+8)^3.  A ghost zone takes the value of the valid
// zone that owns its image: periodic axes wrap, outflow axes clamp to the
// nearest valid zone, reflecting axes mirror about the wall with the normal
// momentum negated.  Ghost zones beyond a coarse-fine face are left as they
// are (the two-level advance interpolates them).  Ghost zones beyond an
// inflow face (bc 4, at most one per layout) take the prescribed state of
// that face, inflow[face]: 5 components over the domain's extents of the two
// other axes t1 < t2, order [c][t2][t1], at the image of the zone's
// transverse coordinates under those axes' rules (momentum signs as for a
// copy).  Returns 0, or -1 if an image has no owner or inflow data are
// missing.
static int fill_level(int nbox, const int* lo, const int* hi, const int dlo[3], const int dhi[3],
                      const int bc[6], double* arena, const long long* off, int ncomp, bool momentum,
                      const double* const* inflow = nullptr);

int oracle_fill(int nbox, const int* lo, const int* hi, const int dlo[3], const int dhi[3],
                const int bc[6], double* arena, const long long* off) {
  return fill_level(nbox, lo, hi, dlo, dhi, bc, arena, off, 5, true);
}

// The state fill with inflow faces: inflow[6] (null entries for the faces
// that are not inflow faces).
int oracle_fill_inflow(int nbox, const int* lo, const int* hi, const int dlo[3], const int dhi[3],
                       const int bc[6], double* arena, const long long* off, const double* const* inflow) {
  return fill_level(nbox, lo, hi, dlo, dhi, bc, arena, off, 5, true, inflow);
}

// The same fill for ncomp scalar fields per box (passive species): no
// component changes sign at a reflecting wall.
int oracle_fill_scalars(int nbox, const int* lo, const int* hi, const int dlo[3], const int dhi[3],
                        const int bc[6], double* arena, const long long* off, int ncomp) {
  if (ncomp < 1) return -1;
  return fill_level(nbox, lo, hi, dlo, dhi, bc, arena, off, ncomp, false);
}

static int fill_level(int nbox, const int* lo, const int* hi, const int dlo[3], const int dhi[3],
                      const int bc[6], double* arena, const long long* off, int ncomp, bool momentum,
                      const double* const* inflow) {
  int ninflow = 0;
  for (int f = 0; f < 6; ++f)
    if (bc[f] == BC_INFLOW) {
      ++ninflow;
      if (!inflow || !inflow[f] || ncomp != 5) return -1;
    }
  if (ninflow > 1) return -1;
  int L[3];
  for (int d = 0; d < 3; ++d) L[d] = dhi[d] - dlo[d] + 1;
  // owner of every valid zone of the domain, painted box by box
  std::vector<int> owner((size_t)L[0] * L[1] * L[2], -1);
  for (int b = 0; b < nbox; ++b) {
    const int bl[3] = {lo[3 * b] - dlo[0], lo[3 * b + 1] - dlo[1], lo[3 * b + 2] - dlo[2]};
    const int bh[3] = {hi[3 * b] - dlo[0], hi[3 * b + 1] - dlo[1], hi[3 * b + 2] - dlo[2]};
    for_region(bl, bh, [&](const int x[3]) {
      owner[((size_t)x[2] * L[1] + x[1]) * L[0] + x[0]] = b;
    });
  }
  for (int b = 0; b < nbox; ++b) {
    int n[3], N[3];
    for (int d = 0; d < 3; ++d) { n[d] = hi[3 * b + d] - lo[3 * b + d] + 1; N[d] = n[d] + 2 * NG; }
    const int gl[3] = {-NG, -NG, -NG}, gh[3] = {n[0] + NG - 1, n[1] + NG - 1, n[2] + NG - 1};
    double* dst = arena + off[b];
    bool bad = false;
    for_region(gl, gh, [&](const int x[3]) {
      if (x[0] >= 0 && x[0] < n[0] && x[1] >= 0 && x[1] < n[1] && x[2] >= 0 && x[2] < n[2]) return;
      int g[3];
      double sgn[3] = {1, 1, 1};  // momentum components 1..3
      int inface = -1;
      for (int d = 0; d < 3; ++d) {
        const int v = lo[3 * b + d] + x[d] - dlo[d];
        if ((v < 0 && bc[2 * d] == BC_COARSE_FINE) || (v >= L[d] && bc[2 * d + 1] == BC_COARSE_FINE)) return;
      }
      for (int d = 0; d < 3; ++d) {
        int v = lo[3 * b + d] + x[d] - dlo[d];  // domain-relative index
        if (v < 0 || v >= L[d]) {
          const int face = (v < 0) ? 2 * d : 2 * d + 1;
          if (bc[face] == BC_INFLOW) {
            inface = face;
            v = 0;
          } else if (bc[face] == BC_PERIODIC) {
            v = ((v % L[d]) + L[d]) % L[d];
          } else if (bc[face] == BC_OUTFLOW) {
            v = (v < 0) ? 0 : L[d] - 1;
          } else {
            v = (v < 0) ? (-1 - v) : (2 * L[d] - 1 - v);
            sgn[d] = -sgn[d];
          }
        }
        g[d] = v;
      }
      if (inface >= 0) {
        const int d = inface / 2, t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
        const double* src = inflow[inface];
        for (int c = 0; c < 5; ++c) {
          const double v = src[((size_t)c * L[t2] + g[t2]) * L[t1] + g[t1]];
          const double sg = (c >= 1 && c <= 3) ? sgn[c - 1] : 1.0;
          dst[(((size_t)c * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)] = sg * v;
        }
        return;
      }
      const int ob = owner[((size_t)g[2] * L[1] + g[1]) * L[0] + g[0]];
      if (ob < 0) { bad = true; return; }
      int on[3], ON[3], ol[3];
      for (int d = 0; d < 3; ++d) {
        on[d] = hi[3 * ob + d] - lo[3 * ob + d] + 1;
        ON[d] = on[d] + 2 * NG;
        ol[d] = g[d] + dlo[d] - lo[3 * ob + d];
      }
      const double* src = arena + off[ob];
      for (int c = 0; c < ncomp; ++c) {
        const double v = src[(((size_t)c * ON[2] + (ol[2] + NG)) * ON[1] + (ol[1] + NG)) * ON[0] + (ol[0] + NG)];
        const double sg = (momentum && c >= 1 && c <= 3) ? sgn[c - 1] : 1.0;
        dst[(((size_t)c * N[2] + (x[2] + NG)) * N[1] + (x[1] + NG)) * N[0] + (x[0] + NG)] = sg * v;
      }
    });
    if (bad) return -1;
  }
  return 0;
}

}  // extern "C"

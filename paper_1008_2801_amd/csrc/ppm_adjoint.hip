// gfx950 kernels of the adjoint (reverse-mode derivative) of one step,
// dt frozen and every branch decision frozen at the forward values.
//
// Given the step's input state U (ghosts filled) and the adjoint Ub' of the
// new state's valid zones, the adjoint of U's valid zones is formed as
//   recompute: prim, flatten, trace, riemann1, riemann2   (forward kernels)
//   adj_riemann3  final fluxes' adjoint (from Ub' through the update and its
//                 Heun source) -> corrected-state adjoints (U3b) and
//                 traced-state adjoints
//   adj_riemann2  stage-2 fluxes' adjoint (from U3b) -> U2b, traced states
//   adj_riemann1  stage-1 fluxes' adjoint (from U2b) -> traced states
//   adj_trace     traced-state adjoints -> per-zone contributions to the
//                 primitives of the 5-zone stencil of each axis
//   adj_flatten   flattening adjoint -> contributions to the pressure stencil
//   adj_gather    per stored zone: the contributions that reach it, then the
//                 primitive conversion's adjoint -> conserved adjoints (plus,
//                 on valid zones, Ub' through the update)
//   adj_fill      ghost adjoints gathered into their owning valid zones
// Along y and z the Riemann reverses run one lane per face slot and pass
// per-zone-side planes on.  Along x, where a workgroup's lanes hold
// neighbouring zones (runs of traced zones with halo lanes), the stage-3
// and stage-2 reverses add each zone's two sides in LDS, and the stage-1
// reverse and the trace reverse are one kernel that keeps each zone's
// traced-state adjoints in registers and adds its stencil contributions in
// LDS; every sum keeps the order of terms of the per-zone form.
// Every reverse stage writes only the entries it owns or accumulates through
// a gather in a fixed order: no atomics, results reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "ppm_device.h"
#include "ppm_internal.h"
#include "ppm_math.h"
#include "ppm_vjp.h"

namespace ppm {
namespace {

// Adjoint workspace planes: traced grid (A_*) and stored grid (AS_*).  The
// trace reverse's stencil contributions (GT) reuse the stage-3
// corrected-state planes and the first stage-2 ones: the x trace reverse,
// which runs while the y and z stage-1 reverses' planes are still being
// read (by its own stage-1 part), writes only the first 25, and those are
// dead once the stage-2 reverse has run; the y and z ones are written after
// every stage-1 reverse.  The sound-speed and flattening-coefficient
// adjoints (CB, PHB) have planes of their own.
constexpr int A_TB = 0;              // 30: traced-state adjoints [d][side][m]
constexpr int A_U3 = A_TB + 30;      // 30: stage-3 corrected-state adjoints [d][side][m]
constexpr int A_U2 = A_U3 + 30;      // 60: stage-2 corrected-state adjoints [pair][side][m]
constexpr int A_GT = A_U3;           // 75: trace contributions [d][m][offset + 2]
constexpr int A_GF = A_U2 + 60;      // 7: flattening contributions to p [offset + 3]
constexpr int A_SEL = A_GF + 7;      // 1: axis selected by the flattening minimum (-1: none)
constexpr int A_CB = A_SEL + 1;      // 3: sound-speed adjoint per axis
constexpr int A_PHB = A_CB + 3;      // 3: flattening-coefficient adjoint per axis
constexpr int A_EPLANES = A_PHB + 3;
static_assert(A_GT + 75 <= A_U2 + 60, "trace contributions must fit in the corrected-state planes");
static_assert(A_GT + 25 <= A_U3 + 30, "the x trace contributions must fit in the stage-3 planes");
constexpr int AS_UB = 0;             // 5: conserved adjoints
constexpr int A_SPLANES = 5;

__device__ __forceinline__ bool in_e(const int x[3], const DevBox& B) {
  return x[0] >= -1 && x[0] <= B.n[0] && x[1] >= -1 && x[1] <= B.n[1] && x[2] >= -1 && x[2] <= B.n[2];
}
__device__ __forceinline__ long long eidx(const DevBox& B, int x, int y, int z) {
  return ((long long)(z + 1) * (B.n[1] + 2) + (y + 1)) * (B.n[0] + 2) + (x + 1);
}

// Reverse of the update's Heun source at one valid zone (FP64, as the
// update).  ub: the new state's adjoint there.  uf: the adjoint of the
// pre-source state (what the flux divergence receives); direct: the part
// that reaches the zone's own old state through the source.  The source is
// S(U) = (0, rho g, (rho u).g), so S^T V = ((g.V_mom), g V_E, 0).
__device__ __forceinline__ void heun_reverse(const double ub[5], int grav, double dt, double hdt, double g0,
                                             double g1, double g2, double uf[5], double direct[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) { uf[m] = ub[m]; direct[m] = ub[m]; }
  if (!grav) return;
  auto st = [&](const double v[5], double o[5]) {
    o[0] = (g0 * v[1] + g1 * v[2]) + g2 * v[3];
    o[1] = g0 * v[4];
    o[2] = g1 * v[4];
    o[3] = g2 * v[4];
    o[4] = 0.0;
  };
  double s[5], s1[5];
  st(ub, s);
#pragma unroll
  for (int m = 0; m < 5; ++m) uf[m] = ub[m] + hdt * s[m];
  st(uf, s1);
#pragma unroll
  for (int m = 0; m < 5; ++m) direct[m] = uf[m] + (dt * s1[m] - hdt * s[m]);
}

// Pre-source adjoint of zone (x, y, z) of box B from the new state's adjoint
// (zero outside the valid zones).
__device__ __forceinline__ void pre_source_adjoint(const double* __restrict__ Ubn, const DevBox& B, int x, int y,
                                                   int z, int grav, const StepConsts* __restrict__ sc,
                                                   double g0, double g1, double g2, double uf[5]) {
  if (x < 0 || x >= B.n[0] || y < 0 || y >= B.n[1] || z < 0 || z >= B.n[2]) {
#pragma unroll
    for (int m = 0; m < 5; ++m) uf[m] = 0.0;
    return;
  }
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
  const long long NS = (long long)N0 * N1 * N2;
  const long long li = ((long long)(z + NG) * N1 + (y + NG)) * N0 + (x + NG);
  double ub[5], direct[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) ub[m] = Ubn[B.soff + li + m * NS];
  heun_reverse(ub, grav, sc->dt, sc->hdt, g0, g1, g2, uf, direct);
}

// Corrected state of axis d at zone offset `off` from the lane's zone,
// forward stage-3 form (traced state minus both stage-2 flux differences).
template <int d, class S>
__device__ __forceinline__ void r3_state(const S* w, long long LE, long long off, int side, long long s1,
                                         long long s2, S c1, S c2, const Gas<S>& G, S qe[5], S ue[5]) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  constexpr int p12 = pair_index(t1, t2), p21 = pair_index(t2, t1);
#pragma unroll
  for (int m = 0; m < 5; ++m) qe[m] = w[(E_TRACE + (d * 2 + side) * 5 + m) * LE + off];
  prim_to_cons(qe, G, ue);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* fa = w + (E_F2 + p12 * 5 + m) * LE + off;
    const S* fb = w + (E_F2 + p21 * 5 + m) * LE + off;
    ue[m] = ue[m] - c1 * (fa[s1] - fa[0]) - c2 * (fb[s2] - fb[0]);
  }
}

// Reverse of the stage-3 solve of the face at zone slot x along d (a face:
// x_d >= 0 and both transverse indices valid): from the new state's adjoint
// of the face's two zones (through the update and its Heun source) and the
// flux output's adjoint, the adjoints of the two corrected states (uLb of
// zone x - e_d, uRb of zone x) and of their traced states (tLb, tRb).
template <int d, class S>
__device__ __forceinline__ void adj_r3_face(const DevBox& B, const EZone& z, const S* __restrict__ w, long long LE,
                                            const Gas<S>& G, const StepConsts* __restrict__ sc,
                                            const double* __restrict__ Ubn, const FluxBar& fbar, int grav,
                                            double g0, double g1, double g2, S uLb[5], S uRb[5], S tLb[5],
                                            S tRb[5]) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const long long sd = stride(z.E, d), s1 = stride(z.E, t1), s2 = stride(z.E, t2);
  const S c1 = SC<S>::dt2h(sc)[t1], c2 = SC<S>::dt2h(sc)[t2];
  // the final flux's adjoint from the pre-source adjoints of the face's two
  // zones (the update is FP64)
  double ufR[5], ufL[5];
  pre_source_adjoint(Ubn, B, z.x[0], z.x[1], z.x[2], grav, sc, g0, g1, g2, ufR);
  pre_source_adjoint(Ubn, B, z.x[0] - (d == 0), z.x[1] - (d == 1), z.x[2] - (d == 2), grav, sc, g0, g1, g2, ufL);
  S Fb[5];
  const double dtdx = sc->dtdx[d];
  // plus the adjoint of the face's flux output, when given (face-centred
  // arena of axis d: extents n + e_d, order [c][k][j][i])
  double fo[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (fbar.p[d]) {
    int fe[3] = {B.n[0], B.n[1], B.n[2]};
    fe[d] += 1;
    const long long FN = (long long)fe[0] * fe[1] * fe[2];
    const double* q = fbar.p[d] + B.foff[d] + ((long long)z.x[2] * fe[1] + z.x[1]) * fe[0] + z.x[0];
#pragma unroll
    for (int m = 0; m < 5; ++m) fo[m] = q[m * FN];
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) Fb[m] = (S)(dtdx * (ufR[m] - ufL[m]) + fo[m]);
  S qeL[5], ueL[5], qeR[5], ueR[5], L[5], R[5];
  bool rfL, pfL, rfR, pfR;
  r3_state<d>(w, LE, -sd, 0, s1, s2, c1, c2, G, qeL, ueL);
  r3_state<d>(w, LE, 0, 1, s1, s2, c1, c2, G, qeR, ueR);
  cons_to_prim_dec(ueL, G, L, rfL, pfL);
  cons_to_prim_dec(ueR, G, R, rfR, pfR);
  // a state replaced by a wall mirror gets no adjoint below, so L and R can
  // be overwritten in place
  const int ws = wall_states<d>(B, z.x[d], L, R);
  S Lb[5] = {0, 0, 0, 0, 0}, Rb[5] = {0, 0, 0, 0, 0};
  riemann_vjp<d>(L, R, G, Fb, Lb, Rb);
  wall_states_vjp<d>(ws, Lb, Rb);
#pragma unroll
  for (int m = 0; m < 5; ++m) uLb[m] = uRb[m] = tLb[m] = tRb[m] = S(0);
  cons_to_prim_vjp_q(L, rfL, pfL, G, Lb, uLb);
  cons_to_prim_vjp_q(R, rfR, pfR, G, Rb, uRb);
  prim_to_cons_vjp(qeL, G, uLb, tLb);
  prim_to_cons_vjp(qeR, G, uRb, tRb);
}

// Face slot x along d is a stage-3 face when x_d >= 0 and both transverse
// indices are valid.  The lane of slot x writes the adjoints of the two
// states of its face (zone x - e_d, high side; zone x, low side); every zone
// side not on a face is written as zero by the zone's own lane, so each
// entry of the U3 and traced-state planes is written exactly once here.
template <int d, class S>
__device__ __forceinline__ void adj_r3_body(const Tile* __restrict__ tiles, int ntiles,
                                            const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                            long long LE, S* __restrict__ aw, const Gas<S>& G,
                                            const StepConsts* __restrict__ sc, const double* __restrict__ Ubn,
                                            const FluxBar& fbar, int grav, double g0, double g1, double g2) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  S* a = aw + B.eoff + z.e;
  const bool tv = z.x[t1] >= 0 && z.x[t1] < B.n[t1] && z.x[t2] >= 0 && z.x[t2] < B.n[t2];
  const bool face = tv && z.x[d] >= 0;
  const bool hi_face = tv && z.x[d] + 1 <= B.n[d];  // slot x + e_d is a face
  if (!hi_face) {
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      a[(A_U3 + (d * 2 + 0) * 5 + m) * LE] = S(0);
      a[(A_TB + (d * 2 + 0) * 5 + m) * LE] = S(0);
    }
  }
  if (!face) {
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      a[(A_U3 + (d * 2 + 1) * 5 + m) * LE] = S(0);
      a[(A_TB + (d * 2 + 1) * 5 + m) * LE] = S(0);
    }
    return;
  }
  const long long sd = stride(z.E, d);
  S uLb[5], uRb[5], tLb[5], tRb[5];
  adj_r3_face<d>(B, z, work + B.eoff + z.e, LE, G, sc, Ubn, fbar, grav, g0, g1, g2, uLb, uRb, tLb, tRb);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    a[(A_U3 + (d * 2 + 0) * 5 + m) * LE - sd] = uLb[m];
    a[(A_U3 + (d * 2 + 1) * 5 + m) * LE] = uRb[m];
    a[(A_TB + (d * 2 + 0) * 5 + m) * LE - sd] = tLb[m];
    a[(A_TB + (d * 2 + 1) * 5 + m) * LE] = tRb[m];
  }
}

// Axes y and z (blockIdx.y 0, 1); x runs in k_adj_r3_x.
template <class S>
__device__ __forceinline__ void adj_r3_axes(const Tile* __restrict__ tiles, int ntiles,
                                            const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                            long long LE, S* __restrict__ aw, const Gas<S> G,
                                            const StepConsts* __restrict__ sc, const double* __restrict__ Ubn,
                                            const FluxBar& fbar, int grav, double g0, double g1, double g2) {
  if (blockIdx.y == 0)
    adj_r3_body<1, S>(tiles, ntiles, boxes, work, LE, aw, G, sc, Ubn, fbar, grav, g0, g1, g2);
  else
    adj_r3_body<2, S>(tiles, ntiles, boxes, work, LE, aw, G, sc, Ubn, fbar, grav, g0, g1, g2);
}

// FP64: held to 3 waves per SIMD (it fits without spilling); FP32 fits 5.
__global__ void __launch_bounds__(MAX_TILE) __attribute__((amdgpu_waves_per_eu(3)))
k_adj_r3_f64(const Tile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
             const double* __restrict__ work, long long LE, double* __restrict__ aw, Gas<double> G,
             const StepConsts* __restrict__ sc, const double* __restrict__ Ubn, FluxBar fbar, int grav,
             double g0, double g1, double g2) {
  adj_r3_axes<double>(tiles, ntiles, boxes, work, LE, aw, G, sc, Ubn, fbar, grav, g0, g1, g2);
}
__global__ void __launch_bounds__(MAX_TILE)
k_adj_r3_f32(const Tile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
             const float* __restrict__ work, long long LE, float* __restrict__ aw, Gas<float> G,
             const StepConsts* __restrict__ sc, const double* __restrict__ Ubn, FluxBar fbar, int grav,
             double g0, double g1, double g2) {
  adj_r3_axes<float>(tiles, ntiles, boxes, work, LE, aw, G, sc, Ubn, fbar, grav, g0, g1, g2);
}

// Stage-3 reverse along x over runs of XF_OWNED traced slots: lane l takes
// the face at slot start + l, and one lane past the run the next face, so
// that each zone's two corrected-state adjoints (high side from the face
// above it, low side from its own face) are added in LDS and stored as one
// plane per field (the sum the stage-2 reverse forms, in its order: high
// side + low side).  The traced-state adjoints are written per side as in
// k_adj_r3_f64.
template <class S>
__global__ void __launch_bounds__(XF_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_adj_r3_x(const Tile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
           const S* __restrict__ work, long long LE, S* __restrict__ aw, Gas<S> G,
           const StepConsts* __restrict__ sc, const double* __restrict__ Ubn, FluxBar fbar, int grav, double g0,
           double g1, double g2) {
  __shared__ S buf[5][XF_THREADS];
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;  // the whole workgroup
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  const int l = threadIdx.x;
  EZone z;
  z.E[0] = B.n[0] + 2; z.E[1] = B.n[1] + 2; z.E[2] = B.n[2] + 2;
  const int NE = z.E[0] * z.E[1] * z.E[2];
  const int i = tl.start + l, nown = tl.end - tl.start;
  const bool own = l < nown;
  const bool act = l <= nown && i < NE;  // the run's slots and the next one
  bool face = false, hi_face = false;
  if (act) {
    const unsigned r = div31((unsigned)i, B.de[0]), k = div31(r, B.de[1]);
    z.e = i;
    z.x[0] = i - (int)r * z.E[0] - 1;
    z.x[1] = (int)(r - k * (unsigned)z.E[1]) - 1;
    z.x[2] = (int)k - 1;
    const bool tv = z.x[1] >= 0 && z.x[1] < B.n[1] && z.x[2] >= 0 && z.x[2] < B.n[2];
    face = tv && z.x[0] >= 0;
    hi_face = tv && z.x[0] + 1 <= B.n[0];
  }
  S uLb[5] = {0, 0, 0, 0, 0}, uRb[5] = {0, 0, 0, 0, 0}, tLb[5] = {0, 0, 0, 0, 0}, tRb[5] = {0, 0, 0, 0, 0};
  if (face) adj_r3_face<0>(B, z, work + B.eoff + i, LE, G, sc, Ubn, fbar, grav, g0, g1, g2, uLb, uRb, tLb, tRb);
  S* a = aw + B.eoff + (act ? i : 0);
  if (own) {
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      if (!hi_face) a[(A_TB + m) * LE] = S(0);
      if (face) {
        a[(A_TB + m) * LE - 1] = tLb[m];
        a[(A_TB + 5 + m) * LE] = tRb[m];
      } else {
        a[(A_TB + 5 + m) * LE] = S(0);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) buf[m][l] = uLb[m];
  __syncthreads();
  if (own) {
#pragma unroll
    for (int m = 0; m < 5; ++m)
      a[(A_U3 + m) * LE] = (hi_face ? buf[m][l + 1] : S(0)) + (face ? uRb[m] : S(0));
  }
}

// Stage-2 pair (d, t) of the face at the lane's slot: F2^{d|t} adjoint from
// the stage-3 states of the third axis r (difference along d), reverse of the
// corrected states, adjoints of the two traced states (accumulated) and of
// the corrected states (written to U2, or with OUT returned in uLo, uRo).
template <int d, int t, bool OUT, class S>
__device__ __forceinline__ void adj_r2_pair(const S* __restrict__ w, S* __restrict__ a, long long LE,
                                            long long sd, long long stt, const S qeL[5], const S qeR[5],
                                            const S ue0L[5], const S ue0R[5], const Gas<S>& G,
                                            const StepConsts* __restrict__ sc, const DevBox& B, int xd,
                                            S tLb[5], S tRb[5], S* uLo = nullptr, S* uRo = nullptr) {
  constexpr int pr = pair_index(d, t);
  constexpr int r = 3 - d - t;
  const S c3 = SC<S>::dt3h(sc)[t];
  S Fb[5];
  const S c2d = SC<S>::dt2h(sc)[d];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* up = a + (A_U3 + (r * 2 + 0) * 5 + m) * LE;
    const S* um = a + (A_U3 + (r * 2 + 1) * 5 + m) * LE;
    if constexpr (r == 0)  // along x the stage-3 reverse stored each zone's two sides summed
      Fb[m] = c2d * (up[0] - up[-sd]);
    else
      Fb[m] = c2d * ((up[0] + um[0]) - (up[-sd] + um[-sd]));
  }
  S ueL[5], ueR[5], L[5], R[5];
  bool rfL, pfL, rfR, pfR;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* fL = w + (E_F1 + t * 5 + m) * LE - sd;
    const S* fR = w + (E_F1 + t * 5 + m) * LE;
    ueL[m] = ue0L[m] - c3 * (fL[stt] - fL[0]);
    ueR[m] = ue0R[m] - c3 * (fR[stt] - fR[0]);
  }
  cons_to_prim_dec(ueL, G, L, rfL, pfL);
  cons_to_prim_dec(ueR, G, R, rfR, pfR);
  const int ws = wall_states<d>(B, xd, L, R);  // a replaced state gets no adjoint
  S Lb[5] = {0, 0, 0, 0, 0}, Rb[5] = {0, 0, 0, 0, 0};
  riemann_vjp<d, true>(L, R, G, Fb, Lb, Rb);
  wall_states_vjp<d>(ws, Lb, Rb);
  S uLb[5] = {0, 0, 0, 0, 0}, uRb[5] = {0, 0, 0, 0, 0};
  cons_to_prim_vjp_q(L, rfL, pfL, G, Lb, uLb);
  cons_to_prim_vjp_q(R, rfR, pfR, G, Rb, uRb);
  prim_to_cons_vjp(qeL, G, uLb, tLb);
  prim_to_cons_vjp(qeR, G, uRb, tRb);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if constexpr (OUT) {
      uLo[m] = uLb[m];
      uRo[m] = uRb[m];
    } else {
      a[(A_U2 + (pr * 2 + 0) * 5 + m) * LE - sd] = uLb[m];
      a[(A_U2 + (pr * 2 + 1) * 5 + m) * LE] = uRb[m];
    }
  }
}

// Both stage-2 pairs of axis d in one lane (traced states loaded once); the
// traced-state adjoints of the face's two zones receive both pairs' parts.
// Zone sides that are not on a pair's face get zero U2 entries from their
// own lane.
template <int d, class S>
__device__ __forceinline__ void adj_r2_body(const Tile* __restrict__ tiles, int ntiles,
                                            const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                            long long LE, S* __restrict__ aw, const Gas<S>& G,
                                            const StepConsts* __restrict__ sc) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  constexpr int pa = pair_index(d, t1), pb = pair_index(d, t2);
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  S* a = aw + B.eoff + z.e;
  const bool ta = z.x[t1] >= 0 && z.x[t1] < B.n[t1];
  const bool tb = z.x[t2] >= 0 && z.x[t2] < B.n[t2];
  const bool up = z.x[d] + 1 <= B.n[d];
  const bool va = ta && z.x[d] >= 0, vb = tb && z.x[d] >= 0;
  if (!(ta && up)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) a[(A_U2 + (pa * 2 + 0) * 5 + m) * LE] = S(0);
  }
  if (!(tb && up)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) a[(A_U2 + (pb * 2 + 0) * 5 + m) * LE] = S(0);
  }
  if (!va) {
#pragma unroll
    for (int m = 0; m < 5; ++m) a[(A_U2 + (pa * 2 + 1) * 5 + m) * LE] = S(0);
  }
  if (!vb) {
#pragma unroll
    for (int m = 0; m < 5; ++m) a[(A_U2 + (pb * 2 + 1) * 5 + m) * LE] = S(0);
  }
  if (!va && !vb) return;
  const long long sd = stride(z.E, d);
  const S* w = work + B.eoff + z.e;
  S qeL[5], qeR[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    qeL[m] = w[(E_TRACE + (d * 2 + 0) * 5 + m) * LE - sd];
    qeR[m] = w[(E_TRACE + (d * 2 + 1) * 5 + m) * LE];
  }
  S ue0L[5], ue0R[5];
  prim_to_cons(qeL, G, ue0L);
  prim_to_cons(qeR, G, ue0R);
  S tLb[5] = {0, 0, 0, 0, 0}, tRb[5] = {0, 0, 0, 0, 0};
  if (va)
    adj_r2_pair<d, t1, false, S>(w, a, LE, sd, stride(z.E, t1), qeL, qeR, ue0L, ue0R, G, sc, B, z.x[d], tLb, tRb);
  if (vb)
    adj_r2_pair<d, t2, false, S>(w, a, LE, sd, stride(z.E, t2), qeL, qeR, ue0L, ue0R, G, sc, B, z.x[d], tLb, tRb);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    a[(A_TB + (d * 2 + 0) * 5 + m) * LE - sd] += tLb[m];
    a[(A_TB + (d * 2 + 1) * 5 + m) * LE] += tRb[m];
  }
}

// Axes y and z (blockIdx.y 0, 1); x runs in k_adj_r2_x.
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_adj_r2(const Tile* __restrict__ tiles, int ntiles,
                                                 const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                                 long long LE, S* __restrict__ aw, Gas<S> G,
                                                 const StepConsts* __restrict__ sc) {
  if (blockIdx.y == 0)
    adj_r2_body<1, S>(tiles, ntiles, boxes, work, LE, aw, G, sc);
  else
    adj_r2_body<2, S>(tiles, ntiles, boxes, work, LE, aw, G, sc);
}

// Stage-2 reverse along x over runs of XF_OWNED traced slots (lane l: the
// face at slot start + l, one lane past the run the next face): per pair,
// each zone's two corrected-state adjoints (high side from the face above,
// low side from its own face) are added in LDS and stored as one plane per
// field, in the order the stage-1 reverse adds them.  The traced-state
// adjoints are accumulated per side as in k_adj_r2.
template <class S>
__global__ void __launch_bounds__(XF_THREADS) k_adj_r2_x(const Tile* __restrict__ tiles, int ntiles,
                                                     const DevBox* __restrict__ boxes,
                                                     const S* __restrict__ work, long long LE,
                                                     S* __restrict__ aw, Gas<S> G,
                                                     const StepConsts* __restrict__ sc) {
  constexpr int pa = pair_index(0, 1), pb = pair_index(0, 2);
  __shared__ S buf[5][XF_THREADS];
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;  // the whole workgroup
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  const int l = threadIdx.x;
  EZone z;
  z.E[0] = B.n[0] + 2; z.E[1] = B.n[1] + 2; z.E[2] = B.n[2] + 2;
  const int NE = z.E[0] * z.E[1] * z.E[2];
  const int i = tl.start + l, nown = tl.end - tl.start;
  const bool own = l < nown;
  const bool act = l <= nown && i < NE;  // the run's slots and the next one
  bool ta = false, tb = false, up = false, va = false, vb = false;
  if (act) {
    const unsigned r = div31((unsigned)i, B.de[0]), k = div31(r, B.de[1]);
    z.e = i;
    z.x[0] = i - (int)r * z.E[0] - 1;
    z.x[1] = (int)(r - k * (unsigned)z.E[1]) - 1;
    z.x[2] = (int)k - 1;
    ta = z.x[1] >= 0 && z.x[1] < B.n[1];
    tb = z.x[2] >= 0 && z.x[2] < B.n[2];
    up = z.x[0] + 1 <= B.n[0];
    va = ta && z.x[0] >= 0;
    vb = tb && z.x[0] >= 0;
  }
  S* a = aw + B.eoff + (act ? i : 0);
  const S* w = work + B.eoff + (act ? i : 0);
  S qeL[5], qeR[5], ue0L[5], ue0R[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) qeL[m] = qeR[m] = S(0);
  if (va || vb) {
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      qeL[m] = w[(E_TRACE + m) * LE - 1];
      qeR[m] = w[(E_TRACE + 5 + m) * LE];
    }
  }
  prim_to_cons(qeL, G, ue0L);
  prim_to_cons(qeR, G, ue0R);
  S tLb[5] = {0, 0, 0, 0, 0}, tRb[5] = {0, 0, 0, 0, 0};
  // one pair's corrected-state adjoints -> each owned zone's sum of sides
  auto sides = [&](int pr, bool hi_ok, bool lo_ok, const S uL[5], const S uR[5]) {
#pragma unroll
    for (int m = 0; m < 5; ++m) buf[m][l] = uL[m];
    __syncthreads();
    if (own) {
#pragma unroll
      for (int m = 0; m < 5; ++m)
        a[(A_U2 + (pr * 2 + 0) * 5 + m) * LE] = (hi_ok ? buf[m][l + 1] : S(0)) + (lo_ok ? uR[m] : S(0));
    }
    __syncthreads();
  };
  {
    S uL[5] = {0, 0, 0, 0, 0}, uR[5] = {0, 0, 0, 0, 0};
    if (va)
      adj_r2_pair<0, 1, true, S>(w, a, LE, 1, z.E[0], qeL, qeR, ue0L, ue0R, G, sc, B, z.x[0], tLb, tRb, uL, uR);
    sides(pa, ta && up, va, uL, uR);
  }
  {
    S uL[5] = {0, 0, 0, 0, 0}, uR[5] = {0, 0, 0, 0, 0};
    if (vb)
      adj_r2_pair<0, 2, true, S>(w, a, LE, 1, (long long)z.E[0] * z.E[1], qeL, qeR, ue0L, ue0R, G, sc, B, z.x[0],
                                 tLb, tRb, uL, uR);
    sides(pb, tb && up, vb, uL, uR);
  }
  if (own && (va || vb)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      a[(A_TB + m) * LE - 1] += tLb[m];
      a[(A_TB + 5 + m) * LE] += tRb[m];
    }
  }
}

template <int d, class S>
__device__ __forceinline__ void adj_r1_body(const Tile* __restrict__ tiles, int ntiles,
                                            const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                            long long LE, S* __restrict__ aw, const Gas<S>& G,
                                            const StepConsts* __restrict__ sc) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  constexpr int da = (d == 0) ? 1 : 0, db = (d == 2) ? 1 : 2;  // the two axes whose pairs use F1^d
  constexpr int pa = pair_index(da, d), pb = pair_index(db, d);
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0) return;
  const long long sd = stride(z.E, d);
  const S* w = work + B.eoff + z.e;
  S* a = aw + B.eoff + z.e;
  const S c3 = SC<S>::dt3h(sc)[d];
  S Fb[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* ap = a + (A_U2 + (pa * 2 + 0) * 5 + m) * LE;
    const S* am = a + (A_U2 + (pa * 2 + 1) * 5 + m) * LE;
    const S* bp = a + (A_U2 + (pb * 2 + 0) * 5 + m) * LE;
    const S* bm = a + (A_U2 + (pb * 2 + 1) * 5 + m) * LE;
    // pairs of the x faces: the stage-2 reverse stored each zone's two sides summed
    S sa;
    if constexpr (da == 0)
      sa = ap[0] - ap[-sd];
    else
      sa = (ap[0] + am[0]) - (ap[-sd] + am[-sd]);
    const S sb = (bp[0] + bm[0]) - (bp[-sd] + bm[-sd]);
    // formed before the solve starts (opaque): otherwise the twenty loads
    // stay in flight, in registers, through the forward solve
    Fb[m] = opaque(c3 * sa + c3 * sb);
  }
  S L[5], R[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    L[m] = w[(E_TRACE + (d * 2 + 0) * 5 + m) * LE - sd];
    R[m] = w[(E_TRACE + (d * 2 + 1) * 5 + m) * LE];
  }
  const int ws = wall_states<d>(B, z.x[d], L, R);
  S Lb[5] = {0, 0, 0, 0, 0}, Rb[5] = {0, 0, 0, 0, 0};
  riemann_vjp<d>(L, R, G, Fb, Lb, Rb);
  wall_states_vjp<d>(ws, Lb, Rb);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    a[(A_TB + (d * 2 + 0) * 5 + m) * LE - sd] += Lb[m];
    a[(A_TB + (d * 2 + 1) * 5 + m) * LE] += Rb[m];
  }
}

// Axes y and z (blockIdx.y 0, 1); x runs in k_adj_r1_trace_x.
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_adj_r1(const Tile* __restrict__ tiles, int ntiles,
                                                 const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                                 long long LE, S* __restrict__ aw, Gas<S> G,
                                                 const StepConsts* __restrict__ sc) {
  if (blockIdx.y == 0)
    adj_r1_body<1, S>(tiles, ntiles, boxes, work, LE, aw, G, sc);
  else
    adj_r1_body<2, S>(tiles, ntiles, boxes, work, LE, aw, G, sc);
}

// Trace reverse of one traced zone along axis d: the contributions of its
// primitives' parabolas to the primitives of its 5-zone stencil, one field
// at a time — the transverse velocities first (each alone), then density,
// normal velocity and pressure together — handed to out(m, ab) in that
// order (ab[o]: the contribution to the zone at offset o - 2), plus the
// sound-speed (cb) and flattening-coefficient (phib) adjoints; tbv(side, m):
// the zone's traced-state adjoint of field m on that side.  act false:
// no memory is touched and out receives zeros (the lane still calls out,
// which may hold workgroup barriers).
template <int d, class S, class TB, class Out>
__device__ __forceinline__ void trace_reverse_zone(bool act, const S* __restrict__ prim, long long LS,
                                                   long long base, long long st, S phi, TB&& tbv,
                                                   const Gas<S>& G, S dtdx, S& cb_out, S& phib_out,
                                                   Out&& out) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  constexpr int fm[3] = {0, 1 + d, 4};
  S un = 0, c = 0;
  if (act) {
    un = prim[(1 + d) * LS + base];
    c = sound_speed(prim[base], prim[4 * LS + base], G);
  }
  S phib = 0;
  // one field's parabola adjoint -> its stencil contributions (the stencil
  // reloaded through an opaque address, so that the first loads' registers
  // do not stay live in between)
  auto contrib = [&](int m, S aLb, S aRb, S a6b, S centre) {
    S ab[5] = {0, 0, 0, 0, 0};
    if (act) {
      const S* p = opaque(prim + m * LS + base);
      const S as5[5] = {p[-2 * st], p[-st], p[0], p[st], p[2 * st]};
      ppm_parabola_vjp(as5, phi, G, aLb, aRb, a6b, ab, phib);
      ab[2] += centre;
    }
    out(m, ab);
  };
  // the transverse velocities one at a time
  S lambt[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = (i == 0) ? 1 + t1 : 1 + t2;
    S aLb = 0, aRb = 0, a6b = 0;
    if (act) {
      const S* p = opaque(prim + m * LS + base);
      S aL, aR, a6;
      ppm_parabola(p[-2 * st], p[-st], p[0], p[st], p[2 * st], phi, G, aL, aR, a6);
      trace_transverse_vjp(aL, aR, a6, un, c, dtdx, tbv(0, m), tbv(1, m), aLb, aRb, a6b, lambt);
    }
    contrib(m, aLb, aRb, a6b, S(0));
  }
  // then density, normal velocity and pressure together
  S aL[5], aR[5], a6[5], qpb[5], qmb[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int m = fm[i];
    aL[m] = aR[m] = a6[m] = qpb[m] = qmb[m] = S(0);
    if (act) {
      const S* p = opaque(prim + m * LS + base);
      ppm_parabola(p[-2 * st], p[-st], p[0], p[st], p[2 * st], phi, G, aL[m], aR[m], a6[m]);
      qpb[m] = tbv(0, m);
      qmb[m] = tbv(1, m);
    }
  }
  const S r = act ? prim[base] : S(1);
  S aLb[5], aRb[5], a6b[5], rb = 0, unb = 0, cb = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) aLb[fm[i]] = aRb[fm[i]] = a6b[fm[i]] = S(0);
  if (act) trace_zone_vjp<d>(aL, aR, a6, r, un, c, dtdx, G, qpb, qmb, lambt, aLb, aRb, a6b, rb, unb, cb);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int m = fm[i];
    contrib(m, aLb[m], aRb[m], a6b[m], m == 0 ? rb : (m == 1 + d ? unb : S(0)));
  }
  cb_out = cb;
  phib_out = phib;
}

// Trace adjoint of axis d: per traced zone, the contributions to the
// primitives of its 5-zone stencil along d (GT of axis d), the sound speed
// (CB of axis d) and the flattening coefficient (PHB of axis d), stored
// non-temporally: only the gather, several launches later, reads them.  One launch
// per axis: the bodies of several axes in one kernel would share the
// register budget of the largest and spill.  The two field groups keep the
// FP64 kernel at 168 registers, 3 waves per SIMD (a few values spill).
template <int d, class S>
__global__ void __launch_bounds__(MAX_TILE) __attribute__((amdgpu_waves_per_eu(3)))
k_adj_trace(const Tile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
            const S* __restrict__ prim, long long LS, const S* __restrict__ work, long long LE,
            S* __restrict__ aw, Gas<S> G, const StepConsts* __restrict__ sc) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  const int NS[3] = {B.n[0] + 2 * NG, B.n[1] + 2 * NG, B.n[2] + 2 * NG};
  const long long base = pidx(B, z.x[0], z.x[1], z.x[2]);
  const long long st = stride(NS, d);
  const S phi = work[E_FLAT * LE + B.eoff + z.e];
  S* a = aw + B.eoff + z.e;
  S cb, phib;
  trace_reverse_zone<d>(true, prim, LS, base, st, phi,
                        [&](int side, int m) { return a[(A_TB + (d * 2 + side) * 5 + m) * LE]; }, G,
                        SC<S>::dtdx(sc)[d], cb, phib, [&](int m, const S ab[5]) {
#pragma unroll
                          for (int o = 0; o < 5; ++o) __builtin_nontemporal_store(ab[o], &a[(A_GT + (d * 5 + m) * 5 + o) * LE]);
                        });
  __builtin_nontemporal_store(cb, &a[(A_CB + d) * LE]);
  __builtin_nontemporal_store(phib, &a[(A_PHB + d) * LE]);
}

// Stage-1 reverse and trace adjoint along x in one kernel, over runs of
// XF_OWNED - 1 traced zones: lane l takes slot start - 2 + l, so the run's
// zones have two traced halo zones on each side and the last lane one more
// slot.  Each lane first reverses the stage-1 solve of the x face at its
// slot; the zone's traced-state adjoints are then what the stage-3 and
// stage-2 reverses left plus the two faces' parts (the high side's from the
// next lane, through LDS), so they are never written back.  The trace
// reverse follows; each field's stencil contributions are summed in LDS, so
// that a traced zone's own GT[x][m] centre slot holds the whole x part of its
// primitive adjoint (the gather's order of terms, the same bits).
// Contributions to the stored zones beyond a row's traced range (x < -1 or
// x > n) stay in their GT slots, as in the per-zone form.
template <class S>
__global__ void __launch_bounds__(XF_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_adj_r1_trace_x(const Tile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
                 const S* __restrict__ prim, long long LS, const S* __restrict__ work, long long LE,
                 S* __restrict__ aw, Gas<S> G, const StepConsts* __restrict__ sc) {
  constexpr int pa = pair_index(1, 0), pb = pair_index(2, 0);  // the pairs that use the x stage-1 fluxes
  __shared__ S buf[5][XF_THREADS];
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;  // the whole workgroup
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  const int l = threadIdx.x;
  const int E0 = B.n[0] + 2;
  const int NE = E0 * (B.n[1] + 2) * (B.n[2] + 2);
  const int i = tl.start - 2 + l;
  const bool slot = i >= 0 && i < NE;
  const bool act = slot && l < XF_THREADS - 1;  // the zones this run traces
  const bool own = i >= tl.start && i < tl.end;
  int x = 0, y = 0, zz = 0;
  if (slot) {
    const unsigned r = div31((unsigned)i, B.de[0]), k = div31(r, B.de[1]);
    x = i - (int)r * E0 - 1;
    y = (int)(r - k * (unsigned)(B.n[1] + 2)) - 1;
    zz = (int)k - 1;
  }
  S* a = aw + B.eoff + (slot ? i : 0);
  const S* w = work + B.eoff + (slot ? i : 0);
  // stage-1 reverse of the face at the lane's slot (zone i - 1 high side,
  // zone i low side)
  const bool face = slot && x >= 0;
  S Lb[5] = {0, 0, 0, 0, 0}, Rb[5] = {0, 0, 0, 0, 0};
  if (face) {
    const S c3 = SC<S>::dt3h(sc)[0];
    S Fb[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const S* ap = a + (A_U2 + (pa * 2 + 0) * 5 + m) * LE;
      const S* am = a + (A_U2 + (pa * 2 + 1) * 5 + m) * LE;
      const S* bp = a + (A_U2 + (pb * 2 + 0) * 5 + m) * LE;
      const S* bm = a + (A_U2 + (pb * 2 + 1) * 5 + m) * LE;
      const S sa = (ap[0] + am[0]) - (ap[-1] + am[-1]);
      const S sb = (bp[0] + bm[0]) - (bp[-1] + bm[-1]);
      Fb[m] = opaque(c3 * sa + c3 * sb);
    }
    S L[5], R[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      L[m] = w[(E_TRACE + m) * LE - 1];
      R[m] = w[(E_TRACE + 5 + m) * LE];
    }
    const int ws = wall_states<0>(B, x, L, R);
    riemann_vjp<0>(L, R, G, Fb, Lb, Rb);
    wall_states_vjp<0>(ws, Lb, Rb);
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) buf[m][l] = Lb[m];
  __syncthreads();
  // the zone's traced-state adjoints, complete
  S qp[5] = {0, 0, 0, 0, 0}, qm[5] = {0, 0, 0, 0, 0};
  if (act) {
    const bool up = x + 1 <= B.n[0];  // the face above the zone is in its row
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const S p0 = a[(A_TB + m) * LE], m0 = a[(A_TB + 5 + m) * LE];
      qp[m] = up ? p0 + buf[m][l + 1] : p0;
      qm[m] = face ? m0 + Rb[m] : m0;
    }
  }
  __syncthreads();
  const long long base = act ? pidx(B, x, y, zz) : 0;
  const S phi = act ? work[E_FLAT * LE + B.eoff + i] : S(0);
  S cb, phib;
  trace_reverse_zone<0>(act, prim, LS, base, 1, phi, [&](int side, int m) { return side == 0 ? qp[m] : qm[m]; },
                        G, SC<S>::dtdx(sc)[0], cb, phib, [&](int m, const S ab[5]) {
#pragma unroll
                          for (int o = 0; o < 5; ++o) buf[o][l] = ab[o];
                          __syncthreads();
                          if (own) {
                            // zone x receives slot o + 2 of zone x - o, o = -2..2, while
                            // that zone lies in the row's traced range
                            S sum = S(0);
#pragma unroll
                            for (int o = -2; o <= 2; ++o)
                              if (x - o >= -1 && x - o <= B.n[0]) sum += buf[o + 2][l - o];
                            a[(A_GT + m * 5 + 2) * LE] = sum;
#pragma unroll
                            for (int o = 0; o < 5; ++o)
                              if (o != 2 && (x + o - 2 < -1 || x + o - 2 > B.n[0]))
                                a[(A_GT + m * 5 + o) * LE] = ab[o];
                          }
                          __syncthreads();
                        });
  if (own) {
    a[A_CB * LE] = cb;
    a[A_PHB * LE] = phib;
  }
}

// Flattening adjoint: the derivative of phi = min_d (1 - chi_d) through the
// selected axis, the selected shock-detector coefficient and its clamp,
// into the pressures at offsets -3..3 along that axis (A_GF, A_SEL).
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_adj_flatten(const Tile* __restrict__ tiles, int ntiles,
                                                      const DevBox* __restrict__ boxes,
                                                      const S* __restrict__ prim, long long LS,
                                                      S* __restrict__ aw, long long LE, Gas<S> G) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  S* a = aw + B.eoff + z.e;
  S gf[7] = {0, 0, 0, 0, 0, 0, 0};
  int sel = -1;
  if (G.flattening) {
    const int NS[3] = {B.n[0] + 2 * NG, B.n[1] + 2 * NG, B.n[2] + 2 * NG};
    const long long base = pidx(B, z.x[0], z.x[1], z.x[2]);
    S phi = ONE;
    int dsel = 0, osel = 0;
    bool live = false;
    S ps[7];  // pressures along the selected axis
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long long st = stride(NS, d);
      const S* pp = prim + 4 * LS + base;
      const S* uu = prim + (1 + d) * LS + base;
      S p[7], u[5];
#pragma unroll
      for (int o = -3; o <= 3; ++o) p[o + 3] = pp[o * st];
#pragma unroll
      for (int o = -2; o <= 2; ++o) u[o + 2] = uu[o * st];
      // chit(o): value and whether its derivative is live
      auto chit = [&](int o, bool& alive) -> S {
        const S dp1 = p[o + 4] - p[o + 2];
        const S dp2 = p[o + 5] - p[o + 1];
        const S zeta = sabs(dp1) / smax(sabs(dp2), G.small_pres);
        const S x = TEN * (zeta - C075);
        const S zz = smin(smax(x, S(0)), ONE);
        const bool compress = (u[o + 1] - u[o + 3]) > S(0);
        const bool strong = sabs(dp1) > C033 * smin(p[o + 4], p[o + 2]);
        alive = compress && strong && !(x < S(0)) && !(ONE < x);
        return (compress && strong) ? zz : S(0);
      };
      const S dp1 = p[4] - p[2];
      bool am, a0, ap;
      const S cm = chit(-1, am), c0 = chit(0, a0), cp = chit(1, ap);
      S chi;
      int o;
      if (dp1 > S(0)) { chi = smax(c0, cm); o = (c0 < cm) ? -1 : 0; }
      else if (dp1 < S(0)) { chi = smax(c0, cp); o = (c0 < cp) ? 1 : 0; }
      else {
        const S m1 = smax(cm, c0);
        const int o1 = (cm < c0) ? 0 : -1;
        chi = smax(m1, cp);
        o = (m1 < cp) ? 1 : o1;
      }
      const bool lv = (o == -1) ? am : (o == 0 ? a0 : ap);
      const S val = ONE - chi;
      if (d == 0 || val < phi) {
        phi = val;
        dsel = d;
        osel = o;
        live = lv;
#pragma unroll
        for (int k = 0; k < 7; ++k) ps[k] = p[k];
      }
    }
    const S phib = (a[A_PHB * LE] + a[(A_PHB + 1) * LE]) + a[(A_PHB + 2) * LE];
    if (live && phib != S(0)) {
      const int o = osel;
      // p index k <-> offset k - 3; the detector at o uses k = o+1, o+2, o+4, o+5
      const S p1 = (o < 0) ? ps[0] : (o == 0 ? ps[1] : ps[2]);
      const S p2 = (o < 0) ? ps[1] : (o == 0 ? ps[2] : ps[3]);
      const S p4 = (o < 0) ? ps[3] : (o == 0 ? ps[4] : ps[5]);
      const S p5 = (o < 0) ? ps[4] : (o == 0 ? ps[5] : ps[6]);
      const S dp1 = p4 - p2;
      const S dp2 = p5 - p1;
      const S a2 = sabs(dp2);
      const bool use2 = !(a2 < G.small_pres);
      const S D = smax(a2, G.small_pres);
      const S zeta = sabs(dp1) / D;
      const S zetab = -phib * TEN;  // phi = 1 - chi, chi = zz, zz = 10 (zeta - 0.75)
      const S dp1b = zetab * ((dp1 < S(0)) ? -ONE : ONE) / D;
      const S Db = -zetab * zeta / D;
      const S dp2b = use2 ? Db * ((dp2 < S(0)) ? -ONE : ONE) : S(0);
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        S v = S(0);
        if (k == o + 4) v += dp1b;
        if (k == o + 2) v -= dp1b;
        if (k == o + 5) v += dp2b;
        if (k == o + 1) v -= dp2b;
        gf[k] = v;
      }
      sel = dsel;
    }
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) a[(A_GF + k) * LE] = gf[k];
  a[A_SEL * LE] = (S)sel;
}

// Gather of all primitive adjoints of a stored zone (the trace contributions
// of the zones whose stencils cover it, its sound-speed adjoints, the
// flattening contributions), then the reverse of its primitive conversion:
// UB = (valid ? update part : 0) + J^T qb.  Clears the output's ghost zones
// (its valid zones are written by the fill transpose).
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_adj_gather(const Tile* __restrict__ tilesS, int ntiles,
                                                     const DevBox* __restrict__ boxes,
                                                     const S* __restrict__ aw, long long LE,
                                                     const double* __restrict__ U, double* __restrict__ as,
                                                     long long LS, Gas<S> G, double* __restrict__ Ub,
                                                     const double* __restrict__ Ubn,
                                                     const StepConsts* __restrict__ sc, int grav, double g0,
                                                     double g1, double g2) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tilesS[tt];
  const DevBox B = boxes[tl.box];
  const int NS[3] = {B.n[0] + 2 * NG, B.n[1] + 2 * NG, B.n[2] + 2 * NG};
  const long long NSS = (long long)NS[0] * NS[1] * NS[2];
  const int idx = tl.start + (int)threadIdx.x;  // below 2^31: tile bounds are ints
  if (idx >= tl.end) return;
  int j[3];
  const unsigned r = div31((unsigned)idx, B.ds[0]), k = div31(r, B.ds[1]);
  j[0] = idx - (int)r * NS[0] - NG;
  j[1] = (int)(r - k * (unsigned)NS[1]) - NG;
  j[2] = (int)k - NG;
  S qb[6] = {0, 0, 0, 0, 0, 0};
  // along x the trace adjoint left the summed contributions in each traced
  // zone's centre slot; stored zones beyond a row's traced range read the
  // slots of the traced zones within two
  const bool xin = j[0] >= -1 && j[0] <= B.n[0];
  if (xin && in_e(j, B)) {
    const S* g = aw + B.eoff + eidx(B, j[0], j[1], j[2]);
#pragma unroll
    for (int m = 0; m < 5; ++m) qb[m] = g[(A_GT + m * 5 + 2) * LE];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d == 0 && xin) continue;
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      int y[3] = {j[0], j[1], j[2]};
      y[d] -= o;
      if (!in_e(y, B)) continue;
      const S* g = aw + B.eoff + eidx(B, y[0], y[1], y[2]);
#pragma unroll
      for (int m = 0; m < 5; ++m) qb[m] += g[(A_GT + (d * 5 + m) * 5 + (o + 2)) * LE];
    }
  }
  if (in_e(j, B)) {
    const S* g = aw + B.eoff + eidx(B, j[0], j[1], j[2]);
    qb[5] = (g[A_CB * LE] + g[(A_CB + 1) * LE]) + g[(A_CB + 2) * LE];
  }
  if (G.flattening) {
    S acc = S(0);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int o = -3; o <= 3; ++o) {
        int y[3] = {j[0], j[1], j[2]};
        y[d] -= o;
        if (!in_e(y, B)) continue;
        const long long e = B.eoff + eidx(B, y[0], y[1], y[2]);
        if (aw[A_SEL * LE + e] == (S)d) acc += aw[(A_GF + o + 3) * LE + e];
      }
    qb[4] += acc;
  }
  S uc[5], ub[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 5; ++c) uc[c] = (S)U[B.soff + idx + c * NSS];
  prim_cell_vjp(uc, G, qb, ub);
  const bool valid = j[0] >= 0 && j[0] < B.n[0] && j[1] >= 0 && j[1] < B.n[1] && j[2] >= 0 && j[2] < B.n[2];
  // valid zones: plus the new state's adjoint through the update (identity
  // and Heun source); ghost zones: only what the stencils gave them
  double direct[5] = {0, 0, 0, 0, 0};
  if (valid) {
    double ubn[5], uf[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) ubn[c] = Ubn[B.soff + idx + c * NSS];
    heun_reverse(ubn, grav, sc->dt, sc->hdt, g0, g1, g2, uf, direct);
  }
  double* u = as + AS_UB * LS + B.poff + idx;
#pragma unroll
  for (int c = 0; c < 5; ++c) u[c * LS] = direct[c] + (double)ub[c];
  if (!valid) {
#pragma unroll
    for (int c = 0; c < 5; ++c) Ub[B.soff + idx + c * NSS] = 0.0;
  }
}

// Transpose of the ghost fill: every valid zone of a source box sums the
// adjoints of the ghost zones that copied it (signs of reflections applied),
// in the fixed order of the plan; writes the result to Ub (valid zones).
// Only the descriptors listed for the zone's class are visited; zones more
// than NG from every face have none.
__global__ void __launch_bounds__(MAX_TILE) k_adj_fill(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   const FillDesc* __restrict__ desc,
                                                   const int* __restrict__ inv_start, const int* __restrict__ inv_idx,
                                                   const double* __restrict__ as, long long LS,
                                                   double* __restrict__ Ub) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[0] < 0 || z.x[0] >= B.n[0] || z.x[1] < 0 || z.x[1] >= B.n[1] || z.x[2] < 0 || z.x[2] >= B.n[2]) return;
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
  const long long NS = (long long)N0 * N1 * N2;
  const long long li = ((long long)(z.x[2] + NG) * N1 + (z.x[1] + NG)) * N0 + (z.x[0] + NG);
  double acc[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) acc[c] = as[(AS_UB + c) * LS + B.poff + li];
  const int cls = inv_axis_class(z.x[0], B.n[0]) + 4 * inv_axis_class(z.x[1], B.n[1]) +
                  16 * inv_axis_class(z.x[2], B.n[2]);
  const int k0 = inv_start[tl.box * INV_CLASSES + cls], k1 = inv_start[tl.box * INV_CLASSES + cls + 1];
  for (int k = k0; k < k1; ++k) {
    const FillDesc D = desc[inv_idx[k]];
    int lo[3], hi[3];
    bool hit = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int y = z.x[d];
      if (D.a[d] == 1) { lo[d] = hi[d] = y - D.c[d]; }
      else if (D.a[d] == -1) { lo[d] = hi[d] = D.c[d] - y; }
      else { hit = hit && y == D.c[d]; lo[d] = D.lo[d]; hi[d] = D.hi[d]; }
      hit = hit && lo[d] >= D.lo[d] && hi[d] <= D.hi[d];
    }
    if (!hit) continue;
    const DevBox Bd = boxes[D.dst];
    const int M0 = Bd.n[0] + 2 * NG, M1 = Bd.n[1] + 2 * NG;
    for (int x2 = lo[2]; x2 <= hi[2]; ++x2)
      for (int x1 = lo[1]; x1 <= hi[1]; ++x1)
        for (int x0 = lo[0]; x0 <= hi[0]; ++x0) {
          const long long gi = Bd.poff + ((long long)(x2 + NG) * M1 + (x1 + NG)) * M0 + (x0 + NG);
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            const double v = as[(AS_UB + c) * LS + gi];
            const bool neg = c >= 1 && c <= 3 && ((D.sign >> (c - 1)) & 1);
            acc[c] += neg ? -v : v;
          }
        }
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) Ub[B.soff + li + c * NS] = acc[c];
}

template <class S>
hipError_t adjoint_impl(const DevLevel& L, int nS, int nE, int nX, int nXA, const double* U, const double* Ubn,
                        FluxBar fb,
                        double* Ub, const void* work, void* awork, const Gas<S>& G, int grav, const double g[3],
                        hipStream_t s) {
  const S* prim = (const S*)work;
  const S* ework = prim + P_PLANES * L.LS;
  double* as = (double*)awork;
  S* aw = (S*)(as + A_SPLANES * L.LS);
  const dim3 blk(L.tile);
  // every workspace entry is written before it is read: each reverse stage
  // writes all entries it owns, zeros included
  const int gE = xcd_grid(nE), gS = xcd_grid(nS);
  hipLaunchKernelGGL(k_adj_r3_x<S>, dim3(xcd_grid(nX)), dim3(XF_THREADS), 0, s, L.tilesX, nX, L.boxes, ework, L.LE,
                     aw, G, L.consts, Ubn, fb, grav, g[0], g[1], g[2]);
  if constexpr (sizeof(S) == sizeof(double))
    hipLaunchKernelGGL(k_adj_r3_f64, dim3(gE, 2), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, aw, G, L.consts,
                       Ubn, fb, grav, g[0], g[1], g[2]);
  else
    hipLaunchKernelGGL(k_adj_r3_f32, dim3(gE, 2), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, aw, G, L.consts,
                       Ubn, fb, grav, g[0], g[1], g[2]);
  hipLaunchKernelGGL(k_adj_r2_x<S>, dim3(xcd_grid(nX)), dim3(XF_THREADS), 0, s, L.tilesX, nX, L.boxes, ework, L.LE,
                     aw, G, L.consts);
  hipLaunchKernelGGL(k_adj_r2<S>, dim3(gE, 2), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, aw, G, L.consts);
  hipLaunchKernelGGL(k_adj_r1<S>, dim3(gE, 2), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, aw, G, L.consts);
  hipLaunchKernelGGL(k_adj_r1_trace_x<S>, dim3(xcd_grid(nXA)), dim3(XF_THREADS), 0, s, L.tilesXA, nXA, L.boxes,
                     prim, L.LS, ework, L.LE, aw, G, L.consts);
  hipLaunchKernelGGL((k_adj_trace<1, S>), dim3(gE), blk, 0, s, L.tilesE, nE, L.boxes, prim, L.LS, ework, L.LE,
                     aw, G, L.consts);
  hipLaunchKernelGGL((k_adj_trace<2, S>), dim3(gE), blk, 0, s, L.tilesE, nE, L.boxes, prim, L.LS, ework, L.LE,
                     aw, G, L.consts);
  if (G.flattening)
    hipLaunchKernelGGL(k_adj_flatten<S>, dim3(gE), blk, 0, s, L.tilesE, nE, L.boxes, prim, L.LS, aw, L.LE, G);
  hipLaunchKernelGGL(k_adj_gather<S>, dim3(gS), blk, 0, s, L.tilesS, nS, L.boxes, aw, L.LE, U, as, L.LS, G, Ub,
                     Ubn, L.consts, grav, g[0], g[1], g[2]);
  hipLaunchKernelGGL(k_adj_fill, dim3(gE), blk, 0, s, L.tilesE, nE, L.boxes, L.desc, L.inv_start, L.inv_idx, as,
                     L.LS, Ub);
  return hipGetLastError();
}

}  // namespace

size_t adjoint_workspace_bytes(long long LS, long long LE, int precision) {
  const size_t se = precision == 1 ? sizeof(float) : sizeof(double);
  return sizeof(double) * (size_t)(A_SPLANES * LS) + se * (size_t)(A_EPLANES * LE);
}

hipError_t launch_adjoint(const DevLevel& L, int precision, int nS, int nE, int nX, int nXA, const double* U,
                          const double* Ubn,
                          FluxBar fb, double* Ub, const void* work, void* awork, double gamma, double small_dens,
                          double small_pres, int limiter, int flattening, int iters, int grav, const double g[3],
                          hipStream_t s) {
  if (precision == 1)
    return adjoint_impl<float>(L, nS, nE, nX, nXA, U, Ubn, fb, Ub, work, awork,
                               make_gas<float>(gamma, small_dens, small_pres, limiter, flattening, iters, grav),
                               grav, g, s);
  return adjoint_impl<double>(L, nS, nE, nX, nXA, U, Ubn, fb, Ub, work, awork,
                              make_gas<double>(gamma, small_dens, small_pres, limiter, flattening, iters, grav),
                              grav, g, s);
}

}  // namespace ppm

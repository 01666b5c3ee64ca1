// gfx950 kernels of the unsplit PPM step.
//
// The step runs as a chain of stages, each one launch over a flat tile list
// (all boxes of the level, or one box for the per-box form):
//   prim     conserved -> primitive on every stored zone            (O2)
//   flatten  shock-flattening coefficient on the traced zones        (O3)
//   trace    PPM parabolas + characteristic tracing, one axis/thread (O4, O5)
//   riemann1 normal-predictor fluxes F^d                             (O7)
//   riemann2 single-transverse corrected states, fluxes F^{d|t}      (O8)
//   riemann3 double-transverse corrected states, fluxes F^{d,n+1/2}  (O9)
//   update   conservative update in FP64 (+ Heun gravity source)     (O10)
// Intermediates live in structure-of-arrays planes in HBM (one plane per
// quantity, every box's grid contiguous inside a plane), so each lane of a
// wavefront touches consecutive addresses on every load and store.
//
// Fused forms of some stage pairs cut that traffic and give the same bits:
// the front end (trace + riemann1) along x with the face states exchanged
// by lane shuffles (k_front_x, the default), also along y and z
// (k_front_yz), or streamed along z through LDS (k_front_stream); the final
// stage (riemann3 + update) in bricks (k_final_update) or streamed along z
// (k_final_stream), the final fluxes kept in LDS.
//
// Every formula is a C expression evaluated as written (no contraction:
// built with -ffp-contract=off).  The pointwise arithmetic (ppm_math.h)
// uses reciprocal forms of the method's divisions, so the results agree
// with a serial evaluation of the plain definition to rounding.
#include <hip/hip_runtime.h>

#include "ppm_device.h"
#include "ppm_internal.h"
#include "ppm_math.h"

namespace ppm {
namespace {

// ------------------------------------------------------------- kernels -----
__device__ __forceinline__ void step_consts(StepConsts* c, double dt, const double* dt_dev, double h0, double h1,
                                            double h2, double g0, double g1, double g2) {
  const double t = dt_dev ? dt_dev[0] : dt;
  const double h[3] = {h0, h1, h2}, g[3] = {g0, g1, g2};
  c->dt = t;
  c->hdt = 0.5 * t;
  for (int d = 0; d < 3; ++d) {
    c->dtdx[d] = t / h[d];
    c->d_dtdx[d] = t / h[d];
    c->d_dt2h[d] = t / (2.0 * h[d]);
    c->d_dt3h[d] = t / (3.0 * h[d]);
    c->d_hdtg[d] = 0.5 * t * g[d];
    c->f_dtdx[d] = (float)c->d_dtdx[d];
    c->f_dt2h[d] = (float)c->d_dt2h[d];
    c->f_dt3h[d] = (float)c->d_dt3h[d];
    c->f_hdtg[d] = (float)c->d_hdtg[d];
  }
}

__global__ void __launch_bounds__(64) k_step_consts(StepConsts* c, double dt, const double* dt_dev,
                                                    double h0, double h1, double h2, double g0,
                                                    double g1, double g2) {
  if (threadIdx.x == 0) step_consts(c, dt, dt_dev, h0, h1, h2, g0, g1, g2);
}

// O2 on every stored zone: (rho, u, v, w, p) planes.  The sound speed is
// formed here for the range check only: the stages that use it form it again
// from rho and p (one plane less to write and to read).
// t: the tile (-1: none), here and in the other stage bodies.
template <class S>
__device__ __forceinline__ void prim_body(int t, const Tile* __restrict__ tiles, const DevBox* __restrict__ boxes,
                                          const double* __restrict__ U, S* __restrict__ prim, long long LS,
                                          const Gas<S>& G, int* flags) {
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  const long long NS = (long long)(B.n[0] + 2 * NG) * (B.n[1] + 2 * NG) * (B.n[2] + 2 * NG);
  const long long idx = (long long)tl.start + threadIdx.x;
  if (idx >= tl.end) return;
  const double* u = U + B.soff + idx;
  S uc[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) uc[c] = (S)u[c * NS];
  int fl = 0;
  const S r = uc[0];
  const S vx = uc[1] / r, vy = uc[2] / r, vz = uc[3] / r;
  const S ke = HALF * r * ((vx * vx + vy * vy) + vz * vz);
  S p = G.gm1 * (uc[4] - ke);
  bool fin = true;
#pragma unroll
  for (int c = 0; c < 5; ++c) fin = fin && __builtin_isfinite(uc[c]);
  if (!fin || !(r > S(0)) || !(p > S(0))) fl |= PPM_FLAG_NONPHYS;
  if (p < G.small_pres) fl |= PPM_FLAG_FLOOR;
  p = smax(p, G.small_pres);
  const S c = sound_speed(r, p, G);
  // magnitudes for which the shortened FP64 divisions and roots of the
  // later stages are the IEEE results (zero velocities included)
  if (!(in_range(r) && in_range(p) && in_range(c) && speed_in_range(vx) && speed_in_range(vy) &&
        speed_in_range(vz)))
    fl |= PPM_FLAG_RANGE;
  S* q = prim + B.poff + idx;
  __builtin_nontemporal_store(r, &q[0]);
  __builtin_nontemporal_store(vx, &q[LS]);
  __builtin_nontemporal_store(vy, &q[2 * LS]);
  __builtin_nontemporal_store(vz, &q[3 * LS]);
  __builtin_nontemporal_store(p, &q[4 * LS]);
  raise_flags(flags, fl);
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_prim(const Tile* __restrict__ tiles, int ntiles,
                                               const DevBox* __restrict__ boxes,
                                               const double* __restrict__ U, S* __restrict__ prim,
                                               long long LS, Gas<S> G, int* flags) {
  prim_body(xcd_tile(ntiles), tiles, boxes, U, prim, LS, G, flags);
}


// O3 on the traced zones.
template <class S>
__device__ __forceinline__ void flatten_body(int t, const Tile* __restrict__ tiles,
                                             const DevBox* __restrict__ boxes, const S* __restrict__ prim,
                                             long long LS, S* __restrict__ work, long long LE, const Gas<S>& G) {
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  S phi = ONE;
  if (G.flattening) {
    const int NS[3] = {B.n[0] + 2 * NG, B.n[1] + 2 * NG, B.n[2] + 2 * NG};
    const long long base = pidx(B, z.x[0], z.x[1], z.x[2]);
    const S* pp = prim + 4 * LS + base;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long long st = stride(NS, d);
      const S* uu = prim + (1 + d) * LS + base;
      // p at offsets -2..2 and u at -2..2 (index offset + 3, offset + 2)
      // are read here; p at -3 and 3 only by a neighbour's coefficient at a
      // strong compression (a branch that, away from shocks, no lane of a
      // wave takes)
      S p[7], u[5];
#pragma unroll
      for (int o = -2; o <= 2; ++o) p[o + 3] = pp[o * st];
#pragma unroll
      for (int o = -2; o <= 2; ++o) u[o + 2] = uu[o * st];
      // shock-detector coefficient at offset o; the pressure ratio (one
      // division) only where the zone is a strong compression
      auto chit = [&](int o) -> S {
        const S dp1 = p[o + 4] - p[o + 2];
        const bool compress = (u[o + 1] - u[o + 3]) > S(0);
        const bool strong = sabs(dp1) > C033 * smin(p[o + 4], p[o + 2]);
        if (!(compress && strong)) return S(0);
        if (o != 0) p[3 + 3 * o] = pp[3 * o * st];
        const S dp2 = p[o + 5] - p[o + 1];
        const S zeta = qdiv(sabs(dp1), smax(sabs(dp2), G.small_pres));
        return smin(smax(TEN * (zeta - C075), S(0)), ONE);
      };
      const S dp1 = p[4] - p[2];
      S chi;
      if (dp1 > S(0)) chi = smax(chit(0), chit(-1));
      else if (dp1 < S(0)) chi = smax(chit(0), chit(1));
      else chi = smax(smax(chit(-1), chit(0)), chit(1));
      phi = (d == 0) ? (ONE - chi) : smin(phi, ONE - chi);
    }
  }
  work[E_FLAT * LE + B.eoff + z.e] = phi;
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_flatten(const Tile* __restrict__ tiles, int ntiles,
                                                  const DevBox* __restrict__ boxes,
                                                  const S* __restrict__ prim, long long LS,
                                                  S* __restrict__ work, long long LE, Gas<S> G) {
  flatten_body(xcd_tile(ntiles), tiles, boxes, prim, LS, work, LE, G);
}

// O4 + O5 along axis d for zone (x, y, z) of box B (e: its index in the
// traced grid): the states at the zone's high (qp) and low (qm) d faces.
template <int d, class S>
__device__ __forceinline__ void trace_at(const DevBox& B, int x, int y, int z, long long e,
                                         const S* __restrict__ prim, long long LS, const S* __restrict__ work,
                                         long long LE, const Gas<S>& G, const StepConsts* __restrict__ sc, S qp[5],
                                         S qm[5], int& fl) {
  const int NS[3] = {B.n[0] + 2 * NG, B.n[1] + 2 * NG, B.n[2] + 2 * NG};
  const long long base = pidx(B, x, y, z);
  const long long st = stride(NS, d);
  // every stencil value loaded before any is used: the limiter's branches
  // would otherwise keep the compiler from issuing a field's loads before the
  // previous field's parabola, one memory round trip per field
  S v[5][5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* a = prim + m * LS + base;
#pragma unroll
    for (int o = 0; o < 5; ++o) v[m][o] = a[(o - 2) * st];
  }
  const S c = sound_speed(v[0][2], v[4][2], G);
  const S phi = work[E_FLAT * LE + B.eoff + e];
  S aL[5], aR[5], a6[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) ppm_parabola(v[m][0], v[m][1], v[m][2], v[m][3], v[m][4], phi, G, aL[m], aR[m], a6[m]);
  const S r = v[0][2], un = v[1 + d][2];
  trace_zone<d>(aL, aR, a6, r, un, c, SC<S>::dtdx(sc)[d], G, SC<S>::hdtg(sc), qp, qm, fl);
}

// Traced states of zone e along d into the workspace planes.
template <int d, class S>
__device__ __forceinline__ void store_traced(S* __restrict__ work, long long LE, const DevBox& B, long long e,
                                             const S qp[5], const S qm[5]) {
  S* w = work + B.eoff + e;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    w[(E_TRACE + (d * 2 + 0) * 5 + m) * LE] = qp[m];
    w[(E_TRACE + (d * 2 + 1) * 5 + m) * LE] = qm[m];
  }
}

// O4 + O5 for one axis (blockIdx.y) on the traced zones.
template <int d, class S>
__device__ __forceinline__ void trace_body(int t, const Tile* __restrict__ tiles,
                                           const DevBox* __restrict__ boxes, const S* __restrict__ prim,
                                           long long LS, S* __restrict__ work, long long LE, const Gas<S>& G,
                                           const StepConsts* __restrict__ sc, int* flags) {
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  S qp[5], qm[5];
  int fl = 0;
  trace_at<d>(B, z.x[0], z.x[1], z.x[2], z.e, prim, LS, work, LE, G, sc, qp, qm, fl);
  store_traced<d>(work, LE, B, z.e, qp, qm);
  raise_flags(flags, fl);
}

// d0: the first axis (the grid's rows are axes d0, d0 + 1, ...).
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_trace(const Tile* __restrict__ tiles, int ntiles,
                                                const DevBox* __restrict__ boxes,
                                                const S* __restrict__ prim, long long LS,
                                                S* __restrict__ work, long long LE, Gas<S> G,
                                                const StepConsts* __restrict__ sc, int* flags, int d0) {
  switch (d0 + (int)blockIdx.y) {
    case 0: trace_body<0>(xcd_tile(ntiles), tiles, boxes, prim, LS, work, LE, G, sc, flags); break;
    case 1: trace_body<1>(xcd_tile(ntiles), tiles, boxes, prim, LS, work, LE, G, sc, flags); break;
    default: trace_body<2>(xcd_tile(ntiles), tiles, boxes, prim, LS, work, LE, G, sc, flags); break;
  }
}

// O7 on the d face at slot xd (between zones xd - 1 and xd along d) whose
// high-side zone has traced-grid index e: L, R the traced states on its two
// sides (overwritten), the flux into the stage-1 plane.
template <int d, class S>
__device__ __forceinline__ void stage1_face(const DevBox& B, int xd, S L[5], S R[5], const Gas<S>& G,
                                            S* __restrict__ work, long long LE, long long e, int& fl) {
  S F[5];
  wall_states<d>(B, xd, L, R);
  riemann<d>(L, R, G, F, fl);
  S* f = work + B.eoff + e;
#pragma unroll
  for (int m = 0; m < 5; ++m) __builtin_nontemporal_store(F[m], &f[(E_F1 + d * 5 + m) * LE]);
}

// O7: F^d at d-face slots x_d in [0, n], transverse in [-1, n].
template <int d, class S>
__device__ __forceinline__ void riemann1_body(int t, const Tile* __restrict__ tiles,
                                              const DevBox* __restrict__ boxes, S* __restrict__ work,
                                              long long LE, const Gas<S>& G, int* flags) {
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0) return;
  const long long st = stride(z.E, d);
  const S* w = work + B.eoff + z.e;
  S L[5], R[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    L[m] = w[(E_TRACE + (d * 2 + 0) * 5 + m) * LE - st];
    R[m] = w[(E_TRACE + (d * 2 + 1) * 5 + m) * LE];
  }
  int fl = 0;
  stage1_face<d>(B, z.x[d], L, R, G, work, LE, z.e, fl);
  raise_flags(flags, fl);
}

// Occupancy requests (measured): riemann1 at 8 waves per SIMD and riemann2
// at 5 fit without spills and run 2-3% faster than the compiler's own
// register choice.  riemann3 (7 waves on its own) at 8 and trace at 6
// spill and are slower.
template <class S>
__global__ void __launch_bounds__(MAX_TILE) __attribute__((amdgpu_waves_per_eu(8))) k_riemann1(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   S* __restrict__ work, long long LE, Gas<S> G,
                                                   int* flags, int d0) {
  switch (d0 + (int)blockIdx.y) {
    case 0: riemann1_body<0>(xcd_tile(ntiles), tiles, boxes, work, LE, G, flags); break;
    case 1: riemann1_body<1>(xcd_tile(ntiles), tiles, boxes, work, LE, G, flags); break;
    default: riemann1_body<2>(xcd_tile(ntiles), tiles, boxes, work, LE, G, flags); break;
  }
}


// O4 + O5 + O7 along x in one kernel: each wavefront traces 64 consecutive
// zones of the traced grid, the first of them the previous wavefront's last
// (a halo: traced, not stored), so the two states of every x face it solves
// sit in neighbouring lanes and the low side arrives by a lane shuffle.
// Rows are consecutive in the linear index, so the lane below holds the x
// neighbour of every zone with x >= 0 (a zone at x = -1 solves no face).
// Same arithmetic as trace_at and stage1_face, so the same bits as the
// staged trace and riemann1 kernels along x.
template <class S>
__global__ void __launch_bounds__(XF_THREADS) k_front_x(const Tile* __restrict__ tiles, int ntiles,
                                                    const DevBox* __restrict__ boxes, const S* __restrict__ prim,
                                                    long long LS, S* __restrict__ work, long long LE, Gas<S> G,
                                                    const StepConsts* __restrict__ sc, int* flags) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;  // the whole workgroup
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  const int lane = threadIdx.x & 63;
  const long long idx = (long long)tl.start + (threadIdx.x >> 6) * 63 + lane - 1;
  const bool own = lane > 0 && idx < tl.end;
  const bool have = own || (lane == 0 && idx >= 0 && idx < tl.end);
  const int E0 = B.n[0] + 2, E1 = B.n[1] + 2;
  const unsigned row = have ? div31((unsigned)idx, B.de[0]) : 0u, k = div31(row, B.de[1]);
  const int x = have ? (int)(idx - (long long)row * E0) - 1 : 0;
  const int y = (int)(row - k * (unsigned)E1) - 1, z = (int)k - 1;
  S qp[5], qm[5];
  int fl = 0;
  if (have) {
    trace_at<0>(B, x, y, z, idx, prim, LS, work, LE, G, sc, qp, qm, fl);
    if (own) store_traced<0>(work, LE, B, idx, qp, qm);
  } else {
#pragma unroll
    for (int m = 0; m < 5; ++m) qp[m] = qm[m] = S(0);
  }
  S L[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) L[m] = __shfl_up(qp[m], 1, 64);
  if (own && x >= 0) stage1_face<0>(B, x, L, qm, G, work, LE, idx, fl);
  raise_flags(flags, fl);
}

// O4 + O5 + O7 along d (y or z) in one kernel: each wavefront traces an
// 8 x 8 patch of the x-d plane (8 consecutive x slots, 8 slots along d, the
// first of them the previous patch's last: a halo, traced, not stored), so
// the two states of every d face it solves sit 8 lanes apart and the low
// side arrives by a lane shuffle.  A workgroup is 4 patches side by side in
// x at one slot of the third axis; its index w within the box (Tile.start)
// runs over x first, then the bands of 7 slots along d, then that third
// axis.  Same arithmetic as trace_at and stage1_face, so the same bits as
// the staged trace and riemann1 kernels along d.
template <int d, class S>
__global__ void __launch_bounds__(XF_THREADS) k_front_yz(const Tile* __restrict__ tiles, int ntiles,
                                                     const DevBox* __restrict__ boxes, const S* __restrict__ prim,
                                                     long long LS, S* __restrict__ work, long long LE, Gas<S> G,
                                                     const StepConsts* __restrict__ sc, int* flags) {
  constexpr int o = 3 - d;  // the third axis
  const int t = xcd_tile(ntiles);
  if (t < 0) return;  // the whole workgroup
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  const int E[3] = {B.n[0] + 2, B.n[1] + 2, B.n[2] + 2};
  const int nq = (E[0] + 31) / 32, nb = (E[d] + 6) / 7;
  const int w = tl.start;
  const int q = w % nq, band = (w / nq) % nb, so = w / (nq * nb);
  const int lane = threadIdx.x & 63, i = lane & 7, j = lane >> 3;
  const int xs = 32 * q + 8 * (int)(threadIdx.x >> 6) + i;  // slots: zone = slot - 1
  const int ds = 7 * band + j - 1;
  const bool act = xs < E[0] && ds >= 0 && ds < E[d];
  const bool own = act && j >= 1;
  int X[3];
  X[0] = xs - 1;
  X[d] = ds - 1;
  X[o] = so - 1;
  const long long e = ((long long)(X[2] + 1) * E[1] + (X[1] + 1)) * E[0] + (X[0] + 1);
  S qp[5], qm[5];
  int fl = 0;
  if (act) {
    trace_at<d>(B, X[0], X[1], X[2], e, prim, LS, work, LE, G, sc, qp, qm, fl);
    if (own) store_traced<d>(work, LE, B, e, qp, qm);
  } else {
#pragma unroll
    for (int m = 0; m < 5; ++m) qp[m] = qm[m] = S(0);
  }
  S L[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) L[m] = __shfl_up(qp[m], 8, 64);
  if (own && X[d] >= 0) stage1_face<d>(B, X[d], L, qm, G, work, LE, e, fl);
  raise_flags(flags, fl);
}

// O4-O7 fused and streamed along z: a workgroup owns an x-y tile of
// ex x ey zones of the traced grid and walks it through a run of z planes.
// It has a group of lanes per axis (whole wavefronts; lane r of group d
// owns zone r of the tile along d) and one group tracing the zones just
// below the tile's low x and y edges.  Per plane each owner lane traces its
// zone along its axis (the traced states still go to the workspace: the
// later stages read them), the x and y lanes put the high-face state into
// LDS, and after a barrier each owner lane solves the stage-1 problem on its
// zone's low face: the x and y neighbours' states from LDS, the z
// neighbour's from the lane's own registers (the plane below; the run's
// first plane traces the plane below it once more).  This stage never reads
// the traced states back.  The arithmetic is trace_at and stage1_face, so
// the results are the staged trace and riemann1 kernels' bit for bit.
// mx, my: the largest tile extents of the list (LDS layout and lane groups).
template <int d, class S>
__device__ __forceinline__ void front_plane_trace(const DevBox& B, int x, int y, int z, long long e,
                                                  const S* __restrict__ prim, long long LS, S* __restrict__ work,
                                                  long long LE, const Gas<S>& G, const StepConsts* __restrict__ sc,
                                                  S qp[5], S qm[5], int& fl) {
  trace_at<d>(B, x, y, z, e, prim, LS, work, LE, G, sc, qp, qm, fl);
  store_traced<d>(work, LE, B, e, qp, qm);
}

template <class S>
__global__ void __launch_bounds__(FRONT_MAX_THREADS) k_front_stream(
    const Brick* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes, const S* __restrict__ prim,
    long long LS, S* __restrict__ work, long long LE, Gas<S> G, const StepConsts* __restrict__ sc, int mx, int my,
    int* flags) {
  extern __shared__ unsigned char smem_raw[];
  const int k = xcd_tile(ntiles);
  if (k < 0) return;  // the whole workgroup
  const Brick K = tiles[k];  // o: the tile's first zone (traced grid, from -1); e: extents
  const DevBox B = boxes[K.box];
  const int PXN = (mx + 1) * my, PYN = mx * (my + 1);
  S* Px = (S*)smem_raw;  // [m][j][i + 1], i in [-1, ex): high x-face states of row j
  S* Py = Px + 5 * PXN;  // [m][j + 1][i], j in [-1, ey): high y-face states of column i
  const int ex = K.e[0], ey = K.e[1], nown = ex * ey;
  const int E0 = B.n[0] + 2, E1 = B.n[1] + 2;
  const int A = front_group(mx, my);
  const int g = threadIdx.x / A, r = threadIdx.x - g * A;
  // group 0-2: owner of zone (i, j) along axis g; group 3: the x halo of
  // row j (zone i = -1) or the y halo of column i (zone j = -1)
  bool act = false;
  int i = 0, j = 0;
  if (g < 3) {
    act = r < nown;
    j = act ? r / ex : 0;
    i = act ? r - j * ex : 0;
  } else if (r < ey) {
    act = K.o[0] >= 0;
    j = r;
    i = -1;
  } else if (r < ey + ex) {
    act = K.o[1] >= 0;
    i = r - ey;
    j = -1;
  }
  const int x = K.o[0] + i, y = K.o[1] + j;
  const bool hx = g == 3 && i < 0;
  int fl = 0;
  S qz[5];  // z lanes: high z-face state of the zone below
  if (g == 2 && act && K.o[2] >= 0) {
    const int z = K.o[2] - 1;
    S qm[5];
    trace_at<2>(B, x, y, z, ((long long)(z + 1) * E1 + (y + 1)) * E0 + (x + 1), prim, LS, work, LE, G, sc, qz, qm,
                fl);
  }
  for (int kz = 0; kz < K.e[2]; ++kz) {
    const int z = K.o[2] + kz;
    const long long e = ((long long)(z + 1) * E1 + (y + 1)) * E0 + (x + 1);
    S qp[5], qm[5];
    if (act) {
      if (g == 0 || hx) {
        trace_at<0>(B, x, y, z, e, prim, LS, work, LE, G, sc, qp, qm, fl);
        if (g == 0) store_traced<0>(work, LE, B, e, qp, qm);
#pragma unroll
        for (int m = 0; m < 5; ++m) Px[m * PXN + j * (mx + 1) + i + 1] = qp[m];
      } else if (g == 1 || g == 3) {
        trace_at<1>(B, x, y, z, e, prim, LS, work, LE, G, sc, qp, qm, fl);
        if (g == 1) store_traced<1>(work, LE, B, e, qp, qm);
#pragma unroll
        for (int m = 0; m < 5; ++m) Py[m * PYN + (j + 1) * mx + i] = qp[m];
      } else {
        front_plane_trace<2>(B, x, y, z, e, prim, LS, work, LE, G, sc, qp, qm, fl);
      }
    }
    __syncthreads();
    if (act && g < 3) {
      S L[5];
      if (g == 0) {
        if (x >= 0) {
#pragma unroll
          for (int m = 0; m < 5; ++m) L[m] = Px[m * PXN + j * (mx + 1) + i];
          stage1_face<0>(B, x, L, qm, G, work, LE, e, fl);
        }
      } else if (g == 1) {
        if (y >= 0) {
#pragma unroll
          for (int m = 0; m < 5; ++m) L[m] = Py[m * PYN + j * mx + i];
          stage1_face<1>(B, y, L, qm, G, work, LE, e, fl);
        }
      } else {
        if (z >= 0) stage1_face<2>(B, z, qz, qm, G, work, LE, e, fl);
#pragma unroll
        for (int m = 0; m < 5; ++m) qz[m] = qp[m];
      }
    }
    __syncthreads();  // before the next plane's states overwrite the LDS
  }
  raise_flags(flags, fl);
}

// O8: for axis d = blockIdx.y, both pairs (d, t1) and (d, t2) in one lane:
// the traced states of axis d are loaded once, corrected by the stage-1
// flux difference along t1 (dt/3h_t1) and along t2 (dt/3h_t2), and the
// fluxes F^{d|t} computed at d-face slots x_d in [0, n] with x_t in
// [0, n-1] and the remaining axis in [-1, n] (each pair under its own mask).
template <int d, int t, class S>
__device__ __forceinline__ void riemann2_pair(const S* __restrict__ w, S* __restrict__ o, long long LE,
                                              long long sd, long long stt, const S qeL[5], const S qeR[5],
                                              const Gas<S>& G, S c3, const DevBox& B, int xd, int& fl) {
  constexpr int pr = pair_index(d, t);
  S ueL[5], ueR[5], L[5], R[5];
  prim_to_cons(qeL, G, ueL);
  prim_to_cons(qeR, G, ueR);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* fL = w + (E_F1 + t * 5 + m) * LE - sd;
    const S* fR = w + (E_F1 + t * 5 + m) * LE;
    ueL[m] = ueL[m] - c3 * (fL[stt] - fL[0]);
    ueR[m] = ueR[m] - c3 * (fR[stt] - fR[0]);
  }
  cons_to_prim_floor(ueL, G, L, fl);
  cons_to_prim_floor(ueR, G, R, fl);
  wall_states<d>(B, xd, L, R);
  S F[5];
  riemann<d>(L, R, G, F, fl);
#pragma unroll
  for (int m = 0; m < 5; ++m) __builtin_nontemporal_store(F[m], &o[(E_F2 + pr * 5 + m) * LE]);
}

template <int d, class S>
__device__ __forceinline__ void riemann2_body(int tt, const Tile* __restrict__ tiles,
                                              const DevBox* __restrict__ boxes, S* __restrict__ work,
                                              long long LE, const Gas<S>& G,
                                              const StepConsts* __restrict__ sc, int* flags) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0) return;
  const bool va = z.x[t1] >= 0 && z.x[t1] < B.n[t1];  // pair (d, t1)
  const bool vb = z.x[t2] >= 0 && z.x[t2] < B.n[t2];  // pair (d, t2)
  if (!va && !vb) return;
  const long long sd = stride(z.E, d);
  const S* w = work + B.eoff + z.e;
  S* o = work + B.eoff + z.e;
  S qeL[5], qeR[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    qeL[m] = w[(E_TRACE + (d * 2 + 0) * 5 + m) * LE - sd];
    qeR[m] = w[(E_TRACE + (d * 2 + 1) * 5 + m) * LE];
  }
  int fl = 0;
  if (va) riemann2_pair<d, t1>(w, o, LE, sd, stride(z.E, t1), qeL, qeR, G, SC<S>::dt3h(sc)[t1], B, z.x[d], fl);
  if (vb) riemann2_pair<d, t2>(w, o, LE, sd, stride(z.E, t2), qeL, qeR, G, SC<S>::dt3h(sc)[t2], B, z.x[d], fl);
  raise_flags(flags, fl);
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) __attribute__((amdgpu_waves_per_eu(5))) k_riemann2(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   S* __restrict__ work, long long LE, Gas<S> G,
                                                   const StepConsts* __restrict__ sc, int* flags) {
  switch (blockIdx.y) {
    case 0: riemann2_body<0>(xcd_tile(ntiles), tiles, boxes, work, LE, G, sc, flags); break;
    case 1: riemann2_body<1>(xcd_tile(ntiles), tiles, boxes, work, LE, G, sc, flags); break;
    default: riemann2_body<2>(xcd_tile(ntiles), tiles, boxes, work, LE, G, sc, flags); break;
  }
}

// O9: states of axis d corrected by F^{t1|t2} and F^{t2|t1} (dt/2h), then
// the final flux at the d-face slot x (x_d in [0, n], transverse valid).
template <int d, class S>
__device__ __forceinline__ void riemann3_face(const DevBox& B, const int x[3], const S* __restrict__ work,
                                              long long LE, const Gas<S>& G, const StepConsts* __restrict__ sc,
                                              S F[5], int& fl) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const int E[3] = {B.n[0] + 2, B.n[1] + 2, B.n[2] + 2};
  const long long e = ((long long)(x[2] + 1) * E[1] + (x[1] + 1)) * E[0] + (x[0] + 1);
  const long long sd = stride(E, d), s1 = stride(E, t1), s2 = stride(E, t2);
  const S c1 = SC<S>::dt2h(sc)[t1], c2 = SC<S>::dt2h(sc)[t2];
  constexpr int p12 = pair_index(t1, t2), p21 = pair_index(t2, t1);
  const S* w = work + B.eoff + e;
  S L[5], R[5];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const long long off = side == 0 ? -sd : 0;
    S qe[5], ue[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) qe[m] = w[(E_TRACE + (d * 2 + side) * 5 + m) * LE + off];
    prim_to_cons(qe, G, ue);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const S* fa = w + (E_F2 + p12 * 5 + m) * LE + off;
      const S* fb = w + (E_F2 + p21 * 5 + m) * LE + off;
      ue[m] = ue[m] - c1 * (fa[s1] - fa[0]) - c2 * (fb[s2] - fb[0]);
    }
    cons_to_prim_floor(ue, G, side == 0 ? L : R, fl);
  }
  wall_states<d>(B, x[d], L, R);
  riemann<d>(L, R, G, F, fl);
}

// Face-centred flux output of face slot x along d (FP64, extents n + e_d).
template <int d, class S>
__device__ __forceinline__ void write_flux(const DevBox& B, const int x[3], const S F[5], double* fo) {
  int fe[3] = {B.n[0], B.n[1], B.n[2]};
  fe[d] += 1;
  const long long FN = (long long)fe[0] * fe[1] * fe[2];
  const long long li = ((long long)x[2] * fe[1] + x[1]) * fe[0] + x[0];
  double* q = fo + B.foff[d] + li;
#pragma unroll
  for (int m = 0; m < 5; ++m) q[m * FN] = (double)F[m];
}

template <int d, class S>
__device__ __forceinline__ void riemann3_body(int tt, const Tile* __restrict__ tiles,
                                              const DevBox* __restrict__ boxes, S* __restrict__ work,
                                              long long LE, const Gas<S>& G,
                                              const StepConsts* __restrict__ sc, double* fx, double* fy,
                                              double* fz, int* flags) {
  if (tt < 0) return;
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0 || z.x[t1] < 0 || z.x[t1] >= B.n[t1] || z.x[t2] < 0 || z.x[t2] >= B.n[t2]) return;
  int fl = 0;
  S F[5];
  riemann3_face<d>(B, z.x, work, LE, G, sc, F, fl);
  S* o = work + B.eoff + z.e;
#pragma unroll
  for (int m = 0; m < 5; ++m) o[(E_F3 + d * 5 + m) * LE] = F[m];
  double* fo = d == 0 ? fx : (d == 1 ? fy : fz);
  if (fo) write_flux<d>(B, z.x, F, fo);
  raise_flags(flags, fl);
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_riemann3(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   S* __restrict__ work, long long LE, Gas<S> G,
                                                   const StepConsts* __restrict__ sc,
                                                   double* fx, double* fy, double* fz, int* flags) {
  switch (blockIdx.y) {
    case 0: riemann3_body<0>(xcd_tile(ntiles), tiles, boxes, work, LE, G, sc, fx, fy, fz, flags); break;
    case 1: riemann3_body<1>(xcd_tile(ntiles), tiles, boxes, work, LE, G, sc, fx, fy, fz, flags); break;
    default: riemann3_body<2>(xcd_tile(ntiles), tiles, boxes, work, LE, G, sc, fx, fy, fz, flags); break;
  }
}

// O10 for one zone: U' = U - ((dt/h_x dFx + dt/h_y dFy) + dt/h_z dFz), then
// the Heun constant-gravity source.
__device__ __forceinline__ void update_zone(const double uo[5], const double fxd[5], const double fyd[5],
                                            const double fzd[5], double dtdx0, double dtdx1, double dtdx2,
                                            const StepConsts* __restrict__ sc, int grav, double g0, double g1,
                                            double g2, double un[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) un[m] = uo[m] - ((dtdx0 * fxd[m] + dtdx1 * fyd[m]) + dtdx2 * fzd[m]);
  if (grav) {
    const double adt = sc->dt, hdt = sc->hdt;
    double s0[5], s1[5];
    s0[1] = uo[0] * g0;
    s0[2] = uo[0] * g1;
    s0[3] = uo[0] * g2;
    s0[4] = (uo[1] * g0 + uo[2] * g1) + uo[3] * g2;
#pragma unroll
    for (int m = 1; m < 5; ++m) un[m] = un[m] + adt * s0[m];
    s1[1] = un[0] * g0;
    s1[2] = un[0] * g1;
    s1[3] = un[0] * g2;
    s1[4] = (un[1] * g0 + un[2] * g1) + un[3] * g2;
#pragma unroll
    for (int m = 1; m < 5; ++m) un[m] = un[m] + hdt * (s1[m] - s0[m]);
  }
}

// O10: conservative update in FP64 (+ Heun source) on the valid zones.
// Fold of one valid zone's signal speeds (|u_d| + c) / h_d into the running
// maximum s, from its conserved state (rho, rho u, rho v, rho w, rho E).
// A NaN speed (a non-physical zone) never replaces s.  The dt kernel and the
// update's fused form both use it, so their maxima agree bit for bit.
__device__ __forceinline__ double fold_signal_speed(double s, double r, double mx, double my, double mz,
                                                    double E, double h0, double h1, double h2, double gamma,
                                                    double gm1, double small_pres) {
  const double vx = mx / r, vy = my / r, vz = mz / r;
  const double ke = 0.5 * r * ((vx * vx + vy * vy) + vz * vz);
  double p = gm1 * (E - ke);
  p = smax(p, small_pres);
  const double c = __builtin_sqrt(gamma * p / r);
  const double sx = (sabs(vx) + c) / h0;
  const double sy = (sabs(vy) + c) / h1;
  const double sz = (sabs(vz) + c) / h2;
  return smax(smax(smax(s, sx), sy), sz);
}

// Maximum of s over the workgroup, max-accumulated into *bits (the bits of
// a non-negative double order like the doubles).  One atomic per
// workgroup, skipped when the running maximum is already as large.  Every
// lane of the workgroup must call it.
__device__ __forceinline__ void block_max_to(double s, unsigned long long* bits) {
  for (int off = 32; off > 0; off >>= 1) s = smax(s, __shfl_xor(s, off, 64));
  __shared__ double wmax[MAX_TILE / 64];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) m = smax(m, wmax[w]);
    const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
    if (mb > __hip_atomic_load(bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(bits, mb);
  }
}

// The update of one valid zone; returns its signal speed folded into 0 when
// so.bits is set (else 0).
template <class S>
__device__ __forceinline__ double update_body(const Tile& tl, const DevBox& B, const EZone& z,
                                              const double* __restrict__ U, double* __restrict__ Unew,
                                              const S* __restrict__ work, long long LE,
                                              const StepConsts* __restrict__ sc, int grav, double g0, double g1,
                                              double g2, const SpeedOut& so) {
  const long long sy = z.E[0], sz = (long long)z.E[0] * z.E[1];
  const double dtdx0 = sc->dtdx[0], dtdx1 = sc->dtdx[1], dtdx2 = sc->dtdx[2];
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
  const long long NS = (long long)N0 * N1 * N2;
  const long long ui = B.soff + ((long long)(z.x[2] + NG) * N1 + (z.x[1] + NG)) * N0 + (z.x[0] + NG);
  const S* w = work + B.eoff + z.e;
  double fxd[5], fyd[5], fzd[5], uo[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S* f0 = w + (E_F3 + 0 * 5 + m) * LE;
    const S* f1 = w + (E_F3 + 1 * 5 + m) * LE;
    const S* f2 = w + (E_F3 + 2 * 5 + m) * LE;
    fxd[m] = (double)f0[1] - (double)f0[0];
    fyd[m] = (double)f1[sy] - (double)f1[0];
    fzd[m] = (double)f2[sz] - (double)f2[0];
    uo[m] = U[ui + m * NS];
  }
  double un[5];
  update_zone(uo, fxd, fyd, fzd, dtdx0, dtdx1, dtdx2, sc, grav, g0, g1, g2, un);
#pragma unroll
  for (int m = 0; m < 5; ++m) Unew[ui + m * NS] = un[m];
  if (!so.bits) return 0.0;
  return fold_signal_speed(0.0, un[0], un[1], un[2], un[3], un[4], so.h[0], so.h[1], so.h[2], so.gamma, so.gm1,
                           so.small_pres);
}

// The update of the valid zones of tile tt; returns the lane's signal speed
// (0 without so.bits or off the valid zones).
template <class S>
__device__ __forceinline__ double update_tile(int tt, const Tile* __restrict__ tiles,
                                              const DevBox* __restrict__ boxes, const double* __restrict__ U,
                                              double* __restrict__ Unew, const S* __restrict__ work, long long LE,
                                              const StepConsts* __restrict__ sc, int grav, double g0, double g1,
                                              double g2, const SpeedOut& so) {
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  const bool valid = ezone(tl, B, z) && z.x[0] >= 0 && z.x[0] < B.n[0] && z.x[1] >= 0 && z.x[1] < B.n[1] &&
                     z.x[2] >= 0 && z.x[2] < B.n[2];
  return valid ? update_body(tl, B, z, U, Unew, work, LE, sc, grav, g0, g1, g2, so) : 0.0;
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_update(const Tile* __restrict__ tiles, int ntiles,
                                                 const DevBox* __restrict__ boxes,
                                                 const double* __restrict__ U, double* __restrict__ Unew,
                                                 const S* __restrict__ work, long long LE,
                                                 const StepConsts* __restrict__ sc, int grav,
                                                 double g0, double g1, double g2, SpeedOut so) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;  // the whole workgroup
  const double smax_lane = update_tile(tt, tiles, boxes, U, Unew, work, LE, sc, grav, g0, g1, g2, so);
  if (so.bits) block_max_to(smax_lane, so.bits);
}


// O9 + O10 fused on a brick of valid zones: the final fluxes of every face
// of the brick (its boundary faces are computed by both bricks that share
// them) go to LDS instead of HBM, then each zone of the brick is updated
// from them and, with so.bits, its signal speed folded into the next dt's
// maximum.  The arithmetic is riemann3_face, update_zone and
// fold_signal_speed, so the results are those of the staged kernels bit for
// bit.
template <int d, class S>
__device__ __forceinline__ void brick_faces(const Brick& K, const DevBox& B, const S* __restrict__ work,
                                            long long LE, const Gas<S>& G, const StepConsts* __restrict__ sc,
                                            S* __restrict__ Fs, double* fo, int& fl) {
  int ex[3] = {K.e[0], K.e[1], K.e[2]};
  ex[d] += 1;
  const int nf = ex[0] * ex[1] * ex[2];
  for (int f = threadIdx.x; f < nf; f += BRICK_THREADS) {
    const unsigned r = div31((unsigned)f, K.d0[d == 0]), k = div31(r, K.d1[d == 1]);
    const int x[3] = {K.o[0] + f - (int)r * ex[0], K.o[1] + (int)(r - k * (unsigned)ex[1]), K.o[2] + (int)k};
    S F[5];
    riemann3_face<d>(B, x, work, LE, G, sc, F, fl);
#pragma unroll
    for (int m = 0; m < 5; ++m) Fs[m * BRICK_FACES + f] = F[m];
    if (fo) write_flux<d>(B, x, F, fo);
  }
}

template <class S>
__global__ void __launch_bounds__(BRICK_THREADS) k_final_update(const Brick* __restrict__ bricks, int nbricks,
                                                            const DevBox* __restrict__ boxes,
                                                            const S* __restrict__ work, long long LE, Gas<S> G,
                                                            const StepConsts* __restrict__ sc,
                                                            const double* __restrict__ U, double* __restrict__ Unew,
                                                            double* fx, double* fy, double* fz, int grav, double g0,
                                                            double g1, double g2, SpeedOut so, int* flags) {
  __shared__ S Fs[3 * 5 * BRICK_FACES];
  const int k = xcd_tile(nbricks);
  if (k < 0) return;
  const Brick K = bricks[k];
  const DevBox B = boxes[K.box];
  int fl = 0;
  brick_faces<0>(K, B, work, LE, G, sc, Fs, fx, fl);
  brick_faces<1>(K, B, work, LE, G, sc, Fs + 5 * BRICK_FACES, fy, fl);
  brick_faces<2>(K, B, work, LE, G, sc, Fs + 10 * BRICK_FACES, fz, fl);
  raise_flags(flags, fl);
  __syncthreads();
  const int e0 = K.e[0], e1 = K.e[1], e2 = K.e[2];
  const double dtdx0 = sc->dtdx[0], dtdx1 = sc->dtdx[1], dtdx2 = sc->dtdx[2];
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
  const long long NS = (long long)N0 * N1 * N2;
  double smax_lane = 0.0;
  for (int z = threadIdx.x; z < e0 * e1 * e2; z += BRICK_THREADS) {
    const unsigned r = div31((unsigned)z, K.d0[0]), k = div31(r, K.d1[0]);
    const int l0 = z - (int)r * e0, l1 = (int)(r - k * (unsigned)e1), l2 = (int)k;
    const int ix = (l2 * e1 + l1) * (e0 + 1) + l0;        // x-face below the zone
    const int iy = (l2 * (e1 + 1) + l1) * e0 + l0;        // y-face below
    const int iz = (l2 * e1 + l1) * e0 + l0;              // z-face below
    const long long ui = B.soff + ((long long)(K.o[2] + l2 + NG) * N1 + (K.o[1] + l1 + NG)) * N0 +
                         (K.o[0] + l0 + NG);
    double fxd[5], fyd[5], fzd[5], uo[5], un[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const S* F0 = Fs + m * BRICK_FACES;
      const S* F1 = Fs + (5 + m) * BRICK_FACES;
      const S* F2 = Fs + (10 + m) * BRICK_FACES;
      fxd[m] = (double)F0[ix + 1] - (double)F0[ix];
      fyd[m] = (double)F1[iy + e0] - (double)F1[iy];
      fzd[m] = (double)F2[iz + e0 * e1] - (double)F2[iz];
      uo[m] = U[ui + m * NS];
    }
    update_zone(uo, fxd, fyd, fzd, dtdx0, dtdx1, dtdx2, sc, grav, g0, g1, g2, un);
#pragma unroll
    for (int m = 0; m < 5; ++m) Unew[ui + m * NS] = un[m];
    if (so.bits)
      smax_lane = smax(smax_lane, fold_signal_speed(0.0, un[0], un[1], un[2], un[3], un[4], so.h[0], so.h[1],
                                                    so.h[2], so.gamma, so.gm1, so.small_pres));
  }
  if (so.bits) block_max_to(smax_lane, so.bits);
}

// O9 + O10 fused, streamed along z: a workgroup owns an x-y tile of
// ex x ey valid zones and walks it through a run of z planes.  Per plane the
// stage-3 problems of the tile's faces are work items dealt round-robin to
// the workgroup's lanes, x faces first, then y faces, then the zones' high
// z faces (so a wave seldom mixes axes): (ex + 1) ey + ex (ey + 1) + ex ey
// solves, the x and y fluxes into LDS, the z fluxes into one of two LDS
// planes, the low z flux of a zone being the high one of the plane below
// (the run's first plane solves its low faces once more).  Every face is
// solved once, except the faces shared by neighbouring tiles and runs, and
// the final fluxes never go to HBM.  Then the plane's zones are updated.
// The arithmetic is riemann3_face and update_zone, so the results are the
// staged kernels' bit for bit.
template <class S>
__device__ __forceinline__ void stream_face(int f, const Brick& K, const DevBox& B, const S* __restrict__ work,
                                            long long LE, const Gas<S>& G, const StepConsts* __restrict__ sc,
                                            int z, int sx, int sy, S* Fx, S* Fy, S* Fz, double* fx, double* fy,
                                            double* fz, int& fl) {
  const int ex = K.e[0], ey = K.e[1];
  const int nfx = (ex + 1) * ey, nfy = ex * (ey + 1);
  const int FXN = (sx + 1) * sy, FYN = sx * (sy + 1), FZN = sx * sy;
  S F[5];
  if (f < nfx) {  // x face i of row j (i in [0, ex])
    const int j = f / (ex + 1), i = f - j * (ex + 1);
    const int x[3] = {K.o[0] + i, K.o[1] + j, z};
    riemann3_face<0>(B, x, work, LE, G, sc, F, fl);
#pragma unroll
    for (int m = 0; m < 5; ++m) Fx[m * FXN + j * (sx + 1) + i] = F[m];
    if (fx) write_flux<0>(B, x, F, fx);
  } else if ((f -= nfx) < nfy) {  // y face j of column i (j in [0, ey])
    const int j = f / ex, i = f - j * ex;
    const int x[3] = {K.o[0] + i, K.o[1] + j, z};
    riemann3_face<1>(B, x, work, LE, G, sc, F, fl);
#pragma unroll
    for (int m = 0; m < 5; ++m) Fy[m * FYN + j * sx + i] = F[m];
    if (fy) write_flux<1>(B, x, F, fy);
  } else {  // z face z of zone (i, j)
    f -= nfy;
    const int j = f / ex, i = f - j * ex;
    const int x[3] = {K.o[0] + i, K.o[1] + j, z};
    riemann3_face<2>(B, x, work, LE, G, sc, F, fl);
#pragma unroll
    for (int m = 0; m < 5; ++m) Fz[m * FZN + j * sx + i] = F[m];
    if (fz) write_flux<2>(B, x, F, fz);
  }
}

template <class S>
__global__ void __launch_bounds__(STREAM_MAX_THREADS) k_final_stream(
    const Brick* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes, const S* __restrict__ work,
    long long LE, Gas<S> G, const StepConsts* __restrict__ sc, const double* __restrict__ U,
    double* __restrict__ Unew, double* fx, double* fy, double* fz, int grav, double g0, double g1, double g2,
    int sx, int sy, SpeedOut so, int* flags) {
  extern __shared__ unsigned char smem_raw[];
  const int k = xcd_tile(ntiles);
  if (k < 0) return;  // the whole workgroup
  const Brick K = tiles[k];
  const DevBox B = boxes[K.box];
  const int FXN = (sx + 1) * sy, FYN = sx * (sy + 1), FZN = sx * sy;
  S* Fx = (S*)smem_raw;  // [m][j][i], i in [0, sx]: x faces of row j
  S* Fy = Fx + 5 * FXN;  // [m][j][i], j in [0, sy]: y faces of column i
  S* Fz0 = Fy + 5 * FYN;  // two planes [m][j][i] of z faces
  S* Fz1 = Fz0 + 5 * FZN;
  const int t = threadIdx.x, nt = blockDim.x;
  const int ex = K.e[0], ey = K.e[1];
  const int nfx = (ex + 1) * ey, nfy = ex * (ey + 1), nz = ex * ey;
  const double dtdx0 = sc->dtdx[0], dtdx1 = sc->dtdx[1], dtdx2 = sc->dtdx[2];
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
  const long long NS = (long long)N0 * N1 * N2;
  int fl = 0;
  double smax_lane = 0.0;
  // the run's first low z faces (the box's own low face is written once, here);
  // the work-item loops are not unrolled: one face solve is live at a time
#pragma nounroll
  for (int f = t; f < nz; f += nt)
    stream_face<S>(nfx + nfy + f, K, B, work, LE, G, sc, K.o[2], sx, sy, Fx, Fy, Fz0,
                   nullptr, nullptr, K.o[2] == 0 ? fz : nullptr, fl);
  S* Flo = Fz0;
  S* Fhi = Fz1;
  for (int kz = 0; kz < K.e[2]; ++kz) {
    const int z = K.o[2] + kz;
#pragma nounroll
    for (int f = t; f < nfx + nfy; f += nt)
      stream_face<S>(f, K, B, work, LE, G, sc, z, sx, sy, Fx, Fy, Fhi, fx, fy, fz, fl);
#pragma nounroll
    for (int f = t; f < nz; f += nt)  // high z faces: slot z + 1
      stream_face<S>(nfx + nfy + f, K, B, work, LE, G, sc, z + 1, sx, sy, Fx, Fy, Fhi, fx, fy, fz, fl);
    __syncthreads();
#pragma nounroll
    for (int q = t; q < nz; q += nt) {
      const int j = q / ex, i = q - j * ex;
      const int x0 = K.o[0] + i, y0 = K.o[1] + j;
      double fxd[5], fyd[5], fzd[5], uo[5], un[5];
      const long long ui = B.soff + ((long long)(z + NG) * N1 + (y0 + NG)) * N0 + (x0 + NG);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        fxd[m] = (double)Fx[m * FXN + j * (sx + 1) + i + 1] - (double)Fx[m * FXN + j * (sx + 1) + i];
        fyd[m] = (double)Fy[m * FYN + (j + 1) * sx + i] - (double)Fy[m * FYN + j * sx + i];
        fzd[m] = (double)Fhi[m * FZN + j * sx + i] - (double)Flo[m * FZN + j * sx + i];
        uo[m] = U[ui + m * NS];
      }
      update_zone(uo, fxd, fyd, fzd, dtdx0, dtdx1, dtdx2, sc, grav, g0, g1, g2, un);
#pragma unroll
      for (int m = 0; m < 5; ++m) Unew[ui + m * NS] = un[m];
      if (so.bits)
        smax_lane = smax(smax_lane, fold_signal_speed(0.0, un[0], un[1], un[2], un[3], un[4], so.h[0], so.h[1],
                                                      so.h[2], so.gamma, so.gm1, so.small_pres));
    }
    S* tmp = Flo;
    Flo = Fhi;
    Fhi = tmp;
    __syncthreads();  // before the next plane's faces overwrite the LDS
  }
  raise_flags(flags, fl);
  if (so.bits) block_max_to(smax_lane, so.bits);
}

// O11: max over valid zones and axes of (|u_d| + c)/h_d, FP64.  A fixed grid
// strides over the tiles; each lane keeps a running max, the workgroup
// reduces it with wave64 shuffles and LDS, and one atomic max per workgroup
// (on the bit pattern: non-negative doubles order like their unsigned bit
// patterns) combines the workgroups.  max is exact, so the result does not
// depend on the order.
__global__ void __launch_bounds__(MAX_TILE) k_wavespeed(const Tile* __restrict__ tiles, int ntiles,
                                                    const DevBox* __restrict__ boxes,
                                                    const double* __restrict__ U, double h0, double h1,
                                                    double h2, double gamma, double gm1,
                                                    double small_pres,
                                                    unsigned long long* __restrict__ smax_bits) {
  double s = 0.0;
  for (int tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
    const Tile tl = tiles[tt];
    const DevBox B = boxes[tl.box];
    EZone z;
    if (ezone(tl, B, z) && z.x[0] >= 0 && z.x[0] < B.n[0] && z.x[1] >= 0 && z.x[1] < B.n[1] &&
        z.x[2] >= 0 && z.x[2] < B.n[2]) {
      const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
      const long long NS = (long long)N0 * N1 * N2;
      const double* u = U + B.soff + ((long long)(z.x[2] + NG) * N1 + (z.x[1] + NG)) * N0 + (z.x[0] + NG);
      s = fold_signal_speed(s, u[0], u[NS], u[2 * NS], u[3 * NS], u[4 * NS], h0, h1, h2, gamma, gm1, small_pres);
    }
  }
  block_max_to(s, smax_bits);
}

__global__ void __launch_bounds__(64) k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0) p[0] = 0ull;
}

__global__ void __launch_bounds__(64) k_finish_dt(double* dt_dev, double cfl) {
  if (threadIdx.x == 0) {
    const double s = __longlong_as_double((long long)(((unsigned long long*)dt_dev)[1]));
    dt_dev[1] = s;
    dt_dev[0] = cfl / s;
  }
}

// O1: ghost fill over the plan.  One lane per destination ghost zone.  A
// lane's descriptor is the last one whose zone-count prefix does not exceed
// the lane's zone: one binary search per wavefront for its first zone (in
// scalar registers, so the dependent loads go through the scalar cache),
// then each lane steps forward over the few descriptors the wavefront's 64
// zones span.  Zone offsets within a descriptor (a slab of a ghost shell)
// stay below 2^31, so the region is decoded in 32 bits.
__global__ void __launch_bounds__(FILL_THREADS) k_fill(const FillDesc* __restrict__ desc,
                                               const long long* __restrict__ start, int d0, int d1,
                                               long long z0, long long z1,
                                               const DevBox* __restrict__ boxes, double* U, InflowView inf) {
  const long long gidx = z0 + (long long)blockIdx.x * FILL_THREADS + threadIdx.x;
  if (gidx >= z1) return;  // lane 0 of a wavefront has its smallest zone
  const long long gw =
      z0 + (long long)blockIdx.x * FILL_THREADS + __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
  int lo = d0, hi = d1 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= gw) lo = mid; else hi = mid - 1;
  }
  while (lo + 1 < d1 && start[lo + 1] <= gidx) ++lo;
  const FillDesc D = desc[lo];
  const unsigned l = (unsigned)(gidx - start[lo]);
  const unsigned ex = (unsigned)(D.hi[0] - D.lo[0] + 1), ey = (unsigned)(D.hi[1] - D.lo[1] + 1);
  const unsigned q = l / ex, r = q / ey;
  const int x = D.lo[0] + (int)(l - q * ex);
  const int y = D.lo[1] + (int)(q - r * ey);
  const int zz = D.lo[2] + (int)r;
  const int sx = D.a[0] * x + D.c[0], sy = D.a[1] * y + D.c[1], sz = D.a[2] * zz + D.c[2];
  const DevBox Bd = boxes[D.dst];
  const int dN0 = Bd.n[0] + 2 * NG, dN1 = Bd.n[1] + 2 * NG, dN2 = Bd.n[2] + 2 * NG;
  const long long dNS = (long long)dN0 * dN1 * dN2;
  const long long di = Bd.soff + ((long long)(zz + NG) * dN1 + (y + NG)) * dN0 + (x + NG);
  const double* src;
  long long si, sNS;
  if (D.src < 0) {  // prescribed state of an inflow face
    const int f = -1 - D.src, d = f >> 1;
    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int s3[3] = {sx, sy, sz};
    src = inf.p[f];
    sNS = (long long)inf.ext[t1] * inf.ext[t2];
    si = (long long)s3[t2] * inf.ext[t1] + s3[t1];
  } else {
    const DevBox Bs = boxes[D.src];
    const int sN0 = Bs.n[0] + 2 * NG, sN1 = Bs.n[1] + 2 * NG, sN2 = Bs.n[2] + 2 * NG;
    src = U;
    sNS = (long long)sN0 * sN1 * sN2;
    si = Bs.soff + ((long long)(sz + NG) * sN1 + (sy + NG)) * sN0 + (sx + NG);
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double v = src[si + c * sNS];
    const bool neg = c >= 1 && c <= 3 && ((D.sign >> (c - 1)) & 1);
    U[di + c * dNS] = neg ? -v : v;
  }
}


template <class S>
hipError_t step_impl(const DevLevel& L, int tS0, int tS1, int tE0, int tE1, int tB0, int tB1, int tF0, int tF1,
                     const FrontRanges& fr, const double* U,
                     double* Unew, double* const* flux, void* work, Gas<S> G, const double g[3], hipStream_t s,
                     hipEvent_t* ev, int upto, const SpeedOut& so) {
  S* prim = (S*)work;
  S* ework = prim + P_PLANES * L.LS;
  const int nS = tS1 - tS0, nE = tE1 - tE0;
  const Tile* TS = L.tilesS + tS0;
  const Tile* TE = L.tilesE + tE0;
  if (nS <= 0 || nE <= 0) return hipSuccess;
  const dim3 blk(L.tile);
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_prim<S>, dim3(xcd_grid(nS)), blk, 0, s, TS, nS, L.boxes, U, prim, L.LS, G, L.flags);
  if (ev) (void)hipEventRecord(ev[1], s);
  hipLaunchKernelGGL(k_flatten<S>, dim3(xcd_grid(nE)), blk, 0, s, TE, nE, L.boxes, prim, L.LS, ework, L.LE, G);
  if (ev) (void)hipEventRecord(ev[2], s);
  const int nF = tF1 - tF0;
  if (L.front == 1 && nF > 0) {
    // trace and stage-1 solves in one kernel (timed in the trace slot)
    const int mx = L.front_m[0], my = L.front_m[1];
    const size_t lds = sizeof(S) * 5 * (size_t)((mx + 1) * my + mx * (my + 1));
    hipLaunchKernelGGL(k_front_stream<S>, dim3(xcd_grid(nF)), dim3(front_threads(mx, my)), lds, s,
                       L.fbricks + tF0, nF, L.boxes, (const S*)prim, L.LS, ework, L.LE, G, L.consts, mx, my,
                       L.flags);
    if (ev) (void)hipEventRecord(ev[3], s);
    if (ev) (void)hipEventRecord(ev[4], s);
  } else {
    // front forms 2 and 3: the x axis, or every axis, in one kernel each
    // (timed in the trace slot); the other axes staged
    const int nX = fr.x1 - fr.x0, nY = fr.y1 - fr.y0, nZ = fr.z1 - fr.z0;
    const int d0 = (L.front >= 2 && nX > 0) ? 1 : 0;
    if (d0)
      hipLaunchKernelGGL(k_front_x<S>, dim3(xcd_grid(nX)), dim3(XF_THREADS), 0, s, L.tilesX + fr.x0, nX, L.boxes,
                         (const S*)prim, L.LS, ework, L.LE, G, L.consts, L.flags);
    if (L.front == 3 && d0 && nY > 0 && nZ > 0) {
      hipLaunchKernelGGL((k_front_yz<1, S>), dim3(xcd_grid(nY)), dim3(XF_THREADS), 0, s, L.tilesY + fr.y0, nY,
                         L.boxes, (const S*)prim, L.LS, ework, L.LE, G, L.consts, L.flags);
      hipLaunchKernelGGL((k_front_yz<2, S>), dim3(xcd_grid(nZ)), dim3(XF_THREADS), 0, s, L.tilesZ + fr.z0, nZ,
                         L.boxes, (const S*)prim, L.LS, ework, L.LE, G, L.consts, L.flags);
      if (ev) (void)hipEventRecord(ev[3], s);
    } else {
      hipLaunchKernelGGL(k_trace<S>, dim3(xcd_grid(nE), 3 - d0), blk, 0, s, TE, nE, L.boxes, prim, L.LS, ework,
                         L.LE, G, L.consts, L.flags, d0);
      if (ev) (void)hipEventRecord(ev[3], s);
      hipLaunchKernelGGL(k_riemann1<S>, dim3(xcd_grid(nE), 3 - d0), blk, 0, s, TE, nE, L.boxes, ework, L.LE, G,
                         L.flags, d0);
    }
    if (ev) (void)hipEventRecord(ev[4], s);
  }
  hipLaunchKernelGGL(k_riemann2<S>, dim3(xcd_grid(nE), 3), blk, 0, s, TE, nE, L.boxes, ework, L.LE, G,
                     L.consts, L.flags);
  if (upto <= STEP_TO_STAGE2) return hipGetLastError();
  double* fx = flux ? flux[0] : nullptr;
  double* fy = flux ? flux[1] : nullptr;
  double* fz = flux ? flux[2] : nullptr;
  if (ev) (void)hipEventRecord(ev[5], s);
  const int nB = tB1 - tB0;
  if (L.fused == 2 && upto == STEP_FULL && nB > 0) {
    const int sx = L.stream_e[0], sy = L.stream_e[1];
    const size_t lds = sizeof(S) * 5 * (size_t)((sx + 1) * sy + sx * (sy + 1) + 2 * sx * sy);
    hipLaunchKernelGGL(k_final_stream<S>, dim3(xcd_grid(nB)), dim3(stream_threads(sx, sy)), lds, s, L.bricks + tB0,
                       nB, L.boxes,
                       (const S*)ework, L.LE, G, L.consts, U, Unew, fx, fy, fz, G.grav, g[0], g[1], g[2], sx, sy,
                       so, L.flags);
    if (ev) (void)hipEventRecord(ev[6], s);
    if (ev) (void)hipEventRecord(ev[7], s);
    return hipGetLastError();
  }
  if (L.fused == 1 && upto == STEP_FULL && nB > 0) {
    hipLaunchKernelGGL(k_final_update<S>, dim3(xcd_grid(nB)), dim3(BRICK_THREADS), 0, s, L.bricks + tB0, nB,
                       L.boxes, (const S*)ework, L.LE, G, L.consts, U, Unew, fx, fy, fz, G.grav, g[0], g[1], g[2],
                       so, L.flags);
    if (ev) (void)hipEventRecord(ev[6], s);
    if (ev) (void)hipEventRecord(ev[7], s);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_riemann3<S>, dim3(xcd_grid(nE), 3), blk, 0, s, TE, nE, L.boxes, ework, L.LE, G,
                     L.consts, fx, fy, fz, L.flags);
  if (ev) (void)hipEventRecord(ev[6], s);
  hipLaunchKernelGGL(k_update<S>, dim3(xcd_grid(nE)), blk, 0, s, TE, nE, L.boxes, U, Unew,
                     (const S*)ework, L.LE, L.consts, G.grav, g[0], g[1], g[2], so);
  if (ev) (void)hipEventRecord(ev[7], s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step_consts(const DevLevel& L, double dt, const double* dt_dev, const double h[3],
                              const double g[3], hipStream_t s) {
  hipLaunchKernelGGL(k_step_consts, dim3(1), dim3(64), 0, s, L.consts, dt, dt_dev, h[0], h[1], h[2], g[0],
                     g[1], g[2]);
  return hipGetLastError();
}

hipError_t launch_fill(const DevLevel& L, double* U, int desc_begin, int desc_end, long long zone_begin,
                       long long zone_end, hipStream_t s) {
  if (desc_end <= desc_begin || zone_end <= zone_begin) return hipSuccess;
  const long long nz = zone_end - zone_begin;
  const unsigned grid = (unsigned)((nz + FILL_THREADS - 1) / FILL_THREADS);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(FILL_THREADS), 0, s, L.desc, L.desc_start, desc_begin, desc_end,
                     zone_begin, zone_end, L.boxes, U, L.inflow);
  return hipGetLastError();
}

hipError_t launch_compute_dt(const DevLevel& L, int tile_begin, int tile_end, const double* U,
                             const double h[3], double gamma, double small_pres, double cfl,
                             double* dt_dev, hipStream_t s) {
  unsigned long long* bits = (unsigned long long*)(dt_dev + 1);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, bits);
  const int n = tile_end - tile_begin;
  if (n > 0)
    hipLaunchKernelGGL(k_wavespeed, dim3(n < 2048 ? n : 2048), dim3(L.tile), 0, s, L.tilesE + tile_begin, n, L.boxes, U,
                       h[0], h[1], h[2], gamma, gamma - 1.0, small_pres, bits);
  hipLaunchKernelGGL(k_finish_dt, dim3(1), dim3(64), 0, s, dt_dev, cfl);
  return hipGetLastError();
}

hipError_t launch_step(const DevLevel& L, int precision, int tS0, int tS1, int tE0, int tE1, int tB0, int tB1,
                       int tF0, int tF1, const FrontRanges& fr, const double* U, double* Unew, double* const* flux,
                       void* work,
                       const double gamma, const double small_dens, const double small_pres, int limiter,
                       int flattening, int iters, int grav, const double g[3], hipStream_t s, hipEvent_t* ev,
                       int upto, SpeedOut so) {
  if (precision == 1)
    return step_impl<float>(L, tS0, tS1, tE0, tE1, tB0, tB1, tF0, tF1, fr, U, Unew, flux, work,
                            make_gas<float>(gamma, small_dens, small_pres, limiter, flattening, iters, grav),
                            g, s, ev, upto, so);
  return step_impl<double>(L, tS0, tS1, tE0, tE1, tB0, tB1, tF0, tF1, fr, U, Unew, flux, work,
                           make_gas<double>(gamma, small_dens, small_pres, limiter, flattening, iters, grav),
                           g, s, ev, upto, so);
}

hipError_t launch_speed_clear(unsigned long long* bits, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, bits);
  return hipGetLastError();
}

hipError_t launch_speed_finish(double* dt_dev, double cfl, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_dt, dim3(1), dim3(64), 0, s, dt_dev, cfl);
  return hipGetLastError();
}

}  // namespace ppm

// gfx950 kernels of the passive-species part of the step.
//
// A species is a mass fraction X = (rho X)/rho advected with the flow.  It
// rides on the hydro step: the stages below run right after the step's own
// stages and read what those left in the step workspace (primitive density,
// velocities and sound speed, flattening, traced densities, and the mass
// fluxes of the three corner-transport-upwind stages):
//   sp_frac    X = (rho X)/rho on every stored zone
//   sp_trace   PPM parabola of X (the step's limiter and flattening), traced
//              across the entropy wave only, like a transverse velocity
//   sp_flux1   normal-predictor species fluxes  F_rho X_upwind
//   sp_flux2   single-transverse corrected fractions, fluxes of the 6 pairs
//   sp_flux3   double-transverse corrected fractions, final species fluxes
//   sp_update  conservative update of rho X in FP64
// The upwind fraction is the one on the side the mass comes from: the left
// state's when the face's mass flux is positive, otherwise the right one's
// (a zero flux carries nothing either way, which also keeps every wall face
// closed: the wall's mirror states make its mass flux exactly zero).
// The corrected fraction is (rho X)/rho of the conserved pair corrected by
// the transverse flux differences, with the density floored as in the step.
//
// All species of a zone are handled by one lane, so each hydro quantity is
// loaded once per zone.  Species planes: ns planes of X on the stored grid,
// then, on the traced grid, 6 ns traced fractions, 3 ns stage-1, 6 ns
// stage-2 and 3 ns final species fluxes (plane q of species s: q * ns + s).
// Formulas are evaluated in the order of their definition (no contraction),
// so FP64 results agree with a serial evaluation bit for bit.
#include <hip/hip_runtime.h>

#include "ppm_device.h"
#include "ppm_internal.h"
#include "ppm_math.h"

namespace ppm {
namespace {

// Plane groups of the traced-grid species planes: group g holds one plane
// per species, plane (g * ns + s).
constexpr int SP_TRACE = 0;   // g = d*2 + side, side 0 = high face, 1 = low face
constexpr int SP_G1 = 6;      // g = 6 + d
constexpr int SP_G2 = 9;      // g = 9 + pair
constexpr int SP_G3 = 15;     // g = 15 + d
constexpr int SP_EPLANES = 18;

template <class S> __device__ __forceinline__ S carried(S frho, S xl, S xr) {
  return frho > S(0) ? frho * xl : frho * xr;
}

// X = (rho X)/rho on every stored zone; rho is the step's primitive density.
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_sp_frac(const Tile* __restrict__ tiles, int ntiles,
                                                  const DevBox* __restrict__ boxes,
                                                  const double* __restrict__ RX, const S* __restrict__ prim,
                                                  long long LS, int ns, S* __restrict__ X) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  const long long idx = (long long)tl.start + threadIdx.x;
  if (idx >= tl.end) return;
  const long long NS = (long long)(B.n[0] + 2 * NG) * (B.n[1] + 2 * NG) * (B.n[2] + 2 * NG);
  const S r = prim[B.poff + idx];
  const double* rx = RX + ns * B.poff + idx;
  S* x = X + B.poff + idx;
  for (int s = 0; s < ns; ++s) x[s * LS] = (S)rx[s * NS] / r;
}

template <int d, class S>
__device__ __forceinline__ void sp_trace_body(const Tile* __restrict__ tiles, int ntiles,
                                              const DevBox* __restrict__ boxes, const S* __restrict__ prim,
                                              long long LS, const S* __restrict__ work, long long LE,
                                              const S* __restrict__ X, S* __restrict__ sw, int ns,
                                              const Gas<S>& G, const StepConsts* __restrict__ sc) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  const int NS[3] = {B.n[0] + 2 * NG, B.n[1] + 2 * NG, B.n[2] + 2 * NG};
  const long long base = pidx(B, z.x[0], z.x[1], z.x[2]);
  const long long st = stride(NS, d);
  const S phi = work[E_FLAT * LE + B.eoff + z.e];
  const S un = prim[(1 + d) * LS + base], c = sound_speed(prim[base], prim[4 * LS + base], G);
  const S dtdx = SC<S>::dtdx(sc)[d];
  const S zero = S(0);
  const S l1 = un - c, l2 = un, l3 = un + c;
  const S sp3 = smax(l3, zero) * dtdx, sp2 = smax(l2, zero) * dtdx;
  const S sm1 = smax(-l1, zero) * dtdx, sm2 = smax(-l2, zero) * dtdx;
  S* o = sw + B.eoff + z.e;
  for (int s = 0; s < ns; ++s) {
    const S* a = X + s * LS + base;
    S aL, aR, a6;
    ppm_parabola(a[-2 * st], a[-st], a[0], a[st], a[2 * st], phi, G, aL, aR, a6);
    const S da = aR - aL;
    S xp, xm;
    {
      const S ref = ppm_ip(aR, da, a6, sp3);
      const S at = (l2 > zero) ? ref - ppm_ip(aR, da, a6, sp2) : zero;
      xp = ref - at;
    }
    {
      const S ref = ppm_im(aL, da, a6, sm1);
      const S at = (l2 < zero) ? ref - ppm_im(aL, da, a6, sm2) : zero;
      xm = ref - at;
    }
    o[((SP_TRACE + d * 2 + 0) * ns + s) * LE] = xp;
    o[((SP_TRACE + d * 2 + 1) * ns + s) * LE] = xm;
  }
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_sp_trace(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   const S* __restrict__ prim, long long LS,
                                                   const S* __restrict__ work, long long LE,
                                                   const S* __restrict__ X, S* __restrict__ sw, int ns,
                                                   Gas<S> G, const StepConsts* __restrict__ sc) {
  switch (blockIdx.y) {
    case 0: sp_trace_body<0>(tiles, ntiles, boxes, prim, LS, work, LE, X, sw, ns, G, sc); break;
    case 1: sp_trace_body<1>(tiles, ntiles, boxes, prim, LS, work, LE, X, sw, ns, G, sc); break;
    default: sp_trace_body<2>(tiles, ntiles, boxes, prim, LS, work, LE, X, sw, ns, G, sc); break;
  }
}

// Stage 1 at the d-face slots of the step's stage 1: x_d in [0, n],
// transverse in [-1, n].
template <int d, class S>
__device__ __forceinline__ void sp_flux1_body(const Tile* __restrict__ tiles, int ntiles,
                                              const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                              long long LE, S* __restrict__ sw, int ns) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0) return;
  const long long sd = stride(z.E, d);
  const S frho = work[(E_F1 + d * 5) * LE + B.eoff + z.e];
  S* w = sw + B.eoff + z.e;
  for (int s = 0; s < ns; ++s) {
    const S xl = w[((SP_TRACE + d * 2 + 0) * ns + s) * LE - sd];
    const S xr = w[((SP_TRACE + d * 2 + 1) * ns + s) * LE];
    w[((SP_G1 + d) * ns + s) * LE] = carried(frho, xl, xr);
  }
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_sp_flux1(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   const S* __restrict__ work, long long LE,
                                                   S* __restrict__ sw, int ns) {
  switch (blockIdx.y) {
    case 0: sp_flux1_body<0>(tiles, ntiles, boxes, work, LE, sw, ns); break;
    case 1: sp_flux1_body<1>(tiles, ntiles, boxes, work, LE, sw, ns); break;
    default: sp_flux1_body<2>(tiles, ntiles, boxes, work, LE, sw, ns); break;
  }
}

// Stage 2, pair (d, t): the traced fractions of axis d corrected along t
// (dt/3h_t) on both sides of the face, then the species fluxes of the pair.
template <int d, int t, class S>
__device__ __forceinline__ void sp_flux2_pair(const S* __restrict__ work, S* __restrict__ w, long long LE,
                                              long long sd, long long stt, int ns, S c3, S small_dens) {
  constexpr int pr = pair_index(d, t);
  const S* fL = work + (E_F1 + t * 5) * LE - sd;
  const S* fR = work + (E_F1 + t * 5) * LE;
  const S rtL = work[(E_TRACE + (d * 2 + 0) * 5) * LE - sd];
  const S rtR = work[(E_TRACE + (d * 2 + 1) * 5) * LE];
  const S rhoL = smax(rtL - c3 * (fL[stt] - fL[0]), small_dens);
  const S rhoR = smax(rtR - c3 * (fR[stt] - fR[0]), small_dens);
  const S frho = work[(E_F2 + pr * 5) * LE];
  for (int s = 0; s < ns; ++s) {
    const S* gL = w + ((SP_G1 + t) * ns + s) * LE - sd;
    const S* gR = w + ((SP_G1 + t) * ns + s) * LE;
    const S xtL = w[((SP_TRACE + d * 2 + 0) * ns + s) * LE - sd];
    const S xtR = w[((SP_TRACE + d * 2 + 1) * ns + s) * LE];
    const S xl = (rtL * xtL - c3 * (gL[stt] - gL[0])) / rhoL;
    const S xr = (rtR * xtR - c3 * (gR[stt] - gR[0])) / rhoR;
    w[((SP_G2 + pr) * ns + s) * LE] = carried(frho, xl, xr);
  }
}

// Both pairs (d, t1), (d, t2) of axis d in one lane, each under the step's
// own mask: x_d in [0, n], x_t in [0, n-1], the remaining axis in [-1, n].
template <int d, class S>
__device__ __forceinline__ void sp_flux2_body(const Tile* __restrict__ tiles, int ntiles,
                                              const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                              long long LE, S* __restrict__ sw, int ns, const Gas<S>& G,
                                              const StepConsts* __restrict__ sc) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0) return;
  const bool va = z.x[t1] >= 0 && z.x[t1] < B.n[t1];
  const bool vb = z.x[t2] >= 0 && z.x[t2] < B.n[t2];
  const long long sd = stride(z.E, d);
  const S* wk = work + B.eoff + z.e;
  S* w = sw + B.eoff + z.e;
  if (va) sp_flux2_pair<d, t1>(wk, w, LE, sd, stride(z.E, t1), ns, SC<S>::dt3h(sc)[t1], G.small_dens);
  if (vb) sp_flux2_pair<d, t2>(wk, w, LE, sd, stride(z.E, t2), ns, SC<S>::dt3h(sc)[t2], G.small_dens);
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_sp_flux2(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   const S* __restrict__ work, long long LE,
                                                   S* __restrict__ sw, int ns, Gas<S> G,
                                                   const StepConsts* __restrict__ sc) {
  switch (blockIdx.y) {
    case 0: sp_flux2_body<0>(tiles, ntiles, boxes, work, LE, sw, ns, G, sc); break;
    case 1: sp_flux2_body<1>(tiles, ntiles, boxes, work, LE, sw, ns, G, sc); break;
    default: sp_flux2_body<2>(tiles, ntiles, boxes, work, LE, sw, ns, G, sc); break;
  }
}

// Stage 3: fractions of axis d corrected by the pair fluxes (t1|t2) and
// (t2|t1) (dt/2h), then the final species fluxes at x_d in [0, n] with the
// transverse indices valid.
template <int d, class S>
__device__ __forceinline__ void sp_flux3_body(const Tile* __restrict__ tiles, int ntiles,
                                              const DevBox* __restrict__ boxes, const S* __restrict__ work,
                                              long long LE, S* __restrict__ sw, int ns, const Gas<S>& G,
                                              const StepConsts* __restrict__ sc) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  constexpr int p12 = pair_index(t1, t2), p21 = pair_index(t2, t1);
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[d] < 0 || z.x[t1] < 0 || z.x[t1] >= B.n[t1] || z.x[t2] < 0 || z.x[t2] >= B.n[t2]) return;
  const long long sd = stride(z.E, d), s1 = stride(z.E, t1), s2 = stride(z.E, t2);
  const S c1 = SC<S>::dt2h(sc)[t1], c2 = SC<S>::dt2h(sc)[t2];
  const S* wk = work + B.eoff + z.e;
  S* w = sw + B.eoff + z.e;
  S rt[2], rho[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const long long off = side == 0 ? -sd : 0;
    const S* fa = wk + (E_F2 + p12 * 5) * LE + off;
    const S* fb = wk + (E_F2 + p21 * 5) * LE + off;
    rt[side] = wk[(E_TRACE + (d * 2 + side) * 5) * LE + off];
    rho[side] = smax(rt[side] - c1 * (fa[s1] - fa[0]) - c2 * (fb[s2] - fb[0]), G.small_dens);
  }
  const S frho = wk[(E_F3 + d * 5) * LE];
  for (int s = 0; s < ns; ++s) {
    S x[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const long long off = side == 0 ? -sd : 0;
      const S* ga = w + ((SP_G2 + p12) * ns + s) * LE + off;
      const S* gb = w + ((SP_G2 + p21) * ns + s) * LE + off;
      const S xt = w[((SP_TRACE + d * 2 + side) * ns + s) * LE + off];
      x[side] = (rt[side] * xt - c1 * (ga[s1] - ga[0]) - c2 * (gb[s2] - gb[0])) / rho[side];
    }
    w[((SP_G3 + d) * ns + s) * LE] = carried(frho, x[0], x[1]);
  }
}

template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_sp_flux3(const Tile* __restrict__ tiles, int ntiles,
                                                   const DevBox* __restrict__ boxes,
                                                   const S* __restrict__ work, long long LE,
                                                   S* __restrict__ sw, int ns, Gas<S> G,
                                                   const StepConsts* __restrict__ sc) {
  switch (blockIdx.y) {
    case 0: sp_flux3_body<0>(tiles, ntiles, boxes, work, LE, sw, ns, G, sc); break;
    case 1: sp_flux3_body<1>(tiles, ntiles, boxes, work, LE, sw, ns, G, sc); break;
    default: sp_flux3_body<2>(tiles, ntiles, boxes, work, LE, sw, ns, G, sc); break;
  }
}

// rho X update in FP64 on the valid zones, x + y + z in that order.
template <class S>
__global__ void __launch_bounds__(MAX_TILE) k_sp_update(const Tile* __restrict__ tiles, int ntiles,
                                                    const DevBox* __restrict__ boxes,
                                                    const double* __restrict__ RX, double* __restrict__ RXnew,
                                                    const S* __restrict__ sw, long long LE, int ns,
                                                    const StepConsts* __restrict__ sc) {
  const int tt = xcd_tile(ntiles);
  if (tt < 0) return;
  const Tile tl = tiles[tt];
  const DevBox B = boxes[tl.box];
  EZone z;
  if (!ezone(tl, B, z)) return;
  if (z.x[0] < 0 || z.x[0] >= B.n[0] || z.x[1] < 0 || z.x[1] >= B.n[1] || z.x[2] < 0 ||
      z.x[2] >= B.n[2])
    return;
  const long long sy = z.E[0], sz = (long long)z.E[0] * z.E[1];
  const double dtdx0 = sc->dtdx[0], dtdx1 = sc->dtdx[1], dtdx2 = sc->dtdx[2];
  const int N0 = B.n[0] + 2 * NG, N1 = B.n[1] + 2 * NG, N2 = B.n[2] + 2 * NG;
  const long long NS = (long long)N0 * N1 * N2;
  const long long ui = ns * B.poff + ((long long)(z.x[2] + NG) * N1 + (z.x[1] + NG)) * N0 + (z.x[0] + NG);
  const S* w = sw + B.eoff + z.e;
  for (int s = 0; s < ns; ++s) {
    const S* g0 = w + ((SP_G3 + 0) * ns + s) * LE;
    const S* g1 = w + ((SP_G3 + 1) * ns + s) * LE;
    const S* g2 = w + ((SP_G3 + 2) * ns + s) * LE;
    const double gx = (double)g0[1] - (double)g0[0];
    const double gy = (double)g1[sy] - (double)g1[0];
    const double gz = (double)g2[sz] - (double)g2[0];
    RXnew[ui + s * NS] = RX[ui + s * NS] - ((dtdx0 * gx + dtdx1 * gy) + dtdx2 * gz);
  }
}

// Ghost fill of an ns-component scalar arena through the state's fill plan:
// the same copies, no sign changes.
__global__ void __launch_bounds__(FILL_THREADS) k_fill_scalars(const FillDesc* __restrict__ desc,
                                                           const long long* __restrict__ start, int d0, int d1,
                                                           long long z0, long long z1,
                                                           const DevBox* __restrict__ boxes, double* RX, int ns) {
  const long long gidx = z0 + (long long)blockIdx.x * FILL_THREADS + threadIdx.x;
  if (gidx >= z1) return;
  int lo = d0, hi = d1 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= gidx) lo = mid; else hi = mid - 1;
  }
  const FillDesc D = desc[lo];
  if (D.src < 0) return;  // inflow faces carry no species (rejected on the host)
  const long long l = gidx - start[lo];
  const int ex = D.hi[0] - D.lo[0] + 1, ey = D.hi[1] - D.lo[1] + 1;
  const int x = D.lo[0] + (int)(l % ex);
  const int y = D.lo[1] + (int)((l / ex) % ey);
  const int zz = D.lo[2] + (int)(l / ((long long)ex * ey));
  const int sx = D.a[0] * x + D.c[0], sy = D.a[1] * y + D.c[1], sz = D.a[2] * zz + D.c[2];
  const DevBox Bd = boxes[D.dst], Bs = boxes[D.src];
  const int dN0 = Bd.n[0] + 2 * NG, dN1 = Bd.n[1] + 2 * NG, dN2 = Bd.n[2] + 2 * NG;
  const int sN0 = Bs.n[0] + 2 * NG, sN1 = Bs.n[1] + 2 * NG, sN2 = Bs.n[2] + 2 * NG;
  const long long dNS = (long long)dN0 * dN1 * dN2, sNS = (long long)sN0 * sN1 * sN2;
  const long long di = ns * Bd.poff + ((long long)(zz + NG) * dN1 + (y + NG)) * dN0 + (x + NG);
  const long long si = ns * Bs.poff + ((long long)(sz + NG) * sN1 + (sy + NG)) * sN0 + (sx + NG);
  for (int c = 0; c < ns; ++c) RX[di + c * dNS] = RX[si + c * sNS];
}

template <class S>
hipError_t species_impl(const DevLevel& L, int nS, int nE, const double* RX, double* RXnew, int ns,
                        const void* work, void* swork, Gas<S> G, hipStream_t s) {
  const S* prim = (const S*)work;
  const S* ework = prim + P_PLANES * L.LS;
  S* X = (S*)swork;
  S* sw = X + (long long)ns * L.LS;
  if (nS <= 0 || nE <= 0) return hipSuccess;
  const dim3 blk(L.tile);
  hipLaunchKernelGGL(k_sp_frac<S>, dim3(xcd_grid(nS)), blk, 0, s, L.tilesS, nS, L.boxes, RX, prim, L.LS, ns, X);
  hipLaunchKernelGGL(k_sp_trace<S>, dim3(xcd_grid(nE), 3), blk, 0, s, L.tilesE, nE, L.boxes, prim, L.LS, ework,
                     L.LE, (const S*)X, sw, ns, G, L.consts);
  hipLaunchKernelGGL(k_sp_flux1<S>, dim3(xcd_grid(nE), 3), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, sw, ns);
  hipLaunchKernelGGL(k_sp_flux2<S>, dim3(xcd_grid(nE), 3), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, sw, ns,
                     G, L.consts);
  hipLaunchKernelGGL(k_sp_flux3<S>, dim3(xcd_grid(nE), 3), blk, 0, s, L.tilesE, nE, L.boxes, ework, L.LE, sw, ns,
                     G, L.consts);
  hipLaunchKernelGGL(k_sp_update<S>, dim3(xcd_grid(nE)), blk, 0, s, L.tilesE, nE, L.boxes, RX, RXnew,
                     (const S*)sw, L.LE, ns, L.consts);
  return hipGetLastError();
}

}  // namespace

size_t species_workspace_bytes(long long LS, long long LE, int ns, int precision) {
  const size_t sz = precision == 1 ? sizeof(float) : sizeof(double);
  return sz * (size_t)ns * (size_t)(LS + SP_EPLANES * LE);
}

hipError_t launch_species(const DevLevel& L, int precision, int nS, int nE, const double* RX, double* RXnew,
                          int ns, const void* work, void* swork, double gamma, double small_dens,
                          double small_pres, int limiter, int flattening, int iters, int grav, hipStream_t s) {
  if (precision == 1)
    return species_impl<float>(L, nS, nE, RX, RXnew, ns, work, swork,
                               make_gas<float>(gamma, small_dens, small_pres, limiter, flattening, iters, grav), s);
  return species_impl<double>(L, nS, nE, RX, RXnew, ns, work, swork,
                              make_gas<double>(gamma, small_dens, small_pres, limiter, flattening, iters, grav), s);
}

hipError_t launch_fill_scalars(const DevLevel& L, double* RX, int ns, int desc_begin, int desc_end,
                               long long zone_begin, long long zone_end, hipStream_t s) {
  if (desc_end <= desc_begin || zone_end <= zone_begin) return hipSuccess;
  const long long nz = zone_end - zone_begin;
  const unsigned grid = (unsigned)((nz + FILL_THREADS - 1) / FILL_THREADS);
  hipLaunchKernelGGL(k_fill_scalars, dim3(grid), dim3(FILL_THREADS), 0, s, L.desc, L.desc_start, desc_begin,
                     desc_end, zone_begin, zone_end, L.boxes, RX, ns);
  return hipGetLastError();
}

}  // namespace ppm

// Device-side helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "ppm_internal.h"
#include "ppm_math.h"

namespace ppm {

template <class S> struct SC;
template <> struct SC<double> {
  __device__ static const double* dtdx(const StepConsts* c) { return c->d_dtdx; }
  __device__ static const double* dt2h(const StepConsts* c) { return c->d_dt2h; }
  __device__ static const double* dt3h(const StepConsts* c) { return c->d_dt3h; }
  __device__ static const double* hdtg(const StepConsts* c) { return c->d_hdtg; }
};
template <> struct SC<float> {
  __device__ static const float* dtdx(const StepConsts* c) { return c->f_dtdx; }
  __device__ static const float* dt2h(const StepConsts* c) { return c->f_dt2h; }
  __device__ static const float* dt3h(const StepConsts* c) { return c->f_dt3h; }
  __device__ static const float* hdtg(const StepConsts* c) { return c->f_hdtg; }
};

// Tile index of this workgroup.  Consecutive workgroups are dealt round-robin
// to the 8 XCDs; remapping gives each XCD a contiguous run of tiles so that
// the stencil neighbours of a tile sit in the same XCD's L2.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (ntiles + NXCD - 1) / NXCD;
  const int b = blockIdx.x;
  const int t = (b % NXCD) * per + b / NXCD;
  return (t < ntiles) ? t : -1;
}
__host__ inline int xcd_grid(int ntiles) { return ((ntiles + NXCD - 1) / NXCD) * NXCD; }

__device__ __forceinline__ void raise_flags(int* flags, int fl) {
  if (fl) atomicOr(flags, fl);
}

// Zone geometry of a tile lane on the traced grid of a box: E = n + 2 per
// axis, slot s <-> zone s - 1.
struct EZone {
  int x[3];     // zone coordinates, -1..n
  int E[3];
  long long e;  // linear index in the box's traced grid
};

__device__ __forceinline__ bool ezone(const Tile& tl, const DevBox& B, EZone& z) {
  z.E[0] = B.n[0] + 2; z.E[1] = B.n[1] + 2; z.E[2] = B.n[2] + 2;
  const int idx = tl.start + (int)threadIdx.x;  // below 2^31: tile bounds are ints
  if (idx >= tl.end) return false;
  z.e = idx;
  const unsigned r = div31((unsigned)idx, B.de[0]), k = div31(r, B.de[1]);
  z.x[0] = idx - (int)r * z.E[0] - 1;
  z.x[1] = (int)(r - k * (unsigned)z.E[1]) - 1;
  z.x[2] = (int)k - 1;
  return true;
}

// Linear stride along axis d of a grid with extents E.
__device__ __forceinline__ long long stride(const int E[3], int d) {
  return d == 0 ? 1 : (d == 1 ? (long long)E[0] : (long long)E[0] * E[1]);
}

// Primitive-plane index of zone (x, y, z) of box B (stored grid).
__device__ __forceinline__ long long pidx(const DevBox& B, int x, int y, int z) {
  return B.poff + ((long long)(z + NG) * (B.n[1] + 2 * NG) + (y + NG)) * (B.n[0] + 2 * NG) + (x + NG);
}

// Gas and scheme constants in the reconstruction scalar, formed on the host
// in FP64 and rounded once to S.
template <class S>
inline Gas<S> make_gas(double gamma, double small_dens, double small_pres, int limiter, int flattening, int iters,
                int grav) {
  Gas<S> G;
  G.gamma = S(gamma);
  G.gm1 = S(gamma - 1.0);
  G.gm1inv = S(1.0 / (gamma - 1.0));
  G.beta = S((gamma + 1.0) / (2.0 * gamma));
  G.small_dens = S(small_dens);
  G.small_pres = S(small_pres);
  G.ismall_dens = S(1.0 / small_dens);
  G.limiter = limiter;
  G.flattening = flattening && limiter;
  G.iters = iters;
  G.grav = grav;
  return G;
}

// Riemann problem on a reflecting wall: the state outside the wall is the
// mirror image of the state inside it (normal velocity negated), so the solve
// gives u* = 0 and only the pressure acts on the wall.  xd: the face slot
// along d.  Returns which state was replaced: 1 the low side (the box's low
// face is on a wall), 2 the high side, 0 none.
template <int d, class S>
__device__ __forceinline__ int wall_states(const DevBox& B, int xd, S L[5], S R[5]) {
  if (((B.wall >> (2 * d)) & 3) == 0) return 0;  // uniform over the tile: most boxes skip here
  const bool lo = xd == 0 && ((B.wall >> (2 * d)) & 1);
  const bool hi = !lo && xd == B.n[d] && ((B.wall >> (2 * d + 1)) & 1);
  if (!lo && !hi) return 0;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S l = L[m], r = R[m];
    L[m] = lo ? ((m == 1 + d) ? -r : r) : l;
    R[m] = hi ? ((m == 1 + d) ? -l : l) : r;
  }
  return lo ? 1 : (hi ? 2 : 0);
}

// Reverse of wall_states: the replaced state's adjoint goes to the state it
// mirrors; the replaced state itself receives none.
template <int d, class S>
__device__ __forceinline__ void wall_states_vjp(int side, S Lb[5], S Rb[5]) {
  if (side == 0) return;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const S lb = Lb[m], rb = Rb[m];
    const S ml = (m == 1 + d) ? -lb : lb, mr = (m == 1 + d) ? -rb : rb;
    Lb[m] = side == 1 ? S(0) : (side == 2 ? lb + mr : lb);
    Rb[m] = side == 2 ? S(0) : (side == 1 ? rb + ml : rb);
  }
}

__host__ __device__ constexpr int pair_index(int d, int t) { return 2 * d + (t > d ? t - 1 : t); }

}  // namespace ppm

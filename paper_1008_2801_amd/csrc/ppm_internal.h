// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "ppm.h"
#include "ppm_math.h"

namespace ppm {

constexpr int NG = 4;        // ghost zones per side
constexpr int TILE = 256;    // default zones per tile (== threads per workgroup)
constexpr int MAX_TILE = 512;  // largest tile the kernels are built for
constexpr int NXCD = 8;      // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int FILL_THREADS = 256;  // threads per workgroup of the ghost-fill kernels

// Division by an invariant divisor D >= 2 of dividends below 2^31
// (Granlund and Montgomery, 1994): with l = ceil(log2 D) and
// m = ceil(2^(31+l) / D), which is below 2^32, floor(n / D) equals
// (n m) >> (31 + l) for every n < 2^31 — a high multiply and a shift on the
// device instead of a division sequence.
struct Div31 {
  unsigned m;
  int s;  // l - 1
};
inline Div31 make_div31(unsigned D) {
  int l = 0;
  while ((1ull << l) < D) ++l;
  return {(unsigned)(((1ull << (31 + l)) + D - 1) / D), l - 1};
}
#if defined(__HIPCC__)
__device__ __forceinline__ unsigned div31(unsigned n, Div31 q) { return __umulhi(n, q.m) >> q.s; }
#endif

// Per-box metadata on the device.
struct DevBox {
  int n[3];           // valid extents
  int wall;           // faces on a reflecting domain boundary: bit 2d low, bit 2d+1 high
  long long soff;     // element offset of the box in the state arena
  long long poff;     // offset in each plane of the primitive arena (stored grid, (n+8)^3)
  long long eoff;     // offset in each plane of the traced-grid arenas ((n+2)^3)
  long long foff[3];  // element offsets in the three flux arenas
  Div31 de[2];        // division by the traced grid's x and y extents, n + 2
  Div31 ds[2];        // division by the stored grid's x and y extents, n + 8
};

// A tile: TILE (or fewer, at the end of a box) consecutive linear zones
// [start, end) of one box's grid.
struct Tile {
  int box;
  int start;
  int end;
};

// A brick: valid zones [o, o + e) of one box (e_d <= BRICK_E[d]), the
// work unit of the fused final-flux-and-update kernel.  Long in x, so that
// the lanes of a wavefront read runs of consecutive zones.
constexpr int BRICK_E[3] = {32, 4, 4};
constexpr int BRICK_THREADS = 512;
// The streamed final stage: x-y tiles of sx x sy zones (a multiple of 32,
// at most 256); a workgroup of twice as many lanes (at most 512) works
// through the plane's 3 sx sy + sx + sy face solves.
constexpr int STREAM_MAX_THREADS = 512;
// streamed front end: a group of lanes per axis, one per zone of an x-y
// tile, and a group for the rows and columns of its low edges, each group
// in whole wavefronts
constexpr int FRONT_MAX_THREADS = 512;
// front form 2: workgroups of XF_THREADS lanes, each wavefront tracing 64
// consecutive traced zones of which the first is the previous wavefront's
// last (so every x face's two states meet in one wavefront)
constexpr int XF_THREADS = 256;
constexpr int XF_OWNED = XF_THREADS / 64 * 63;
// front form 3 along y and z: each wavefront an 8 x 8 patch (8 x slots, 8
// slots along the axis, the first a halo), a workgroup 4 patches side by
// side in x; workgroups per box: ceil(E0 / 32) x ceil(E_d / 7) x E_other
inline long long front_yz_groups(int E0, int Ed, int Eo) {
  return (long long)((E0 + 31) / 32) * ((Ed + 6) / 7) * Eo;
}
// ranges of the front forms' work lists of a launch
struct FrontRanges {
  int x0, x1, y0, y1, z0, z1;
};
__host__ __device__ inline int front_group(int mx, int my) {
  const int a = mx * my > mx + my ? mx * my : mx + my;
  return ((a + 63) / 64) * 64;
}
inline int front_threads(int mx, int my) { return 4 * front_group(mx, my); }
inline int stream_threads(int sx, int sy) { return 2 * sx * sy < STREAM_MAX_THREADS ? 2 * sx * sy : STREAM_MAX_THREADS; }
// faces of the largest axis of a full brick (LDS slots per axis and component)
constexpr int BRICK_FACES_D(int d) {
  return (BRICK_E[0] + (d == 0)) * (BRICK_E[1] + (d == 1)) * (BRICK_E[2] + (d == 2));
}
constexpr int BRICK_FACES = BRICK_FACES_D(0) > BRICK_FACES_D(1)
                                ? (BRICK_FACES_D(0) > BRICK_FACES_D(2) ? BRICK_FACES_D(0) : BRICK_FACES_D(2))
                                : (BRICK_FACES_D(1) > BRICK_FACES_D(2) ? BRICK_FACES_D(1) : BRICK_FACES_D(2));
struct Brick {
  int box;
  int o[3], e[3];
  Div31 d0[2], d1[2];  // division by e_x and e_x + 1, by e_y and e_y + 1
};
inline void brick_divisors(Brick& K) {
  for (int k = 0; k < 2; ++k) {
    K.d0[k] = make_div31((unsigned)(K.e[0] + k));
    K.d1[k] = make_div31((unsigned)(K.e[1] + k));
  }
}

// One copy of the ghost-fill plan: the dst-box-local region [lo, hi] takes
// its values from src-box-local zone a*x + c (per axis, a in {1, -1, 0}),
// negating the momentum components flagged in sign.  src < 0: the region
// lies beyond inflow face -1 - src and takes the face's prescribed state at
// domain-relative transverse index a*x + c (a = 0 along the face normal).
struct FillDesc {
  int dst, src;
  int lo[3], hi[3];
  int a[3], c[3];
  int sign;
  int count;
};

// Zone classes of the fill transpose: per axis, bit 0 = within NG of the low
// face, bit 1 = within NG of the high face; class = c0 + 4 c1 + 16 c2.
constexpr int INV_CLASSES = 64;
inline __host__ __device__ int inv_axis_class(int y, int n) { return (y < NG ? 1 : 0) | (y >= n - NG ? 2 : 0); }

// Per-step constants formed on the device from dt (so that a graph can take
// dt from device memory).  The reconstruction copies exist in FP64 and FP32.
struct StepConsts {
  double dt, hdt;
  double dtdx[3];
  double d_dtdx[3], d_dt2h[3], d_dt3h[3], d_hdtg[3];
  float f_dtdx[3], f_dt2h[3], f_dt3h[3], f_hdtg[3];
};

// Number of planes in the traced-grid (E) arena: flattening 1, traces 30,
// stage-1 fluxes 15, stage-2 fluxes 30, final fluxes 15.
constexpr int E_FLAT = 0;
constexpr int E_TRACE = 1;          // + (d*2 + side)*5 + m, side 0 = high face, 1 = low face
constexpr int E_F1 = E_TRACE + 30;  // + d*5 + m
constexpr int E_F2 = E_F1 + 15;     // + pair*5 + m, pair = 2*d + (t > d ? t-1 : t)
constexpr int E_F3 = E_F2 + 30;     // + d*5 + m
constexpr int E_PLANES = E_F3 + 15;
constexpr int P_PLANES = 5;         // rho, u, v, w, p

// Prescribed ghost states of inflow faces: p[face] (null if the face is not
// an inflow face) holds 5 conserved components over the domain's extents of
// the two other axes t1 < t2, order [c][t2][t1]; ext: the domain extents.
struct InflowView {
  const double* p[6];
  int ext[3];
};

// Launch-side views of the context's device data.
struct DevLevel {
  const DevBox* boxes;
  const Tile* tilesS;  // tiles over the stored grids
  const Tile* tilesE;  // tiles over the traced grids
  const Tile* tilesX;  // runs of XF_OWNED traced zones (front forms 2, 3)
  const Tile* tilesXA;  // runs of XF_OWNED - 1 traced zones (adjoint along x)
  const Tile* tilesY;  // workgroups of 8 x 8 patches in x-y planes (front form 3)
  const Tile* tilesZ;  // workgroups of 8 x 8 patches in x-z planes (front form 3)
  const FillDesc* desc;
  const long long* desc_start;  // exclusive prefix of zone counts, ndesc+1
  StepConsts* consts;
  int* flags;
  const int* inv_start;  // nbox * INV_CLASSES + 1: descriptors per (source box, zone class)
  const int* inv_idx;
  long long LS, LE;    // plane lengths (elements) of the primitive and traced arenas
  int tile;            // zones per tile of the tile lists (threads per workgroup)
  InflowView inflow;
  const Brick* bricks;  // valid-zone blocks of every box (fused final stage)
  int fused;            // 1: final fluxes and update in one brick kernel (fluxes kept in LDS);
                        // 2: the same in x-y tiles streamed along z (ppm_kernels.hip, k_final_stream)
  int stream_e[3];      // form 2: x, y extents of a tile (threads = product) and the z run
  const Brick* fbricks; // traced-grid x-y tiles with z runs (streamed front end)
  int front;            // 1: trace + stage-1 solves in one kernel streamed along z (k_front_stream);
                        // 2: the x axis's trace + stage-1 solves in one kernel (k_front_x);
                        // 3: every axis's (k_front_x, k_front_yz)
  int front_m[2];       // largest x, y extents of the front tiles (LDS layout, lanes)
};

}  // namespace ppm

// Kernel launchers (ppm_kernels.hip).  Each returns the hipError_t of the launch.
namespace ppm {
hipError_t launch_step_consts(const DevLevel& L, double dt, const double* dt_dev, const double h[3],
                              const double g[3], hipStream_t s);
hipError_t launch_fill(const DevLevel& L, double* U, int desc_begin, int desc_end, long long zone_begin,
                       long long zone_end, hipStream_t s);
hipError_t launch_compute_dt(const DevLevel& L, int tile_begin, int tile_end, const double* U,
                             const double h[3], double gamma, double small_pres, double cfl,
                             double* dt_dev, hipStream_t s);
// The step stages over E-tiles [tE0, tE1), S-tiles [tS0, tS1), bricks
// [tB0, tB1), front tiles [tF0, tF1) and the fused axes' lists fr.  upto: STEP_TO_STAGE2 (prim..riemann2, for the adjoint's
// recompute), STEP_FULL (the whole step; the fused final stage when the
// level asks for it), STEP_FULL_STAGED (the whole step with the final
// fluxes left in the workspace, as the species stages need).
enum { STEP_TO_STAGE2 = 5, STEP_FULL = 7, STEP_FULL_STAGED = 8 };
// Optional output of the staged update: the maximum over the updated valid
// zones of the signal speed max_d (|u_d| + c) / h_d, as the bits of a
// non-negative double, max-accumulated into *bits (null: not computed).
struct SpeedOut {
  unsigned long long* bits;
  double h[3];
  double gamma, gm1, small_pres;
};

hipError_t launch_step(const DevLevel& L, int precision, int tS0, int tS1, int tE0, int tE1, int tB0, int tB1,
                       int tF0, int tF1, const FrontRanges& fr,
                       const double* U, double* Unew, double* const* flux, void* work,
                       const double gamma, const double small_dens, const double small_pres,
                       int limiter, int flattening, int iters, int grav, const double g[3],
                       hipStream_t s, hipEvent_t* ev, int upto = STEP_FULL,
                       SpeedOut so = SpeedOut{nullptr, {0.0, 0.0, 0.0}, 0.0, 0.0, 0.0});
// The speed accumulator of a fused-dt step: cleared before the step's
// launches, turned into dt = cfl / s after them (one lane each).
hipError_t launch_speed_clear(unsigned long long* bits, hipStream_t s);
hipError_t launch_speed_finish(double* dt_dev, double cfl, hipStream_t s);
// Adjoint of one FP64 step (ppm_adjoint.hip); the forward workspace must hold
// the recomputed prim..riemann2 intermediates of the same step.
size_t adjoint_workspace_bytes(long long LS, long long LE, int precision);
// Adjoints of the three flux outputs (flux arenas, FP64; null: none).
struct FluxBar {
  const double* p[3];
};
hipError_t launch_adjoint(const DevLevel& L, int precision, int nS, int nE, int nX, int nXA, const double* U,
                          const double* Ubn,
                          FluxBar fb, double* Ub, const void* work, void* awork, double gamma, double small_dens,
                          double small_pres, int limiter, int flattening, int iters, int grav, const double g[3],
                          hipStream_t s);
// Passive species (ppm_species.hip), run after a full step whose
// intermediates are still in the step workspace `work`.
size_t species_workspace_bytes(long long LS, long long LE, int ns, int precision);
hipError_t launch_species(const DevLevel& L, int precision, int nS, int nE, const double* RX, double* RXnew,
                          int ns, const void* work, void* swork, double gamma, double small_dens,
                          double small_pres, int limiter, int flattening, int iters, int grav, hipStream_t s);
hipError_t launch_fill_scalars(const DevLevel& L, double* RX, int ns, int desc_begin, int desc_end,
                               long long zone_begin, long long zone_end, hipStream_t s);
// Events recorded by launch_step when ev is non-null: before each of the 7
// stage kernels and after the last (STEP_EVENTS in all).
constexpr int STEP_EVENTS = 8;
constexpr int PROF_FILL = PPM_PROF_FILL, PROF_DT = PPM_PROF_DT, PROF_PRIM = PPM_PROF_PRIM,
              PROF_NTAGS = PPM_PROF_NTAGS;
}  // namespace ppm

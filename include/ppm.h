/*
 * ppm.h -- C ABI of the MI355X (gfx950) unsplit PPM hydro step.
 *
 * The library advances the 3-D gamma-law Euler equations by one explicit
 * unsplit Godunov step on the rectangular boxes (FABs) of one refinement
 * level: the compressible code's explicit update of a system of hyperbolic
 * conservation laws (paper Sec. 1), on its MultiFAB / FAB data model with
 * ghost cells filled from intersecting grids, the intersections found by a
 * hash sort of the boxes and cached (Sec. 2).
 *
 * The discretisation (PPM with the Colella-Woodward limiter and flattening,
 * characteristic tracing, a two-shock Riemann solver with a fixed Newton
 * count, 12-solve corner-transport-upwind corrections, conservative update)
 * is the classical one the paper's code is built on; the paper itself only
 * names the advance.
 *
 * Conventions shared by every entry point:
 *  - All device pointers are HIP device memory owned by the caller.  The
 *    library owns only the context (box metadata, fill plan, tile lists,
 *    a few bytes of device constants and status flags).
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*, 0 = the null stream) and never synchronise, except
 *    ppm_check_status and the autotuner.
 *  - Every call returns PPM_OK or an error code; on error nothing was
 *    enqueued and ppm_last_error(ctx) describes it.
 *
 * State arena: one contiguous float64 buffer for the whole level.  Box b
 * (valid extents n = hi - lo + 1, stored extents N = n + 8) starts at
 * element off[b] (ppm_layout_offsets) and holds 5 components (rho, rho u,
 * rho v, rho w, rho E) in the order [c][k][j][i]: element
 *   off[b] + ((c*Nz + k+4)*Ny + j+4)*Nx + i+4
 * is zone (i, j, k) of box b, i in [-4, nx+3] (4 ghost zones per side).
 *
 * Flux arena of axis d: box b starts at element foff_d[b]
 * (ppm_flux_offsets) and holds 5 components over the face-centred extents
 * (n_d + 1 along d, n along the others), order [c][k][j][i]; face i along x
 * lies between zones i-1 and i.  Fluxes are per unit area per unit time,
 * time-centred (the F^{n+1/2} of the update).
 */
#ifndef PPM_H
#define PPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PPM_OK = 0,
  PPM_EINVAL = 1,    /* invalid argument; nothing enqueued */
  PPM_EHIP = 2,      /* HIP runtime error (string kept in ppm_last_error) */
  PPM_ENONPHYS = 3   /* status flags raised (ppm_check_status only) */
};

enum { PPM_BC_PERIODIC = 0, PPM_BC_OUTFLOW = 1, PPM_BC_REFLECT = 2,
       PPM_BC_COARSE_FINE = 3, /* the face borders a coarser level: ghost zones beyond it are left to
                                  the two-level interpolation (ppm_amr_fill_fine), not filled */
       PPM_BC_INFLOW = 4 /* ghost zones beyond the face take a prescribed state (ppm_set_inflow);
                            at most one inflow face per layout */ };

/* status flags accumulated on the device */
enum { PPM_FLAG_NONPHYS = 1, /* rho <= 0, p <= 0 or a non-finite value in an input state */
       PPM_FLAG_FLOOR = 2,   /* a density/pressure floor bound inside the step */
       PPM_FLAG_RANGE = 4 }; /* an input zone's density, pressure or sound speed lies outside
                                [2^-120, 2^120], or a velocity component beyond 2^120 in magnitude:
                                the FP64 divisions and square roots of the step drop the compiler's
                                range scaling and are correctly rounded only for the magnitudes
                                states within those bounds produce (the step is still computed) */

/* launch forms of the step */
enum { PPM_LAUNCH_BATCHED = 0, /* each stage: one launch over the tile list of all boxes */
       PPM_LAUNCH_PER_BOX = 1  /* each stage: one launch per box (the plain baseline) */ };

enum { PPM_MAX_SPECIES = 64 }; /* passive species per species arena */

typedef struct { int32_t lo[3], hi[3]; } ppm_box; /* inclusive valid zones, global index space */

typedef struct {
  int32_t nbox;
  const ppm_box* boxes;  /* disjoint, tiling `domain` exactly */
  ppm_box domain;
  int32_t bc[6];         /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi; periodic axes need both faces periodic */
  int32_t ngrow;         /* ghost width; must be 4 */
} ppm_layout;

typedef struct {
  double gamma;          /* > 1 */
  double cfl;            /* Courant number of the dt rule, in (0, 1) */
  double small_dens, small_pres; /* floors, in [2^-120, 2^120] */
  double grav[3];        /* constant gravity, Heun source; zeros: none */
  int32_t limiter;       /* 1: MC slopes + CW84 limiter; 0: unlimited (smooth) */
  int32_t flattening;    /* 1: CW84 shock flattening (needs limiter = 1) */
  int32_t riemann_iters; /* fixed Newton iterations of the two-shock solver, 0..16 */
  int32_t precision;     /* 0: FP64 throughout; 1: FP32 reconstruction, FP64 fluxes/update */
} ppm_params;

typedef struct ppm_ctx ppm_ctx;
typedef struct ppm_graph ppm_graph;

/* Context for one level layout (paper Sec. 2: replicated box metadata).
 * Validates the layout (disjoint non-empty boxes tiling the domain,
 * ngrow == 4, domain extents >= 4, periodic axes periodic on both faces,
 * fewer than 2^31 zones per box with its ghost layers; boxes may be
 * thinner than the ghost width), builds or reuses
 * the ghost-fill plan (hash-sorted intersections, cached across contexts)
 * and the tile lists, and uploads them.  Allocates device memory for them.
 * Returns PPM_EINVAL for an invalid layout, PPM_EHIP on allocation failure. */
int ppm_ctx_create(const ppm_layout* layout, ppm_ctx** out);
int ppm_ctx_destroy(ppm_ctx* ctx);
const char* ppm_last_error(const ppm_ctx* ctx);

/* off[0..nbox]: element offsets of each box in the state arena; off[nbox]
 * is the arena length.  Caller provides nbox+1 int64 slots. */
int ppm_layout_offsets(const ppm_ctx* ctx, int64_t* off);
/* The same for the flux arena of axis d (0..2). */
int ppm_flux_offsets(const ppm_ctx* ctx, int32_t d, int64_t* off);

/* Device scratch for the step, owned by the caller: bytes needed for the
 * given precision, then the buffer to use (kept until replaced; must stay
 * allocated while work that uses it is in flight).  The step returns
 * PPM_EINVAL if no large-enough workspace is set. */
size_t ppm_workspace_bytes(const ppm_ctx* ctx, int32_t precision);
int ppm_set_workspace(ppm_ctx* ctx, void* dev_ptr, size_t bytes);

/* O1 -- ghost fill (paper Sec. 2: filling ghost cells from intersecting
 * grids).  Writes the 4-deep ghost shells (faces, edges, corners) of every
 * box of U from the owning boxes of their images: periodic axes wrap,
 * outflow faces copy the nearest valid zone, reflecting faces mirror about
 * the wall with the normal momentum negated.  In place; valid zones are
 * read, ghost zones written.  mode: PPM_LAUNCH_BATCHED (one launch) or
 * PPM_LAUNCH_PER_BOX (one launch per destination box). */
int ppm_fill_boundary(ppm_ctx* ctx, double* U, int32_t mode, void* stream);

/* Prescribed state of an inflow face (the inflowing jet of the paper's
 * Sec. 4 enters through such a face): `state` is a device array of 5
 * conserved components over the domain's extents of the two axes t1 < t2
 * other than the face normal, order [c][t2][t1], owned by the caller and
 * read by every later fill.  A ghost zone beyond the face takes the state
 * at the image of its transverse coordinates under those axes' own rules
 * (periodic wrap, outflow clamp, reflecting mirror with the momentum sign).
 * ppm_fill_boundary returns PPM_EINVAL while an inflow face has no state;
 * species fills reject layouts with an inflow face.  PPM_EINVAL if `face`
 * is not an inflow face of the layout. */
int ppm_set_inflow(ppm_ctx* ctx, int32_t face, const double* state);

/* O11 -- CFL rule.  Writes to dt_dev[0] the time step
 *   dt = cfl / max over valid zones and axes of (|u_d| + c) / h_d
 * computed in FP64 from U (valid zones only; ghosts not read), and to
 * dt_dev[1] the maximum signal speed.  dt_dev: 2 device doubles. */
int ppm_compute_dt(ppm_ctx* ctx, const double* U, const double dx[3], const ppm_params* params,
                   double* dt_dev, void* stream);

/* O2-O10 -- one unsplit PPM step (the hot path).  Reads U (valid and ghost
 * zones; ghosts must be filled), writes the valid zones of Unew (ghosts of
 * Unew untouched).  dt: the time step, or, if dt_dev is non-null, read on
 * the device from dt_dev[0] (dt is then ignored).  flux: null, or three
 * flux-arena pointers (any may be null) that receive F^{n+1/2}.  U and Unew
 * must not overlap.  On a face in the plane of a reflecting domain
 * boundary every Riemann problem takes the mirror image of the state inside
 * the wall as the outside state (normal velocity negated): no mass or
 * energy crosses a wall.  Needs a workspace (ppm_set_workspace).  Raises
 * PPM_FLAG_* on the device (ppm_check_status).  PPM_EINVAL for null or
 * overlapping state pointers, invalid parameters, a non-positive dt
 * without dt_dev, or a missing/small workspace. */
int ppm_hydro_step(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                   const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                   void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of ppm_hydro_step, same arguments and results bit for bit, with the step
 * workspace taken from a library-owned device array of
 * PPM_NOALLOC_SCRATCH_BYTES instead of ppm_set_workspace.  The array is
 * static device memory of the library, one copy per GPU, held until the
 * process ends; its address on a device is looked up once, when the first
 * context is created with that device current.  The call allocates and
 * frees nothing (no hipMalloc, no event creation; profiling does not time
 * it).  The caller still owns U, Unew, the fluxes and dt_dev.  Every call on
 * a GPU uses that GPU's one array: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the
 * caller.  The step writes every scratch entry it reads, so nothing is
 * cleared between calls.  PPM_EINVAL for the errors of ppm_hydro_step and
 * when ppm_workspace_bytes(ctx, params->precision) exceeds
 * PPM_NOALLOC_SCRATCH_BYTES (a single box fits up to 53^3 zones in FP64,
 * 67^3 in the FP32-reconstruction mode); PPM_EHIP if the array's address
 * could not be found. */
enum { PPM_NOALLOC_SCRATCH_BYTES = 134217728 /* 128 MiB */ };
int ppm_hydro_step_noalloc(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                           const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                           void* stream);

/* ppm_hydro_step that also leaves the next step's time step: dt_next_dev
 * (2 device doubles) receives what ppm_compute_dt(Unew) would write, bit
 * for bit -- the CFL rule over the valid zones of Unew, which the update
 * (in every form of the final stage) computes from the states it writes
 * instead of a separate pass over Unew.  The
 * ghost fill before the next step does not change valid zones, so the next
 * step can read its dt from dt_next_dev.  dt_next_dev may alias dt_dev (it
 * is written after the step has read dt_dev[0]).  PPM_EINVAL as for
 * ppm_hydro_step, and for a null dt_next_dev or a cfl outside (0, 1). */
int ppm_hydro_step_dt(ppm_ctx* ctx, const double* U, double* Unew, double* const* flux, double dt,
                      const double* dt_dev, const double dx[3], const ppm_params* params, int32_t mode,
                      double* dt_next_dev, void* stream);

/* Adjoint of one step, dt and every branch decision of the forward step
 * frozen: given the step's input U (ghosts filled, as for ppm_hydro_step),
 * the adjoint Unew_bar of the new state's valid zones and optionally the
 * adjoints of the step's flux outputs, writes to U_bar the adjoint of U's
 * valid zones -- the transpose of the step's Jacobian (new state and
 * fluxes) applied to (Unew_bar, flux_bar), the ghost-fill transpose
 * included (ghost adjoints are added into the zones they were copied from)
 * -- and zeros U_bar's ghost zones.  flux_bar: null, or three flux-arena
 * pointers (ppm_flux_offsets layout, any may be null) holding the adjoints
 * of the F^{n+1/2} that ppm_hydro_step writes (the refluxing of a coarser
 * level consumes those fluxes, paper Sec. 2-3); a null entry adds
 * nothing.  The reverse stages run in the precision of the forward step they
 * differentiate (params->precision: 0 all FP64; 1 the reconstruction,
 * tracing and Riemann reverses in FP32, the update's reverse, the
 * conversion's output and U_bar in FP64).  The forward intermediates are
 * recomputed into the step workspace (ppm_set_workspace, sized for the same
 * precision); the reverse stages use a second caller-owned workspace of
 * ppm_adjoint_workspace_bytes(ctx, precision) bytes, 256-byte aligned.
 * U_bar must not overlap U, Unew_bar or a flux adjoint.  Deterministic:
 * no atomics.
 * Returns PPM_EINVAL (message in ppm_last_error) for a null pointer,
 * overlapping buffers, invalid parameters or a missing/small workspace. */
size_t ppm_adjoint_workspace_bytes(const ppm_ctx* ctx, int32_t precision);
int ppm_set_adjoint_workspace(ppm_ctx* ctx, void* dev_ptr, size_t bytes);
int ppm_hydro_step_adjoint(ppm_ctx* ctx, const double* U, const double* Unew_bar, const double* const* flux_bar,
                           double* U_bar, double dt, const double* dt_dev, const double dx[3],
                           const ppm_params* params, void* stream);

/* The same adjoint without the recompute: the step workspace must still
 * hold the intermediates of the forward step from this U with the same dt
 * and params (ppm_hydro_step ran with this workspace and nothing has
 * written to it since).  Results are bitwise those of
 * ppm_hydro_step_adjoint.  For callers that keep one workspace per step of
 * a checkpoint segment (memory for compute); the library cannot check the
 * precondition. */
int ppm_hydro_step_adjoint_saved(ppm_ctx* ctx, const double* U, const double* Unew_bar,
                                 const double* const* flux_bar, double* U_bar, double dt, const double* dt_dev,
                                 const double dx[3], const ppm_params* params, void* stream);

/* Passive species: mass fractions X_s carried with the flow (partial
 * densities rho X_s obey the continuity equation with the mass flux times
 * X_s).  The paper's code advances conserved variables generically (Sec. 1);
 * species are the usual passive-scalar extension of the same advance, not a
 * part the paper spells out.
 *
 * Species arena: one contiguous float64 buffer of ns components for the
 * level; box b starts at element soff[b] (ppm_species_offsets) and holds
 * ns planes rho X_s over the stored extents, order [s][k][j][i], like the
 * state arena (same ghost width, same zone order).  ns in
 * [1, PPM_MAX_SPECIES]. */
int ppm_species_offsets(const ppm_ctx* ctx, int32_t ns, int64_t* off);

/* Device scratch of the species stages (caller-owned, 256-byte aligned):
 * bytes for ns species in the given precision; 0 for invalid arguments. */
size_t ppm_species_workspace_bytes(const ppm_ctx* ctx, int32_t ns, int32_t precision);
int ppm_set_species_workspace(ppm_ctx* ctx, void* dev_ptr, size_t bytes);

/* Ghost fill of a species arena: the copies of ppm_fill_boundary (periodic
 * images, outflow copies, wall mirrors) with no sign change.  In place. */
int ppm_fill_species(ppm_ctx* ctx, double* RX, int32_t ns, int32_t mode, void* stream);

/* The hydro step (exactly ppm_hydro_step, batched launch form) followed by
 * the species update of the same step: each X = (rho X)/rho gets the
 * step's PPM parabola (same limiter and flattening), is traced across the
 * entropy wave only, and is carried through the three corner-transport
 * stages by that stage's mass flux from the side the mass comes from, with
 * the transverse corrections applied to rho X against the corrected
 * density; rho X is updated conservatively in FP64.  Species cross no
 * wall (the wall rule makes the mass flux there exactly zero).  RX:
 * species arena with ghosts filled (ppm_fill_species); RXnew receives the
 * new valid zones (ghosts untouched).  Needs the step workspace and a
 * species workspace for ns.  PPM_EINVAL, nothing enqueued, for the errors
 * of ppm_hydro_step and for a bad ns, null or overlapping species arenas,
 * RXnew overlapping a state arena, or a missing/small species workspace. */
int ppm_hydro_step_species(ppm_ctx* ctx, const double* U, double* Unew, const double* RX, double* RXnew,
                           int32_t ns, double* const* flux, double dt, const double* dt_dev, const double dx[3],
                           const ppm_params* params, void* stream);

/* Two-level hierarchy with subcycling in time, refinement ratio 2 (paper
 * Sec. 1: adaptive mesh refinement; Sec. 2: ghost cells from intersecting
 * grids and synchronisation of the levels; Sec. 3: a coarse time step is
 * one coarse and two fine steps; the multilevel runs refine the inner 12.5%
 * of the domain).  The formulas are the standard Berger-Colella ones:
 *  - dt: one coarse dt = cfl / max(S_c, S_f / 2) (S: the level's maximum of
 *    (|u_d| + c)/h_d over valid zones), two fine steps of dt / 2;
 *  - fine ghost zones beyond the refined region: conservative linear
 *    interpolation of the coarse state at the fine step's start time,
 *    U(th) = (1 - th) U_old + th U_new with th = 0, then 1/2: per component
 *    and axis the MC-limited slope s = copysign(min(|dc|, 2|dl|, 2|dr|), dc)
 *    if dl dr > 0, else 0, and the fine value U + ((s_x o_x + s_y o_y) +
 *    s_z o_z), o = -1/4 / +1/4 for the lower / upper half of the parent;
 *  - flux register: per coarse face of the refined region's surface the
 *    four fine sub-face fluxes summed pairwise, (f00 + f10) + (f01 + f11),
 *    both fine steps added;
 *  - reflux: the uncovered coarse zone next to the face gets
 *    -+ dt/h_d (register / 8 - its coarse flux) (minus where the face is
 *    the zone's high face);
 *  - average down: each covered coarse zone = ((f000 + f100) + (f010 +
 *    f110)) + ((f001 + f101) + (f011 + f111)), times 1/8.
 * The coarse context is any level; the fine context's layout has as its
 * domain the refinement of one rectangle of whole coarse zones at least 3
 * coarse zones from every coarse domain face, PPM_BC_COARSE_FINE on all six
 * faces, and boxes that start and end on coarse-zone boundaries (even lower,
 * odd upper fine indices).  ppm_amr_create checks this (PPM_EINVAL, message
 * in ppm_last_error of the coarse context) and keeps device copies of the
 * interpolation, register and average-down lists and a register of 5
 * doubles per register face (library-owned, freed by ppm_amr_destroy).  The
 * contexts must outlive the hierarchy; each keeps its own step workspace. */
typedef struct ppm_amr ppm_amr;
int ppm_amr_create(ppm_ctx* coarse, ppm_ctx* fine, ppm_amr** out);
int ppm_amr_destroy(ppm_amr* a);
const char* ppm_amr_last_error(const ppm_amr* a);
/* Zones the interpolation writes, faces of the flux register, covered
 * coarse zones (any pointer may be null). */
int ppm_amr_sizes(const ppm_amr* a, int64_t* interp_zones, int64_t* register_faces, int64_t* covered_zones);

/* Fine ghost zones: the fine level's own fill (copies between fine boxes),
 * then the interpolation from the coarse states Uc_old and Uc_new (ghosts
 * filled) at th = half / 2 (half 0 or 1).  Writes Uf's ghost zones only. */
int ppm_amr_fill_fine(ppm_amr* a, const double* Uc_old, const double* Uc_new, int32_t half, double* Uf,
                      void* stream);

/* One coarse step of the hierarchy.  Reads the valid zones of Uc (its ghost
 * zones are filled in place) and Uf; writes the new coarse level to Uc_new
 * (synchronised: refluxed and averaged down) and the new fine level to Uf
 * (Uf_tmp holds the intermediate fine state).  Fc, Ff: three flux arenas
 * per level (ppm_flux_offsets of each context), overwritten.  dt > 0: fixed
 * coarse dt; dt = 0: the rule above.  dt_out (device, 2 doubles, may be
 * null) receives the coarse and the fine dt.  Needs both contexts' step
 * workspaces.  PPM_EINVAL for null or overlapping arenas, cfl outside
 * (0, 1), dt < 0, and the errors of the underlying steps. */
int ppm_amr_step(ppm_amr* a, const double* Uc, double* Uc_new, double* Uf, double* Uf_tmp, double* const* Fc,
                 double* const* Ff, const double dxc[3], const ppm_params* params, double dt, double* dt_out,
                 void* stream);

/* Batched form captured in a HIP graph: nsteps steps alternating
 * A -> B -> A ..., each step = [fill, step] with the CFL dt on the device:
 * the first step's from a dt pass over A, every later step's from the
 * update of the step before it (ppm_hydro_step_dt; the same bits).  After
 * an even nsteps the result is in A, after an odd nsteps in B.  The graph
 * keeps the pointers it was captured with (A, B, the workspace, the tile
 * lists, inflow states); launches replay it on the stream.  A launch
 * returns PPM_EINVAL, and replays nothing, once the context was destroyed
 * or its workspace (another pointer or size), tiling, step form or an
 * inflow state changed since the capture: capture again.  A and B must
 * stay allocated while the graph is launched. */
int ppm_graph_create(ppm_ctx* ctx, double* Ua, double* Ub, const double dx[3],
                     const ppm_params* params, int32_t nsteps, void* stream, ppm_graph** out);
int ppm_graph_launch(ppm_graph* g, void* stream);
int ppm_graph_destroy(ppm_graph* g);

/* Tiling of the stage launches: `tile` zones per tile / threads per
 * workgroup (64, 128, 256 or 512) and the strip height (rows) of the tile
 * order (each strip of the planes is swept through all planes before the
 * next; 0: plane by plane).  Rebuilds and uploads the tile lists;
 * synchronises the device first.  Results do not depend on the tiling. */
int ppm_set_tiling(ppm_ctx* ctx, int32_t tile, int32_t strip_rows);
int ppm_get_tiling(const ppm_ctx* ctx, int32_t* tile, int32_t* strip_rows);

/* Form of the step's last stage.  fused = 0 (the default): the final
 * fluxes go to the workspace and a separate kernel updates the zones.
 * fused = 1: the final fluxes of each brick of 32 x 4 x 4 valid zones are
 * computed into LDS and the brick is updated from them in the same kernel
 * (the fluxes on a brick's faces are computed by both bricks that share
 * them).  fused = 2: each workgroup owns an x-y tile of valid zones
 * (ppm_set_stream_tiling) and walks it through a run of z planes: per plane
 * its lanes solve every x and y face of the tile and each zone's high z
 * face once into LDS (the high z faces serve as the next plane's low ones),
 * then update the plane (only the faces shared with neighbouring tiles and
 * runs are solved twice).  In forms 1 and 2 nothing is written to the
 * workspace's final-flux planes.  Results are identical bit for bit in all
 * forms.  The species step always runs the staged form (it reads the final
 * mass fluxes from the workspace).  The autotuner picks among the forms and
 * the tile shape. */
int ppm_set_step_form(ppm_ctx* ctx, int32_t fused);
int ppm_get_step_form(const ppm_ctx* ctx, int32_t* fused);
/* Tile of the streamed final stage (form 2): sx x sy valid zones in x-y
 * (sx, sy >= 2; sx * sy a multiple of 32 up to 256; the workgroup has twice
 * as many lanes), runs of sz planes in z.  Default 16 x 8 x 32.
 * Synchronises the device when form 2 is active (the tile list is
 * rebuilt).  PPM_EINVAL otherwise. */
int ppm_set_stream_tiling(ppm_ctx* ctx, int32_t sx, int32_t sy, int32_t sz);
int ppm_get_stream_tiling(const ppm_ctx* ctx, int32_t* sx, int32_t* sy, int32_t* sz);

/* Form of the step's front end, the PPM reconstruction with characteristic
 * tracing (paper Sec. 1's explicit advance; O4, O5) and the normal-predictor
 * Riemann solves (O7).  form 0: two staged kernels, the tracing
 * writing the traced face states to the workspace and the solves reading
 * them back.  form 1: one kernel whose workgroups each own an x-y tile of a
 * box's traced zones and walk it through a run of z planes; per plane each
 * zone is traced along the three axes (a lane per zone and axis) and the
 * stage-1 problems on its low faces solved after a barrier, the x and y
 * neighbours' states exchanged through LDS and the z neighbour's kept in
 * registers from the plane before, so the traced states are written (later
 * stages read them) but not read back.
 * form 2: the x axis's tracing and solves in one kernel whose wavefronts
 * each trace 64 consecutive zones, the first of them the previous
 * wavefront's last, so both states of every x face they solve meet in
 * neighbouring lanes (a lane shuffle; no LDS, no barrier); y and z staged
 * (the default).
 * form 3: the same for every axis; along y and z each wavefront traces an
 * 8 x 8 patch of the x-y or x-z plane whose first row along the axis is the
 * previous patch's last (one zone in eight traced twice).
 * Results are identical bit for bit in all forms (also for the adjoint's
 * recompute and the species step, which run the same front end).  Tiles of
 * form 1: ppm_set_front_tiling.  The autotuner picks the form and the
 * tile. */
int ppm_set_front_form(ppm_ctx* ctx, int32_t form);
int ppm_get_front_form(const ppm_ctx* ctx, int32_t* form);
/* Tile of the streamed front end: at most sx x sy traced zones in x-y and
 * runs of at most sz planes in z, each box's traced grid cut as evenly as
 * possible (sx, sy, sz >= 1, sx * sy <= 128, sx + sy <= 128: the workgroup
 * has a group of lanes per axis, one per zone of the tile, and one group
 * for the rows and columns of its low edges, each group whole wavefronts,
 * up to 512 lanes).  Default 16 x 8 x 32.  Synchronises the device (the
 * tile list is rebuilt).  PPM_EINVAL otherwise. */
int ppm_set_front_tiling(ppm_ctx* ctx, int32_t sx, int32_t sy, int32_t sz);
int ppm_get_front_tiling(const ppm_ctx* ctx, int32_t* sx, int32_t* sy, int32_t* sz);

/* Autotuner: times the batched step as graphs and steady loops run it
 * (ppm_hydro_step_dt, the next dt left on the device; reps steps after one
 * warm-up, HIP events on the stream) from the filled state U into Unew for
 * every candidate tile size x strip height, keeps the fastest, then times
 * the final stage staged (form 0), in bricks (form 1) and streamed (form 2)
 * with several tile shapes and keeps the fastest, and appends the choice
 * to the JSON-lines
 * file cache_path (may be null) keyed by device architecture, precision
 * and the histogram of box extents; a matching entry in the file is
 * applied without timing (*from_cache = 1).  Synchronises.  Writes the
 * chosen tiling to *tile, *strip_rows (ppm_get_step_form and
 * ppm_get_stream_tiling give the rest). */
int ppm_autotune(ppm_ctx* ctx, const double* U, double* Unew, const double dx[3], const ppm_params* params,
                 int32_t reps, const char* cache_path, void* stream, int32_t* tile, int32_t* strip_rows,
                 int32_t* from_cache);

/* Stage timing with HIP events recorded on the caller's stream around each
 * batched fill, dt and step stage launch while enabled (per-box launches are
 * not timed).  ppm_profile_read waits for the recorded events, writes the
 * summed milliseconds and the number of timed launches of each stage to
 * ms[PPM_PROF_NTAGS] and count[PPM_PROF_NTAGS], and forgets them. */
enum { PPM_PROF_FILL = 0, PPM_PROF_DT, PPM_PROF_PRIM, PPM_PROF_FLATTEN, PPM_PROF_TRACE,
       PPM_PROF_RIEMANN1, PPM_PROF_RIEMANN2, PPM_PROF_RIEMANN3, PPM_PROF_UPDATE, PPM_PROF_NTAGS };
int ppm_profile_enable(ppm_ctx* ctx, int32_t on);
int ppm_profile_read(ppm_ctx* ctx, double* ms, int64_t* count);

/* Synchronises the stream, returns the accumulated PPM_FLAG_* bits in
 * *flags and clears them.  Returns PPM_ENONPHYS if any flag was set. */
int ppm_check_status(ppm_ctx* ctx, void* stream, int32_t* flags);

/* ---- the ghost-fill plan on the host (no device work, no GPU needed) --- */
/* Builds the fill plan of a layout: brute = 0 takes it from the plan cache
 * (hash-sorted intersections, paper Sec. 2, built on a miss), brute != 0
 * builds it by all-pairs box intersection, O(N^2).  Writes up to max
 * descriptors of 20 int32 each to out20 (may be null) and the descriptor
 * count to *count.  Descriptor: dst box, src box, dst lo[3], dst hi[3]
 * (destination-box-local zone indices), per-axis map src = a*dst + c as
 * a[3], c[3] (source-box-local), sign mask (bit d: momentum d negated),
 * zone count, 4 reserved.  Both forms list the same descriptors in the same
 * order.  PPM_EINVAL for an invalid layout. */
int ppm_plan_build(const ppm_layout* layout, int32_t brute, int32_t max, int32_t* out20, int32_t* count);
/* Executes the cached plan of the layout on a host copy of the state arena. */
int ppm_fill_boundary_host(const ppm_layout* layout, double* U_host);
/* Plan cache statistics: lookups, hits, entries. */
int ppm_plan_cache_stats(int64_t* lookups, int64_t* hits, int32_t* entries);

#ifdef __cplusplus
}
#endif
#endif /* PPM_H */

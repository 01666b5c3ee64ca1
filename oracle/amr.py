"""TEST INFRASTRUCTURE -- oracle of the two-level advance with subcycling.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It imports nothing from the product
package; the single-level steps and fills are the C++ oracle's
(``oracle.py``), the level operations below are plain numpy.

Structured AMR with two levels and refinement ratio 2 (paper Sec. 1: the
compressible code uses adaptive mesh refinement; Sec. 2: ghost cells are
filled from intersecting grids and the solution is synchronised between
levels of refinement; Sec. 3: with subcycling in time a coarse time step is
one step on the coarse grid and two on the fine grid, and the refined region
of the multilevel runs is the inner 12.5% of the domain).  The paper names
these pieces, not their formulas; the reading is the standard
Berger-Colella advance:

  A1 time step: one coarse dt for both levels,
       dt_c = cfl / max(S_c, S_f / 2),
     S the level's maximum over valid zones and axes of (|u_d| + c)/h_d;
     the fine level takes two steps of dt_f = dt_c / 2.
  A2 coarse step: the single-level step on every coarse box (ghosts filled
     by the coarse fill), keeping its face fluxes.
  A3 fine ghost zones: copies from other fine boxes where those exist; beyond
     the refined region, conservative linear interpolation of the coarse
     state at the fine step's start time,
       U(th) = (1 - th) U_old + th U_new,   th = 0, then 1/2,
     with per component and axis the MC-limited slope
       s = copysign(min(|dc|, 2|dl|, 2|dr|), dc) if dl dr > 0 else 0,
       dc = (U[i+1] - U[i-1])/2, dl = U[i] - U[i-1], dr = U[i+1] - U[i],
     and fine value U + ((s_x o_x + s_y o_y) + s_z o_z), o_d = -1/4 for the
     lower and +1/4 for the upper half of the coarse parent along d.  U_new
     is the coarse step's result before synchronisation.
  A4 flux register: on every coarse face of the refined region's surface,
     the fine fluxes of its four sub-faces are summed pairwise,
     (f(0,0) + f(1,0)) + (f(0,1) + f(1,1)) in (t1, t2) offsets (t1 < t2 the
     transverse axes), sub-step 0 then sub-step 1 added to a zeroed
     register, and the sum times 1/8 is the fine flux averaged over the
     coarse face and step (pairwise sums keep equal values exact).
  A5 reflux: the uncovered coarse zone next to such a face is corrected by
     dt_c/h_d (averaged fine flux - its coarse flux): subtracted when the
     face is the zone's high face, added when it is its low face.
  A6 average down: each covered coarse zone becomes the mean of its eight
     fine zones, summed pairwise along x, then y, then z:
     ((f000 + f100) + (f010 + f110)) + ((f001 + f101) + (f011 + f111)),
     times 1/8.

Requirements (checked): the refined region is one rectangle of whole coarse
zones at least 3 coarse zones from every domain face; the fine boxes tile
its refinement exactly and start and end on coarse-zone boundaries (even
lower, odd upper fine indices).
"""
import numpy as np

from . import oracle as O

NG = 4
RATIO = 2
MARGIN = 3  # coarse zones between the refined region and the domain faces
BC_CF = O.BC_COARSE_FINE


def _interior(U):
    return U[:, NG:-NG, NG:-NG, NG:-NG]


class Hierarchy:
    """Coarse level (boxes tiling the domain, face BCs) and a fine level
    tiling the refinement of the coarse-index rectangle `region`."""

    def __init__(self, cboxes, cdomain, cbc, fboxes, region):
        self.cboxes = [(tuple(map(int, lo)), tuple(map(int, hi))) for lo, hi in cboxes]
        self.cdomain = (tuple(map(int, cdomain[0])), tuple(map(int, cdomain[1])))
        self.cbc = tuple(int(v) for v in cbc)
        self.fboxes = [(tuple(map(int, lo)), tuple(map(int, hi))) for lo, hi in fboxes]
        self.region = (tuple(map(int, region[0])), tuple(map(int, region[1])))
        rlo, rhi = self.region
        dlo, dhi = self.cdomain
        for d in range(3):
            if rlo[d] - dlo[d] < MARGIN or dhi[d] - rhi[d] < MARGIN:
                raise ValueError("refined region closer than 3 coarse zones to a domain face")
        self.fdomain = (tuple(RATIO * v for v in rlo), tuple(RATIO * v + 1 for v in rhi))
        cover = np.zeros([self.fdomain[1][d] - self.fdomain[0][d] + 1 for d in (2, 1, 0)], dtype=np.int64)
        for lo, hi in self.fboxes:
            for d in range(3):
                if lo[d] % 2 or hi[d] % 2 != 1:
                    raise ValueError("fine boxes must start and end on coarse-zone boundaries")
                if lo[d] < self.fdomain[0][d] or hi[d] > self.fdomain[1][d]:
                    raise ValueError("fine box outside the refined region")
            sl = tuple(slice(lo[d] - self.fdomain[0][d], hi[d] - self.fdomain[0][d] + 1) for d in (2, 1, 0))
            cover[sl] += 1
        if not np.all(cover == 1):
            raise ValueError("fine boxes do not tile the refined region exactly")
        self.fbc = (BC_CF,) * 6


# ----------------------------------------------------------- level data ----
def coarse_global(h, cstates):
    """The coarse valid zones of all boxes as one (5, Lz, Ly, Lx) array."""
    dlo, dhi = h.cdomain
    L = [dhi[d] - dlo[d] + 1 for d in range(3)]
    G = np.full((5, L[2], L[1], L[0]), np.nan)
    for (lo, hi), U in zip(h.cboxes, cstates):
        sl = (slice(None),) + tuple(slice(lo[d] - dlo[d], hi[d] - dlo[d] + 1) for d in (2, 1, 0))
        G[sl] = _interior(U)
    return G


def _mc_slope(um, u0, up):
    dc = 0.5 * (up - um)
    dl = u0 - um
    dr = up - u0
    m = np.minimum(np.minimum(np.abs(dc), 2.0 * np.abs(dl)), 2.0 * np.abs(dr))
    return np.where(dl * dr > 0.0, np.copysign(m, dc), 0.0)


def interpolate_fine_ghosts(h, Gold, Gnew, theta, fstates):
    """A3: the ghost zones of every fine box that lie outside the refined
    region, from the coarse state at time fraction theta; in place."""
    Gt = (1.0 - theta) * Gold + theta * Gnew
    dlo = h.cdomain[0]
    flo, fhi = h.fdomain
    for (lo, hi), U in zip(h.fboxes, fstates):
        n = [hi[d] - lo[d] + 1 for d in range(3)]
        g = [lo[d] + np.arange(-NG, n[d] + NG) for d in range(3)]  # fine global indices
        out = [(g[d] < flo[d]) | (g[d] > fhi[d]) for d in range(3)]
        mask = out[2][:, None, None] | out[1][None, :, None] | out[0][None, None, :]
        ic = [np.floor_divide(g[d], RATIO) - dlo[d] for d in range(3)]  # coarse index in G
        o = [np.where(g[d] - RATIO * (ic[d] + dlo[d]) == 0, -0.25, 0.25) for d in range(3)]
        iz, iy, ix = np.meshgrid(ic[2], ic[1], ic[0], indexing="ij")
        oz, oy, ox = np.meshgrid(o[2], o[1], o[0], indexing="ij")
        for c in range(5):
            A = Gt[c]
            u0 = A[iz, iy, ix]
            sx = _mc_slope(A[iz, iy, ix - 1], u0, A[iz, iy, ix + 1])
            sy = _mc_slope(A[iz, iy - 1, ix], u0, A[iz, iy + 1, ix])
            sz = _mc_slope(A[iz - 1, iy, ix], u0, A[iz + 1, iy, ix])
            val = u0 + ((sx * ox + sy * oy) + sz * oz)
            U[c][mask] = val[mask]
    return fstates


def fill_fine(h, Gold, Gnew, theta, fstates):
    """Fine ghost zones: intra-level copies, then the interpolation."""
    O.fill(h.fboxes, h.fdomain, h.fbc, fstates)
    return interpolate_fine_ghosts(h, Gold, Gnew, theta, fstates)


# ------------------------------------------------ flux register, reflux ----
def _owner(boxes, x):
    for b, (lo, hi) in enumerate(boxes):
        if all(lo[d] <= x[d] <= hi[d] for d in range(3)):
            return b
    raise ValueError(f"no box owns {x}")


def register_faces(h):
    """Coarse faces of the refined region's surface: list of (d, side,
    (x, y, z) of the uncovered coarse zone, global coarse face index along
    d).  side 0: the region's low face (the face is the zone's high face);
    side 1: its high face (the zone's low face)."""
    rlo, rhi = h.region
    faces = []
    for d in range(3):
        t = [a for a in range(3) if a != d]
        for side in (0, 1):
            fc = rlo[d] if side == 0 else rhi[d] + 1
            zc = fc - 1 if side == 0 else fc
            for k in range(rlo[t[1]], rhi[t[1]] + 1):
                for j in range(rlo[t[0]], rhi[t[0]] + 1):
                    x = [0, 0, 0]
                    x[d], x[t[0]], x[t[1]] = zc, j, k
                    faces.append((d, side, tuple(x), fc))
    return faces


def fine_face_sum(h, Ff, d, fc, j, k):
    """A4 for one coarse face and one fine sub-step: the four fine sub-face
    fluxes (5 components) summed in the stated order.  (j, k): the coarse
    indices along the transverse axes t1 < t2."""
    t1, t2 = [a for a in range(3) if a != d]
    v = {}
    for b2 in (0, 1):
        for b1 in (0, 1):
            x = [0, 0, 0]
            x[d] = RATIO * fc
            x[t1] = RATIO * j + b1
            x[t2] = RATIO * k + b2
            # the fine box that has this face: its zone on the inner side
            inner = list(x)
            if x[d] > h.fdomain[0][d]:
                inner[d] = x[d] - 1
            b = _owner(h.fboxes, inner)
            lo = h.fboxes[b][0]
            loc = [x[a] - lo[a] for a in range(3)]
            v[b1, b2] = Ff[b][d][:, loc[2], loc[1], loc[0]]
    return (v[0, 0] + v[1, 0]) + (v[0, 1] + v[1, 1])


def reflux(h, cnew, Fc, reg, dt, dxc):
    """A5 on the new coarse states (in place).  reg: {face index: summed
    fine flux of both sub-steps}; Fc: per coarse box its three flux arrays."""
    for i, (d, side, x, fc) in enumerate(register_faces(h)):
        b = _owner(h.cboxes, x)
        lo = h.cboxes[b][0]
        loc = [x[a] - lo[a] for a in range(3)]
        fl = list(loc)
        if side == 0:
            fl[d] += 1  # the zone's high face
        fcv = Fc[b][d][:, fl[2], fl[1], fl[0]]
        dF = reg[i] * 0.125 - fcv
        dtdx = dt / dxc[d]
        U = cnew[b]
        z = (slice(None), loc[2] + NG, loc[1] + NG, loc[0] + NG)
        U[z] = U[z] - dtdx * dF if side == 0 else U[z] + dtdx * dF
    return cnew


def average_down(h, cstates, fstates):
    """A6: covered coarse zones take the mean of their fine zones (in place)."""
    flo = h.fdomain[0]
    for (clo, chi), Uc in zip(h.cboxes, cstates):
        for (lo, hi), Uf in zip(h.fboxes, fstates):
            a = [max(clo[d], lo[d] // RATIO) for d in range(3)]
            e = [min(chi[d], hi[d] // RATIO) for d in range(3)]
            if any(a[d] > e[d] for d in range(3)):
                continue
            # fine-box-local index of the first child of coarse zone a
            f0 = [RATIO * a[d] - lo[d] + NG for d in range(3)]
            m = [e[d] - a[d] + 1 for d in range(3)]

            def child(cx, cy, cz):
                return Uf[:, f0[2] + cz:f0[2] + cz + RATIO * m[2]:RATIO,
                          f0[1] + cy:f0[1] + cy + RATIO * m[1]:RATIO,
                          f0[0] + cx:f0[0] + cx + RATIO * m[0]:RATIO]
            s = (((child(0, 0, 0) + child(1, 0, 0)) + (child(0, 1, 0) + child(1, 1, 0)))
                 + ((child(0, 0, 1) + child(1, 0, 1)) + (child(0, 1, 1) + child(1, 1, 1))))
            sl = (slice(None),) + tuple(slice(a[d] - clo[d] + NG, e[d] - clo[d] + NG + 1) for d in (2, 1, 0))
            Uc[sl] = s * 0.125
    del flo
    return cstates


# ------------------------------------------------------------- advance -----
def coarse_dt(h, cstates, fstates, dxc, p):
    """A1: (dt_c, S_c, S_f, flags)."""
    dxf = tuple(v / RATIO for v in dxc)
    sc, sf, fl = 0.0, 0.0, 0
    for U in cstates:
        s, f = O.max_wavespeed(U, dxc, p)
        sc, fl = max(sc, s), fl | f
    for U in fstates:
        s, f = O.max_wavespeed(U, dxf, p)
        sf, fl = max(sf, s), fl | f
    return p.cfl / max(sc, 0.5 * sf), sc, sf, fl


def coarse_step(h, cstates, fstates, dxc, p, dt=None, sync=True):
    """One coarse step of the hierarchy (A1-A6).  Returns (new coarse
    states, new fine states, dt, flags); the inputs are not modified.
    sync=False leaves out A5 and A6 (a control for the tests only)."""
    cstates = [U.copy() for U in cstates]
    fstates = [U.copy() for U in fstates]
    dxf = tuple(v / RATIO for v in dxc)
    O.fill(h.cboxes, h.cdomain, h.cbc, cstates)
    flags = 0
    if dt is None:
        dt, _, _, flags = coarse_dt(h, cstates, fstates, dxc, p)
    # A2
    cnew, Fc = [], []
    for b, U in enumerate(cstates):
        Un, F, fl = O.step(U, dt, dxc, p, fluxes=True, walls=O.box_walls(h.cboxes, h.cdomain, h.cbc, b))
        cnew.append(Un)
        Fc.append(F)
        flags |= fl
    O.fill(h.cboxes, h.cdomain, h.cbc, cnew)
    Gold, Gnew = coarse_global(h, cstates), coarse_global(h, cnew)
    # A3 + fine steps + A4
    faces = register_faces(h)
    reg = [np.zeros(5) for _ in faces]
    dtf = 0.5 * dt
    for k in range(RATIO):
        fill_fine(h, Gold, Gnew, 0.5 * k, fstates)
        fnew, Ff = [], []
        for U in fstates:
            Un, F, fl = O.step(U, dtf, dxf, p, fluxes=True)
            fnew.append(Un)
            Ff.append(F)
            flags |= fl
        for i, (d, side, x, fc) in enumerate(faces):
            t1, t2 = [a for a in range(3) if a != d]
            reg[i] = reg[i] + fine_face_sum(h, Ff, d, fc, x[t1], x[t2])
        fstates = fnew
    # A5, A6
    if sync:
        reflux(h, cnew, Fc, reg, dt, dxc)
        average_down(h, cnew, fstates)
    return cnew, fstates, dt, flags


def advance(h, cstates, fstates, nsteps, dxc, p, dt=None):
    """nsteps coarse steps; returns (coarse states, fine states, dts, flags)."""
    dts, flags = [], 0
    for _ in range(nsteps):
        cstates, fstates, dtn, fl = coarse_step(h, cstates, fstates, dxc, p, dt=dt)
        dts.append(dtn)
        flags |= fl
    return cstates, fstates, dts, flags


def composite_sums(h, cstates, fstates, dxc):
    """Per component, the integral over the domain of the composite solution
    (uncovered coarse zones and fine zones), exactly summed."""
    import math
    rlo, rhi = h.region
    vc = dxc[0] * dxc[1] * dxc[2]
    vf = vc / RATIO ** 3
    out = []
    for c in range(5):
        terms = []
        for (lo, hi), U in zip(h.cboxes, cstates):
            A = _interior(U)[c]
            z = np.arange(lo[2], hi[2] + 1)[:, None, None]
            y = np.arange(lo[1], hi[1] + 1)[None, :, None]
            x = np.arange(lo[0], hi[0] + 1)[None, None, :]
            cov = ((x >= rlo[0]) & (x <= rhi[0]) & (y >= rlo[1]) & (y <= rhi[1]) & (z >= rlo[2]) & (z <= rhi[2]))
            terms.extend((A[~np.broadcast_to(cov, A.shape)] * vc).tolist())
        for U in fstates:
            terms.extend((_interior(U)[c] * vf).ravel().tolist())
        out.append(math.fsum(terms))
    return out

"""Seeded synthetic workloads: box layouts and initial states.

This module builds inputs only.  It holds none of the step's arithmetic; it
is the one module both the library's callers and the test oracle consume, so
that both sides see identical inputs.

A level is a set of disjoint boxes (FABs) tiling a rectangular domain (the
MultiFAB of the paper's Sec. 2).  The state of the level lives in one float64
arena; box b occupies ``arena[off[b] : off[b] + 5*Nz*Ny*Nx]`` with layout
[component][k][j][i], N = n + 8 (4 ghost zones per side).  Components are the
conserved variables (rho, rho u, rho v, rho w, rho E).  Ghost zones are
poisoned with NaN: the ghost fill must overwrite every one of them.

Workloads (the five configurations of the problem statement):
  cfg1  32^3 single box, advected sine density wave, gamma 1.4, periodic
  cfg2  256^3 single box, random-mode density times a planar Sod jump in x,
        constant random velocity, gamma 5/3, periodic
  cfg3  512 boxes, 8x8x8 tensor tiling with edge lengths drawn from
        {16,24,32,48,64}, random smooth fields, gamma 1.4, periodic
  cfg4  128^3 single box, small-amplitude smooth random state, gamma 1.4
  cfg5  512^3 as 8x8x8 boxes of 64^3, Rayleigh-Taylor set-up under g=(0,0,-1),
        periodic in x and y, reflecting walls in z
A "mode sum" is S(x) = sum_m a_m cos(2 pi k_m . x / L + phi_m) with k_m drawn
uniformly from the integer vectors with 1 <= |k| <= K, a_m ~ U(0,1)
normalised to sum 1 (so |S| <= 1) and phi_m ~ U(0, 2 pi).  Fields are point
values at cell centres x = (i + 1/2) h.
"""
from dataclasses import dataclass, field
import math

import numpy as np

NG = 4
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_COARSE_FINE = 0, 1, 2, 3


@dataclass
class Layout:
    """Boxes (inclusive lo/hi global indices) tiling a domain, plus face BCs."""
    lo: np.ndarray          # (nbox, 3) int
    hi: np.ndarray          # (nbox, 3) int
    domain_lo: tuple
    domain_hi: tuple
    bc: tuple = (0, 0, 0, 0, 0, 0)   # x-lo, x-hi, y-lo, y-hi, z-lo, z-hi
    ngrow: int = NG
    _off: np.ndarray = field(default=None, repr=False)

    @property
    def nbox(self):
        return int(self.lo.shape[0])

    def n(self, b):
        return tuple(int(v) for v in (self.hi[b] - self.lo[b] + 1))

    def stored_shape(self, b):
        nx, ny, nz = self.n(b)
        g = 2 * self.ngrow
        return (5, nz + g, ny + g, nx + g)

    def box_size(self, b):
        return int(np.prod(self.stored_shape(b)))

    def offsets(self):
        if self._off is None:
            sz = [self.box_size(b) for b in range(self.nbox)]
            self._off = np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)
        return self._off

    def arena_len(self):
        return int(self.offsets()[-1])

    def view(self, arena, b):
        o = self.offsets()
        return arena[o[b]:o[b + 1]].reshape(self.stored_shape(b))

    def valid_zones(self):
        return int(sum(np.prod(self.n(b)) for b in range(self.nbox)))

    def stored_zones(self):
        return int(sum(np.prod(self.stored_shape(b)[1:]) for b in range(self.nbox)))

    def boxes(self):
        return [(tuple(int(v) for v in self.lo[b]), tuple(int(v) for v in self.hi[b]))
                for b in range(self.nbox)]

    def domain(self):
        return (tuple(self.domain_lo), tuple(self.domain_hi))


def single_box(n, bc=(0, 0, 0, 0, 0, 0)):
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    lo = np.zeros((1, 3), dtype=np.int64)
    hi = np.array([[n[0] - 1, n[1] - 1, n[2] - 1]], dtype=np.int64)
    return Layout(lo, hi, (0, 0, 0), tuple(int(v) for v in hi[0]), tuple(bc))


def tensor_tiling(sx, sy, sz, bc=(0, 0, 0, 0, 0, 0), origin=(0, 0, 0)):
    """Box (a, b, c) spans sizes sx[a] x sy[b] x sz[c]; box index a fastest;
    the first box starts at `origin`."""
    ex = origin[0] + np.concatenate([[0], np.cumsum(sx)])
    ey = origin[1] + np.concatenate([[0], np.cumsum(sy)])
    ez = origin[2] + np.concatenate([[0], np.cumsum(sz)])
    lo, hi = [], []
    for c in range(len(sz)):
        for b in range(len(sy)):
            for a in range(len(sx)):
                lo.append((ex[a], ey[b], ez[c]))
                hi.append((ex[a + 1] - 1, ey[b + 1] - 1, ez[c + 1] - 1))
    lo = np.array(lo, dtype=np.int64)
    hi = np.array(hi, dtype=np.int64)
    return Layout(lo, hi, tuple(int(v) for v in origin), (int(ex[-1] - 1), int(ey[-1] - 1), int(ez[-1] - 1)),
                  tuple(bc))


class ModeSum:
    """Random-phase Fourier mode sum on a periodic box of lengths L."""

    def __init__(self, rng, nmodes, K, L, dims=3):
        r = np.arange(-K, K + 1)
        grids = np.meshgrid(*([r] * dims), indexing="ij")
        kv = np.stack([g.ravel() for g in grids], axis=1)
        nrm = np.sqrt((kv.astype(np.float64) ** 2).sum(axis=1))
        kv = kv[(nrm >= 1.0) & (nrm <= K)]
        idx = rng.integers(0, kv.shape[0], size=nmodes)
        self.k = kv[idx].astype(np.float64)
        a = rng.uniform(0.0, 1.0, size=nmodes)
        self.a = a / a.sum()
        self.phi = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
        self.L = np.asarray(L, dtype=np.float64)
        self.dims = dims

    def __call__(self, *xs):
        """xs: coordinate arrays per axis (broadcastable); returns S."""
        out = 0.0
        for m in range(self.k.shape[0]):
            arg = self.phi[m]
            for d in range(self.dims):
                arg = arg + 2.0 * math.pi * self.k[m, d] * xs[d] / self.L[d]
            out = out + self.a[m] * np.cos(arg)
        return out


def _fill_state(layout, h, gamma, prim_fn, dtype=np.float64):
    """Evaluate prim_fn(x, y, z) -> (rho, u, v, w, p) at the cell centres of
    every box and store the conserved state; ghosts are NaN."""
    arena = np.full(layout.arena_len(), np.nan, dtype=dtype)
    g = layout.ngrow
    for b in range(layout.nbox):
        nx, ny, nz = layout.n(b)
        lo = layout.lo[b]
        x = ((lo[0] + np.arange(nx)) + 0.5)[None, None, :] * h[0]
        y = ((lo[1] + np.arange(ny)) + 0.5)[None, :, None] * h[1]
        z = ((lo[2] + np.arange(nz)) + 0.5)[:, None, None] * h[2]
        rho, u, v, w, p = [np.broadcast_to(np.asarray(f, dtype=np.float64), (nz, ny, nx))
                           for f in prim_fn(x, y, z)]
        U = layout.view(arena, b)
        U[0, g:g + nz, g:g + ny, g:g + nx] = rho
        U[1, g:g + nz, g:g + ny, g:g + nx] = rho * u
        U[2, g:g + nz, g:g + ny, g:g + nx] = rho * v
        U[3, g:g + nz, g:g + ny, g:g + nx] = rho * w
        # initial total energy of the gamma-law gas described by (rho, u, p)
        U[4, g:g + nz, g:g + ny, g:g + nx] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return arena


@dataclass
class Workload:
    name: str
    layout: Layout
    arena: np.ndarray
    dx: tuple
    gamma: float
    nsteps: int
    grav: tuple = (0.0, 0.0, 0.0)
    precision: int = 0
    meta: dict = field(default_factory=dict)


def cfg1(n=32):
    """Advected density wave rho = 1 + 0.2 sin(2 pi (x+y+z)), p = 1,
    u = (1, 0.5, 0.25) on the periodic unit cube."""
    lay = single_box(n)
    h = (1.0 / n,) * 3

    def prim(x, y, z):
        return (1.0 + 0.2 * np.sin(2.0 * math.pi * (x + y + z)), 1.0, 0.5, 0.25, 1.0)
    return Workload("cfg1", lay, _fill_state(lay, h, 1.4, prim), h, 1.4, 10)


def _cfg2_prim(seed):
    rng = np.random.default_rng(seed)
    S = ModeSum(rng, 16, 8, (1.0, 1.0, 1.0))
    vel = rng.uniform(-0.5, 0.5, size=3)

    def prim(x, y, z):
        left = x < 0.5
        rj = np.where(left, 1.0, 0.125)
        pj = np.where(left, 1.0, 0.1)
        return (rj * (1.0 + 0.1 * S(x, y, z)), vel[0], vel[1], vel[2], pj)
    return prim, vel


def cfg2(n=256, seed=2):
    """rho = rho_J(x) (1 + 0.1 S), S: 16 modes with |k| <= 8; p = p_J(x);
    rho_J, p_J = (1, 1) for x < 1/2 and (0.125, 0.1) beyond; constant velocity
    with each component ~ U[-0.5, 0.5]; gamma 5/3, periodic.  RNG draws:
    the density modes, then the three velocity components."""
    lay = single_box(n)
    h = (1.0 / n,) * 3
    prim, vel = _cfg2_prim(seed)
    return Workload("cfg2", lay, _fill_state(lay, h, 5.0 / 3.0, prim), h, 5.0 / 3.0, 20,
                    meta={"velocity": vel.tolist()})


def cfg3_layout(seed=3, sizes=(16, 24, 32, 48, 64), nper=8):
    rng = np.random.default_rng(seed)
    sx = rng.choice(sizes, nper)
    sy = rng.choice(sizes, nper)
    sz = rng.choice(sizes, nper)
    return tensor_tiling(sx, sy, sz), rng


def cfg3(seed=3, sizes=(16, 24, 32, 48, 64), nper=8, h=1.0 / 256):
    """Tensor tiling of nper^3 boxes with per-axis edge lengths drawn from
    sizes; rho = 1.25 + 0.75 S_rho, p = 1.25 + 0.75 S_p, u_d = S_d / sqrt(3)
    (8 modes each, |k| <= 4, periodic on the tiled domain); gamma 1.4.
    RNG draws: sx, sy, sz, then the modes of rho, p, u, v, w."""
    lay, rng = cfg3_layout(seed, sizes, nper)
    hh = (h, h, h)
    L = tuple((np.array(lay.domain_hi) + 1) * h)
    Sr, Sp, Su, Sv, Sw = [ModeSum(rng, 8, 4, L) for _ in range(5)]
    s3 = 1.0 / math.sqrt(3.0)

    def prim(x, y, z):
        return (1.25 + 0.75 * Sr(x, y, z), s3 * Su(x, y, z), s3 * Sv(x, y, z), s3 * Sw(x, y, z),
                1.25 + 0.75 * Sp(x, y, z))
    return Workload("cfg3", lay, _fill_state(lay, hh, 1.4, prim), hh, 1.4, 20)


def cfg4(n=128, seed=4, amp=0.05, bulk=(0.0, 0.0, 0.0)):
    """rho = 1 + amp S_rho, p = 1 + amp S_p, u_d = bulk_d + amp S_d (8 modes
    each, |k| <= 4); gamma 1.4, periodic.  RNG draws: modes of rho, p, u, v, w.
    A bulk velocity keeps every characteristic speed away from zero (the
    tracing and the Riemann fan sampling switch branches where a speed
    changes sign, which finite differences straddle)."""
    rng = np.random.default_rng(seed)
    lay = single_box(n)
    h = (1.0 / n,) * 3
    Sr, Sp, Su, Sv, Sw = [ModeSum(rng, 8, 4, (1.0, 1.0, 1.0)) for _ in range(5)]

    def prim(x, y, z):
        return (1.0 + amp * Sr(x, y, z), bulk[0] + amp * Su(x, y, z), bulk[1] + amp * Sv(x, y, z),
                bulk[2] + amp * Sw(x, y, z), 1.0 + amp * Sp(x, y, z))
    return Workload("cfg4", lay, _fill_state(lay, h, 1.4, prim), h, 1.4, 20)


def _logcosh(x):
    ax = np.abs(x)
    return ax + np.log1p(np.exp(-2.0 * ax)) - math.log(2.0)


def cfg5(nb=8, m=64, seed=5, precision=1):
    """Rayleigh-Taylor: nb^3 boxes of m^3 on the unit cube, h = 1/(nb m),
    g = (0, 0, -1); interface z_I = 1/2 + 0.01 S(x, y) (8 modes, |k| <= 8);
    rho = 1.5 + 0.5 tanh((z - z_I)/delta), delta = 2h; p hydrostatic for the
    unperturbed profile, p(z) = 2.5 - [1.5 z + 0.5 delta ln(cosh((z-1/2)/delta)
    / cosh(1/2/delta))], so p runs from 2.5 (bottom) to 1 (top); u = 0.
    Periodic in x and y, reflecting walls in z."""
    rng = np.random.default_rng(seed)
    sizes = [m] * nb
    lay = tensor_tiling(sizes, sizes, sizes, bc=(0, 0, 0, 0, BC_REFLECT, BC_REFLECT))
    N = nb * m
    h = (1.0 / N,) * 3
    delta = 2.0 * h[2]
    S = ModeSum(rng, 8, 8, (1.0, 1.0), dims=2)

    def prim(x, y, z):
        zi = 0.5 + 0.01 * S(x, y)
        rho = 1.5 + 0.5 * np.tanh((z - zi) / delta)
        p = 2.5 - (1.5 * z + 0.5 * delta * (_logcosh((z - 0.5) / delta) - _logcosh(0.5 / delta)))
        return (rho, 0.0, 0.0, 0.0, p)
    return Workload("cfg5", lay, _fill_state(lay, h, 1.4, prim), h, 1.4, 10, grav=(0.0, 0.0, -1.0),
                    precision=precision)


def uniform(n, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, gamma=1.4, bc=(0, 0, 0, 0, 0, 0)):
    lay = single_box(n, bc)
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    h = tuple(1.0 / v for v in nn)

    def prim(x, y, z):
        return (rho, vel[0], vel[1], vel[2], p)
    return Workload("uniform", lay, _fill_state(lay, h, gamma, prim), h, gamma, 1)


def shock_tube(n, axis=0, ntrans=4, gamma=1.4, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
               x0=0.5, bc_normal=BC_OUTFLOW):
    """Planar Riemann problem along `axis`: (rho, u_n, p) = left for x < x0,
    right beyond; ntrans zones across; outflow at the two normal faces."""
    shape = [ntrans, ntrans, ntrans]
    shape[axis] = n
    bc = [BC_PERIODIC] * 6
    bc[2 * axis] = bc[2 * axis + 1] = bc_normal
    lay = single_box(tuple(shape), tuple(bc))
    h = (1.0 / n,) * 3

    def prim(x, y, z):
        c = (x, y, z)[axis]
        lf = c < x0
        rho = np.where(lf, left[0], right[0])
        un = np.where(lf, left[1], right[1])
        p = np.where(lf, left[2], right[2])
        vel = [0.0, 0.0, 0.0]
        vel[axis] = un
        return (rho, vel[0], vel[1], vel[2], p)
    return Workload("shock_tube", lay, _fill_state(lay, h, gamma, prim), h, gamma, 1)


# ------------------------------------------------------- passive species ----
# A species arena holds the partial densities rho X_s of ns passive species
# for a whole level, box by box: box b holds ns planes over its stored
# extents, order [s][k][j][i], ghosts NaN until filled.
def species_offsets(layout, ns):
    """off[0..nbox]: element offsets of each box in a species arena of ns
    components; off[nbox] is the arena length."""
    sz = [ns * int(np.prod(layout.stored_shape(b)[1:])) for b in range(layout.nbox)]
    return np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)


def species_view(layout, arena, ns, b):
    o = species_offsets(layout, ns)
    return arena[o[b]:o[b + 1]].reshape((ns,) + layout.stored_shape(b)[1:])


def species(wl, ns, seed=11, kind="modes", amp=0.9, nmodes=4, K=3):
    """Partial densities of ns species for workload wl (its state gives rho).

    kind "modes": mass fractions X_s = w_s / sum_r w_r with
      w_s = 1 + amp S_s(x) (independent mode sums over the domain), so each
      lies in (0, 1) and they sum to one.
    kind "density": two species marking the heavy and the light fluid,
      X_0 = (rho - min rho) / (max rho - min rho), X_1 = 1 - X_0 (the
      Rayleigh-Taylor interface tracer).
    kind "const": X_s = (s + 1) / (ns + 1) for ns > 1, X = 1 for ns = 1.
    Returns the arena (ghosts NaN)."""
    lay = wl.layout
    g = lay.ngrow
    arena = np.full(int(species_offsets(lay, ns)[-1]), np.nan)
    rng = np.random.default_rng(seed)
    Ld = [(lay.domain_hi[d] - lay.domain_lo[d] + 1) * wl.dx[d] for d in range(3)]
    S = [ModeSum(rng, nmodes, K, Ld) for _ in range(ns)] if kind == "modes" else None
    if kind == "density":
        if ns != 2:
            raise ValueError("kind 'density' makes two species")
        rhos = [lay.view(wl.arena, b)[0, g:-g, g:-g, g:-g] for b in range(lay.nbox)]
        rmin = min(float(r.min()) for r in rhos)
        rmax = max(float(r.max()) for r in rhos)
    for b in range(lay.nbox):
        nx, ny, nz = lay.n(b)
        lo = lay.lo[b]
        rho = lay.view(wl.arena, b)[0, g:g + nz, g:g + ny, g:g + nx]
        if kind == "modes":
            x = ((lo[0] + np.arange(nx)) + 0.5)[None, None, :] * wl.dx[0]
            y = ((lo[1] + np.arange(ny)) + 0.5)[None, :, None] * wl.dx[1]
            z = ((lo[2] + np.arange(nz)) + 0.5)[:, None, None] * wl.dx[2]
            w = [np.broadcast_to(1.0 + amp * S[s](x, y, z), (nz, ny, nx)) for s in range(ns)]
            tot = sum(w)
            X = [ws / tot for ws in w]
        elif kind == "density":
            X0 = (rho - rmin) / (rmax - rmin)
            X = [X0, 1.0 - X0]
        elif kind == "const":
            X = [np.full((nz, ny, nx), 1.0 if ns == 1 else (s + 1.0) / (ns + 1.0)) for s in range(ns)]
        else:
            raise ValueError(kind)
        V = species_view(lay, arena, ns, b)
        for s in range(ns):
            V[s, g:g + nz, g:g + ny, g:g + nx] = rho * X[s]
    return arena


# ----------------------------------------------------- two-level AMR -------
@dataclass
class TwoLevel:
    """A coarse level tiling the periodic unit cube and a fine level (ratio
    2) tiling the refinement of the coarse-index rectangle `region`; the
    fine layout's domain is that refinement, all its faces coarse-fine."""
    name: str
    coarse: Workload
    fine: Workload
    region: tuple


def _split(total, size):
    sizes = [size] * (total // size)
    if total % size:
        sizes.append(total % size)
    return sizes


def two_level(n, cbox, fbox, prim, gamma, name, grav=(0.0, 0.0, 0.0), region=None):
    """Coarse n^3 zones on the unit cube (periodic) cut into boxes of at
    most cbox per edge; by default the inner half of every axis refined (the
    inner 12.5% of the volume), its n^3 fine zones cut into boxes of at most
    fbox per edge (fbox even).  Both levels sample prim at their own cell
    centres (h_f = h_c / 2)."""
    nc = (n, n, n) if np.isscalar(n) else tuple(n)
    if region is None:
        region = (tuple(v // 4 for v in nc), tuple(3 * v // 4 - 1 for v in nc))
    clay = tensor_tiling(_split(nc[0], cbox), _split(nc[1], cbox), _split(nc[2], cbox))
    hc = tuple(1.0 / v for v in nc)
    rlo, rhi = region
    fe = [2 * (rhi[d] - rlo[d] + 1) for d in range(3)]
    flay = tensor_tiling(_split(fe[0], fbox), _split(fe[1], fbox), _split(fe[2], fbox),
                         bc=(BC_COARSE_FINE,) * 6, origin=tuple(2 * v for v in rlo))
    hf = tuple(v / 2.0 for v in hc)
    cw = Workload(name + "_coarse", clay, _fill_state(clay, hc, gamma, prim), hc, gamma, 1, grav=tuple(grav))
    fw = Workload(name + "_fine", flay, _fill_state(flay, hf, gamma, prim), hf, gamma, 1, grav=tuple(grav))
    return TwoLevel(name, cw, fw, (tuple(rlo), tuple(rhi)))


def amr_wave(n=16, cbox=None, fbox=None):
    """cfg1's advected density wave on a two-level hierarchy."""
    def prim(x, y, z):
        return (1.0 + 0.2 * np.sin(2.0 * math.pi * (x + y + z)), 1.0, 0.5, 0.25, 1.0)
    return two_level(n, cbox or n, fbox or n, prim, 1.4, "amr_wave")


def amr_cfg2(n=256, cbox=None, fbox=None, seed=2):
    """cfg2's state (random-mode density times a Sod jump in x, constant
    velocity, gamma 5/3) with the inner 12.5% refined: n^3 coarse and n^3
    fine zones, so one coarse step (one coarse and two fine steps) costs
    three single-level steps of the coarse level plus the level operations."""
    prim, _ = _cfg2_prim(seed)
    return two_level(n, cbox or n, fbox or n, prim, 5.0 / 3.0, "amr_cfg2")


def amr_random(n=16, cbox=8, fbox=8, seed=21, grav=(0.0, 0.0, 0.0)):
    """Smooth random fields with a density/pressure jump in x, several boxes
    per level: the parity workload of the two-level advance."""
    rng = np.random.default_rng(seed)
    S = [ModeSum(rng, 6, 3, (1.0, 1.0, 1.0)) for _ in range(5)]

    def prim(x, y, z):
        rj = np.where(x < 0.45, 1.0, 0.4)
        pj = np.where(x < 0.45, 1.0, 0.3)
        return (rj * (1.0 + 0.3 * S[0](x, y, z)), 0.5 * S[1](x, y, z), 0.5 * S[2](x, y, z),
                0.5 * S[3](x, y, z), pj * (1.0 + 0.3 * S[4](x, y, z)))
    return two_level(n, cbox, fbox, prim, 1.4, "amr_random", grav=grav)


# --------------------------------------------------------- inflow jet ------
BC_INFLOW = 4


def jet_inflow_velocity(x, cs):
    """Normal velocity of the jet at the inflow face (x in cm): the paper's
    tanh profile, peak Mach number 0.1 of the gas at rest."""
    return cs * (0.01 + 0.045 * (np.tanh(100.0 * (x - 0.4)) + np.tanh(100.0 * (0.6 - x))))


def jet(n=128, nz=4, rho0=1.225e-3, p0=1.01325e6, gamma=1.4):
    """The inflowing jet (compressible side of the paper's end-to-end
    test): a 1 cm x 1 cm domain of n^2 zones, nz zones thick and periodic in
    z (a planar problem); air at rest, rho0 g/cm^3 and p0 dyn/cm^2 (sea-level
    values: the paper says only 'terrestrial'); the face y = 0 is an inflow
    face with density rho0/2, pressure p0 and normal velocity
    jet_inflow_velocity(x, c_s), c_s = sqrt(gamma p0 / rho0) of the gas at
    rest; outflow at the other x and y faces; run to t = 300 us.
    meta['inflow'] = {2: (5, nz, n) conserved inflow state over the y-lo
    face, order [c][z][x]}."""
    lay = single_box((n, n, nz), bc=(BC_OUTFLOW, BC_OUTFLOW, BC_INFLOW, BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC))
    h = (1.0 / n,) * 3
    cs = math.sqrt(gamma * p0 / rho0)

    def prim(x, y, z):
        return (rho0, 0.0, 0.0, 0.0, p0)
    arena = _fill_state(lay, h, gamma, prim)
    x = (np.arange(n) + 0.5) * h[0]
    v = jet_inflow_velocity(x, cs)
    rin = 0.5 * rho0
    face = np.zeros((5, nz, n))
    face[0] = rin
    face[2] = rin * v[None, :]
    face[4] = p0 / (gamma - 1.0) + 0.5 * rin * (v * v)[None, :]
    return Workload("jet", lay, arena, h, gamma, 0,
                    meta={"inflow": {2: face}, "t_end": 3.0e-4, "sound_speed": cs, "rho0": rho0, "p0": p0})

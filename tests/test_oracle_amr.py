"""Pins of the oracle's two-level advance (refinement ratio 2, subcycling,
flux register, reflux, average down) against conservation, exact solutions,
exactness of the interpolation on linear data, symmetry and convergence.
CPU only."""
import math

import numpy as np
import pytest

from oracle import amr as A
from oracle import oracle as O
from paper_1008_2801_amd import inputs as I

NG = 4


def hier(t):
    c, f = t.coarse.layout, t.fine.layout
    return A.Hierarchy(c.boxes(), c.domain(), c.bc, f.boxes(), t.region)


def states(t):
    c, f = t.coarse.layout, t.fine.layout
    return ([c.view(t.coarse.arena, b).copy() for b in range(c.nbox)],
            [f.view(t.fine.arena, b).copy() for b in range(f.nbox)])


def _centres(lo, hi, h, ng=0):
    return [((np.arange(lo[d] - ng, hi[d] + ng + 1)) + 0.5) * h[d] for d in range(3)]


@pytest.mark.parametrize("cbox,fbox,grav", [(8, 8, (0.0, 0.0, 0.0)), (8, 6, (0.0, 0.0, 0.0)),
                                            (16, 4, (0.3, -0.2, 0.1))])
def test_composite_conservation(cbox, fbox, grav):
    """The composite solution (uncovered coarse zones and fine zones)
    conserves mass, momentum (without gravity) and energy (without gravity)
    to round-off over three coarse steps; fine boxes aligned and misaligned
    with the coarse boxes.  Without the synchronisation (reflux and average
    down) it does not: the pin has power."""
    t = I.amr_random(16, cbox, fbox, grav=grav)
    h = hier(t)
    cs, fs = states(t)
    p = O.params(gamma=1.4, grav=grav)
    s0 = A.composite_sums(h, cs, fs, t.coarse.dx)
    scale = A.composite_sums(h, [np.abs(u) for u in cs], [np.abs(u) for u in fs], t.coarse.dx)
    c2, f2, dts, fl = A.advance(h, cs, fs, 3, t.coarse.dx, p)
    assert fl == 0
    s1 = A.composite_sums(h, c2, f2, t.coarse.dx)
    comps = [0] if any(grav) else range(5)
    for c in comps:
        assert abs(s1[c] - s0[c]) <= 1e-14 * scale[c], (c, s1[c] - s0[c])
    # control: the same three steps without synchronisation
    cs3, fs3 = states(t)
    for _ in range(3):
        cs3, fs3, _, _ = A.coarse_step(h, cs3, fs3, t.coarse.dx, p, sync=False)
    s3 = A.composite_sums(h, cs3, fs3, t.coarse.dx)
    assert abs(s3[0] - s0[0]) > 1e-8 * scale[0]


def test_uniform_state_preserved_bitwise():
    def prim(x, y, z):
        return (1.3, 0.3, -0.2, 0.1, 0.7)
    t = I.two_level(16, 8, 8, prim, 1.4, "uniform")
    h = hier(t)
    cs, fs = states(t)
    c2, f2, _, fl = A.advance(h, cs, fs, 2, t.coarse.dx, O.params(gamma=1.4))
    assert fl == 0
    for a, b in zip(cs + fs, c2 + f2):
        assert np.array_equal(a[:, NG:-NG, NG:-NG, NG:-NG], b[:, NG:-NG, NG:-NG, NG:-NG])


def test_uniform_acceleration_needs_the_time_interpolation():
    """Uniform density and pressure under constant gravity: the exact
    solution stays uniform with u(t) = u0 + g t.  Momentum is linear in time,
    so the fine ghost zones of the second sub-step (the coarse state half way
    through the coarse step) get it exactly; the energy is quadratic in t,
    so they get it to O(dt^2), and the composite stays on the exact solution
    to second order in dt (errors fall 4x when dt halves).  Taking the
    coarse state at a wrong time leaves an O(dt) velocity error in the
    ghosts: errors 100x larger, falling only 2x."""
    g = (0.0, 0.0, -2.0)
    u0 = (0.2, 0.1, 0.3)

    def prim(x, y, z):
        return (1.1, u0[0], u0[1], u0[2], 0.9)
    t = I.two_level(16, 8, 8, prim, 1.4, "accel", grav=g)
    h = hier(t)
    p = O.params(gamma=1.4, grav=g)

    def errors(nsteps, dt):
        cs, fs = states(t)
        c2, f2, dts, fl = A.advance(h, cs, fs, nsteps, t.coarse.dx, p, dt=dt)
        assert fl == 0
        T = sum(dts)
        er, ew = 0.0, 0.0
        for U in c2 + f2:
            V = U[:, NG:-NG, NG:-NG, NG:-NG]
            er = max(er, np.abs(V[0] - 1.1).max())
            ew = max(ew, np.abs(V[3] / V[0] - (u0[2] + g[2] * T)).max())
        return er, ew
    e1 = errors(2, 0.016)
    e2 = errors(4, 0.008)
    assert e1[0] <= 1e-4 and e1[1] <= 1e-4, e1
    assert e1[0] / e2[0] >= 3.0 and e1[1] / e2[1] >= 3.0, (e1, e2)


def test_interpolation_is_exact_on_linear_data_and_conservative():
    """Coarse data linear in x, y, z (unlimited slopes = the exact
    gradient): every interpolated fine ghost zone equals the linear function
    at its centre; on random data the mean of the eight fine zones of a
    coarse zone whose children are all interpolated equals that coarse
    value (the offsets +-1/4 cancel)."""
    t = I.amr_random(16, 8, 8)
    h = hier(t)
    hc = t.coarse.dx
    hf = t.fine.dx
    a = np.array([0.7, -1.3, 0.4, 2.1, 0.25])
    grad = np.array([[1.0, -0.5, 0.25], [0.3, 0.2, -0.7], [-0.4, 0.9, 0.1], [0.5, 0.5, 0.5], [-1.1, 0.0, 0.6]])
    dlo, dhi = h.cdomain
    xc = _centres(dlo, dhi, hc)
    G = np.stack([a[c] + grad[c, 0] * xc[0][None, None, :] + grad[c, 1] * xc[1][None, :, None]
                  + grad[c, 2] * xc[2][:, None, None] for c in range(5)])
    _, fs = states(t)
    A.interpolate_fine_ghosts(h, G, G, 0.0, fs)
    flo, fhi = h.fdomain
    nchecked = 0
    for (lo, hi), U in zip(h.fboxes, fs):
        xf = _centres(lo, hi, hf, NG)
        g = [np.arange(lo[d] - NG, hi[d] + NG + 1) for d in range(3)]
        out = [(g[d] < flo[d]) | (g[d] > fhi[d]) for d in range(3)]
        mask = out[2][:, None, None] | out[1][None, :, None] | out[0][None, None, :]
        for c in range(5):
            ex = (a[c] + grad[c, 0] * xf[0][None, None, :] + grad[c, 1] * xf[1][None, :, None]
                  + grad[c, 2] * xf[2][:, None, None])
            assert np.abs(U[c][mask] - ex[mask]).max() <= 1e-14
        nchecked += int(mask.sum())
    assert nchecked > 0
    # conservation on random data: coarse zones one layer outside the region
    rng = np.random.default_rng(3)
    G = rng.uniform(0.5, 2.0, G.shape)
    _, fs = states(t)
    A.interpolate_fine_ghosts(h, G, G, 0.0, fs)
    rlo, rhi = h.region
    worst = 0.0
    for (lo, hi), U in zip(h.fboxes, fs):
        for xc_ in range(lo[0] // 2 - 2, hi[0] // 2 + 3):
            for yc in range(lo[1] // 2 - 2, hi[1] // 2 + 3):
                for zc in range(lo[2] // 2 - 2, hi[2] // 2 + 3):
                    inside = all(rlo[d] <= v <= rhi[d] for d, v in enumerate((xc_, yc, zc)))
                    if inside:
                        continue
                    f0 = [2 * v - lo[d] + NG for d, v in enumerate((xc_, yc, zc))]
                    if any(f0[d] < 0 or f0[d] + 1 >= U.shape[3 - d] for d in range(3)):
                        continue
                    blk = U[:, f0[2]:f0[2] + 2, f0[1]:f0[1] + 2, f0[0]:f0[0] + 2]
                    cz = G[:, zc - dlo[2], yc - dlo[1], xc_ - dlo[0]]
                    worst = max(worst, np.abs(blk.mean(axis=(1, 2, 3)) - cz).max())
    assert worst <= 1e-15


def test_average_down_of_linear_fine_data_is_the_coarse_centre_value():
    """The mean of the eight fine zones of a coarse zone is the midpoint
    value for linear data: covered coarse zones become the linear function
    at their own centres; uncovered zones are not touched."""
    t = I.amr_random(16, 8, 6)
    h = hier(t)
    cs, fs = states(t)
    grad = (0.8, -0.3, 1.7)

    def lin(x):
        return 0.5 + grad[0] * x[0][None, None, :] + grad[1] * x[1][None, :, None] + grad[2] * x[2][:, None, None]
    for (lo, hi), U in zip(h.fboxes, fs):
        U[:] = lin(_centres(lo, hi, t.fine.dx, NG))[None]
    before = [u.copy() for u in cs]
    A.average_down(h, cs, fs)
    rlo, rhi = h.region
    for (lo, hi), U, U0 in zip(h.cboxes, cs, before):
        xc = _centres(lo, hi, t.coarse.dx)
        ex = lin(xc)
        g = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
        cov = [(g[d] >= rlo[d]) & (g[d] <= rhi[d]) for d in range(3)]
        mask = cov[2][:, None, None] & cov[1][None, :, None] & cov[0][None, None, :]
        V, V0 = U[:, NG:-NG, NG:-NG, NG:-NG], U0[:, NG:-NG, NG:-NG, NG:-NG]
        for c in range(5):
            assert np.abs(V[c][mask] - ex[mask]).max() <= 1e-14
            assert np.array_equal(V[c][~mask], V0[c][~mask])


def _mirror_level(boxes, sts, dom, d):
    """Mirror a level's data along axis d (boxes map onto mirrored boxes)."""
    out = []
    dlo, dhi = dom
    for (lo, hi), U in zip(boxes, sts):
        mlo = list(lo)
        mlo[d] = dlo[d] + dhi[d] - hi[d]
        src = [i for i, (l2, h2) in enumerate(boxes) if tuple(l2) == tuple(mlo)]
        assert len(src) == 1
        V = np.flip(sts[src[0]], axis=3 - d).copy()
        V[1 + d] = -V[1 + d]
        out.append(V)
    return out


@pytest.mark.parametrize("d", [0, 1, 2])
def test_mirror_symmetry(d):
    """Mirroring the hierarchy's data along an axis mirrors the result (to
    round-off: the sub-face sums and the averages run in index order, which
    the mirror reverses)."""
    t = I.amr_random(16, 8, 8, seed=30 + d)
    h = hier(t)
    cs, fs = states(t)
    p = O.params(gamma=1.4)
    dt = 0.01
    c2, f2, _, _ = A.coarse_step(h, cs, fs, t.coarse.dx, p, dt=dt)
    cm = _mirror_level(h.cboxes, cs, h.cdomain, d)
    fm = _mirror_level(h.fboxes, fs, h.fdomain, d)
    c3, f3, _, _ = A.coarse_step(h, cm, fm, t.coarse.dx, p, dt=dt)
    for got, ref in ((c3, _mirror_level(h.cboxes, c2, h.cdomain, d)), (f3, _mirror_level(h.fboxes, f2, h.fdomain, d))):
        for a, b in zip(got, ref):
            va, vb = a[:, NG:-NG, NG:-NG, NG:-NG], b[:, NG:-NG, NG:-NG, NG:-NG]
            assert np.abs(va - vb).max() <= 1e-13 * np.abs(vb).max()


def _wave_error(n, T):
    t = I.amr_wave(n)
    h = hier(t)
    cs, fs = states(t)
    p = O.params(gamma=1.4, limiter=0, flattening=0)
    dt0 = 0.4 / n / (1.0 + math.sqrt(1.4 / 0.8))
    m = int(math.ceil(T / dt0))
    c2, f2, _, fl = A.advance(h, cs, fs, m, t.coarse.dx, p, dt=T / m)
    assert fl == 0
    vel = (1.0, 0.5, 0.25)
    err, cnt = 0.0, 0
    for lev, sts, hh in ((h.cboxes, c2, t.coarse.dx), (h.fboxes, f2, t.fine.dx)):
        for (lo, hi), U in zip(lev, sts):
            x = _centres(lo, hi, hh)
            arg = (x[0][None, None, :] - vel[0] * T) + (x[1][None, :, None] - vel[1] * T) + \
                (x[2][:, None, None] - vel[2] * T)
            ex = 1.0 + 0.2 * np.sin(2.0 * math.pi * arg)
            e = np.abs(U[0, NG:-NG, NG:-NG, NG:-NG] - ex)
            err += e.sum()
            cnt += e.size
    return err / cnt


def test_second_order_convergence_of_the_composite_solution():
    """Advected smooth density wave through the refined region: the error
    of the whole hierarchy (both levels) falls at second order."""
    e1 = _wave_error(16, 0.05)
    e2 = _wave_error(32, 0.05)
    assert e1 / e2 >= 3.0, (e1, e2)


def test_hierarchy_requirements_are_checked():
    t = I.amr_random(16, 8, 8)
    c, f = t.coarse.layout, t.fine.layout
    with pytest.raises(ValueError, match="3 coarse zones"):
        A.Hierarchy(c.boxes(), c.domain(), c.bc, f.boxes(), ((2, 4, 4), (11, 11, 11)))
    odd = [((9, 8, 8), (15, 15, 15))] + f.boxes()[1:]
    with pytest.raises(ValueError):
        A.Hierarchy(c.boxes(), c.domain(), c.bc, odd, t.region)
    with pytest.raises(ValueError, match="tile"):
        A.Hierarchy(c.boxes(), c.domain(), c.bc, f.boxes()[1:], t.region)

"""Pins of the oracle's inflow faces (prescribed ghost state) and of the
inflowing-jet workload.  CPU only."""
import math

import numpy as np
import pytest

from oracle import exact_riemann as X
from oracle import oracle as O
from paper_1008_2801_amd import inputs as I

NG = 4
OUT, INF, PER = I.BC_OUTFLOW, I.BC_INFLOW, I.BC_PERIODIC


def _conserved(rho, vel, p, gamma, shape):
    U = np.empty((5,) + shape)
    U[0] = rho
    for d in range(3):
        U[1 + d] = rho * vel[d]
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return U


def _slab(n, prim, bc, gamma=1.4):
    lay = I.single_box(n, bc=bc)
    h = tuple(1.0 / v for v in n)
    return I.Workload("slab", lay, I._fill_state(lay, h, gamma, prim), h, gamma, 1)


def test_inflow_of_the_interior_state_keeps_it_uniform_bitwise():
    """A uniform flow entering through the y-lo face, whose inflow state is
    the flow's own, and leaving through outflow faces stays uniform."""
    vel = (0.1, 0.5, -0.2)
    wl = _slab((8, 12, 6), lambda x, y, z: (1.2, vel[0], vel[1], vel[2], 1.0), (OUT, OUT, INF, OUT, PER, PER))
    inflow = {2: _conserved(1.2, vel, 1.0, 1.4, (6, 8))}
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    out, _, fl, _ = O.advance(lay.boxes(), lay.domain(), lay.bc, st, 5, wl.dx, O.params(gamma=1.4), inflow=inflow)
    assert fl == 0
    a = out[0][:, NG:-NG, NG:-NG, NG:-NG]
    b = st[0][:, NG:-NG, NG:-NG, NG:-NG]
    assert np.array_equal(a, b)


def _inflow_riemann_error(n, t_end=0.25):
    """Gas at rest (1, 0, 1); through y = 0 flows (0.5, v = 0.4, p = 1): the
    face sees the Riemann problem (inflow state | gas at rest), whose exact
    solution for y > 0 the numerical one must approach."""
    L = (0.5, 0.4, 1.0)
    R = (1.0, 0.0, 1.0)
    wl = _slab((4, n, 4), lambda x, y, z: (R[0], 0.0, R[1], 0.0, R[2]), (PER, PER, INF, OUT, PER, PER))
    inflow = {2: _conserved(L[0], (0.0, L[1], 0.0), L[2], 1.4, (4, 4))}
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    p = O.params(gamma=1.4)
    t = 0.0
    while t < t_end - 1e-14:
        O.fill(lay.boxes(), lay.domain(), lay.bc, st, inflow=inflow)
        dt = min(p.cfl / O.max_wavespeed(st[0], wl.dx, p)[0], t_end - t)
        st[0], _, fl = O.step(st[0], dt, wl.dx, p)
        assert fl == 0
        t += dt
    rho = st[0][0, NG:-NG, NG:-NG, NG:-NG]
    assert np.array_equal(rho, np.broadcast_to(rho[:1, :, :1], rho.shape))
    y = (np.arange(n) + 0.5) / n
    exact = np.array([X.sample(L, R, 1.4, yi / t_end)[0] for yi in y])
    return np.abs(rho[0, :, 0] - exact).mean()


def test_planar_inflow_converges_to_the_exact_riemann_solution():
    errs = [_inflow_riemann_error(n) for n in (64, 128, 256)]
    assert errs[0] > errs[1] > errs[2], errs
    assert math.log2(errs[0] / errs[2]) / 2 >= 0.7, errs
    assert errs[2] < 0.01, errs


def test_jet_ghost_zones_carry_the_inflow_profile():
    """Below y = 0 every ghost layer holds the inflow state at its x (the
    outflow ghosts in x clamp to the nearest column); elsewhere the
    boundaries are outflow copies and periodic images."""
    wl = I.jet(16, nz=4)
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    face = wl.meta["inflow"][2]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st, inflow=wl.meta["inflow"])
    U = st[0]
    n = 16
    for gy in range(NG):
        blk = U[:, NG:-NG, gy, :]  # (5, z, x incl. ghosts)
        xs = np.clip(np.arange(-NG, n + NG), 0, n - 1)
        assert np.array_equal(blk, face[:, :, xs])
    assert not np.isnan(U).any()


def test_jet_stays_mirror_symmetric_about_the_jet_axis():
    """The inflow profile is symmetric about x = 1/2, the domain and the
    boundaries too: 20 steps keep the solution symmetric (to the rounding of
    the sampled profile) with the momentum along x antisymmetric."""
    wl = I.jet(32, nz=4)
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    p = O.params(gamma=1.4)
    out, dts, fl, _ = O.advance(lay.boxes(), lay.domain(), lay.bc, st, 20, wl.dx, p, inflow=wl.meta["inflow"])
    assert fl == 0
    U = out[0][:, NG:-NG, NG:-NG, NG:-NG]
    M = np.flip(U, axis=3).copy()
    M[1] = -M[1]
    scale = np.abs(U).max(axis=(1, 2, 3))
    scale[1] = scale[2]
    scale[3] = scale[2]  # no z momentum at all
    err = (np.abs(U - M).max(axis=(1, 2, 3)) / scale).max()
    assert np.all(U[3] == 0)
    assert err <= 1e-10, err
    # something happened: mass entered through the inflow face
    m0 = wl.meta["rho0"]
    assert U[0].mean() != m0 and np.abs(U[2]).max() > 0


def test_inflow_data_are_required_and_single():
    wl = I.jet(8, nz=4)
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    with pytest.raises(ValueError):
        O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    bc2 = (INF, OUT, INF, OUT, PER, PER)
    with pytest.raises(ValueError):
        O.fill(lay.boxes(), lay.domain(), bc2, st, inflow={0: np.zeros((5, 4, 8)), 2: wl.meta["inflow"][2]})

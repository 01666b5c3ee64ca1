"""Pins of the oracle's passive-species step against invariants, the density
equation it must reproduce, and symmetries.  CPU only.

A passive species is a mass fraction X carried with the flow: its partial
density rho X obeys the continuity equation with the mass flux times X.  The
step traces X like a transverse velocity (it changes only across the entropy
wave), carries it with each stage's mass flux from the side the mass comes
from, corrects it transversely like the density, and updates rho X
conservatively in FP64."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1008_2801_amd import inputs as I
from tests.helpers import interior
from tests.test_oracle_step import _random_state, _mirror

NG = 4


def _level(wl, rx, ns):
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    sp = [I.species_view(lay, rx, ns, b).copy() for b in range(lay.nbox)]
    return st, sp


def _advance(wl, rx, ns, nsteps, dt=None, **pk):
    lay = wl.layout
    st, sp = _level(wl, rx, ns)
    p = O.params(gamma=wl.gamma, grav=wl.grav, precision=wl.precision, **pk)
    return O.advance_species(lay.boxes(), lay.domain(), lay.bc, st, sp, nsteps, wl.dx, p, dt=dt)


@pytest.mark.parametrize("precision", [0, 1])
def test_uniform_fraction_stays_uniform(precision):
    """X = const on a flow with a jump: rho X / rho stays that constant (to
    FP64 round-off; with the FP32 reconstruction, to the FP32 rounding of
    the traced fraction)."""
    wl = _random_state(12, 31, jump=True)
    wl.precision = precision
    rx = I.species(wl, 2, kind="const")
    st, sp, dts, fl = _advance(wl, rx, 2, 3)
    assert fl == 0
    rho = interior(st[0])[0]
    for s, x in enumerate((1.0 / 3.0, 2.0 / 3.0)):
        dev = np.abs(interior(sp[0])[s] / rho - x).max()
        assert dev <= (1e-14 if precision == 0 else 4 * 2.0**-24), (s, dev)


@pytest.mark.parametrize("make,precision", [
    (lambda: _random_state(12, 32, jump=True), 0),
    (lambda: _random_state(12, 33, jump=True), 1),
    (lambda: I.cfg5(2, 8, precision=0), 0),
])
def test_unit_fraction_reproduces_the_density_bitwise(make, precision):
    """X = 1: the species' fluxes are the mass fluxes, so rho X follows the
    density to the last bit (walls and gravity included: gravity has no
    density source)."""
    wl = make()
    wl.precision = precision
    rx = I.species(wl, 1, kind="const")
    st, sp, dts, fl = _advance(wl, rx, 1, 3)
    assert fl == 0
    for b in range(wl.layout.nbox):
        assert np.array_equal(interior(sp[b])[0], interior(st[b])[0])


@pytest.mark.parametrize("make,kind", [
    (lambda: _random_state(12, 34, jump=True), "modes"),
    (lambda: I.cfg5(2, 8, precision=0), "density"),
])
def test_species_mass_conserved(make, kind):
    """Periodic faces and reflecting walls: the total of each rho X_s is
    conserved to round-off."""
    wl = make()
    ns = 2
    rx = I.species(wl, ns, kind=kind)
    st, sp, dts, fl = _advance(wl, rx, ns, 3)
    assert fl == 0
    lay = wl.layout
    for s in range(ns):
        a0 = np.concatenate([interior(I.species_view(lay, rx, ns, b))[s].ravel() for b in range(lay.nbox)])
        a1 = np.concatenate([interior(sp[b])[s].ravel() for b in range(lay.nbox)])
        s0, s1 = math.fsum(a0), math.fsum(a1)
        assert abs(s1 - s0) <= 1e-14 * math.fsum(np.abs(a0)), (s, s1 - s0)


@pytest.mark.parametrize("limiter,ns", [(1, 2), (0, 3)])
def test_fractions_keep_summing_to_one(limiter, ns):
    """Two species X and 1 - X (the limiter is symmetric under X -> 1 - X),
    or any number with the unlimited (linear) reconstruction: the partial
    densities keep summing to the density."""
    wl = _random_state(12, 35, jump=True)
    rx = I.species(wl, ns, kind="modes")
    if ns == 2:  # make the pair exactly complementary
        for b in range(wl.layout.nbox):
            V = I.species_view(wl.layout, rx, 2, b)
            U = wl.layout.view(wl.arena, b)
            V[1] = U[0] - V[0]
    st, sp, dts, fl = _advance(wl, rx, ns, 3, limiter=limiter, flattening=limiter)
    assert fl == 0
    rho = interior(st[0])[0]
    tot = interior(sp[0]).sum(axis=0)
    assert np.abs(tot - rho).max() <= 1e-13 * rho.max()


def test_tracer_on_uniform_density_equals_a_contact_in_the_density():
    """A pure contact (rho = f(x), u and p constant) moves like a passive
    scalar: the density of that flow after 3 steps equals rho X of the
    flow with rho = 1 and X = f(x) at the same dt, to round-off.  This ties
    the species' tracing, upwinding, transverse corrections and update to
    the density's own (whose convergence and exactness are pinned
    elsewhere); velocities of both signs exercise both upwind sides."""
    n = (12, 10, 14)  # unequal spacings: each axis has its own dt/h factors
    rng = np.random.default_rng(36)
    lay = I.single_box(n)
    h = tuple(1.0 / v for v in n)
    Sx = I.ModeSum(rng, 5, 3, (1.0, 1.0, 1.0))
    vel = (0.7, -0.4, 0.3)

    def f(x, y, z):
        return 1.0 + 0.5 * Sx(x, y, z)

    wa = I.Workload("contact", lay, I._fill_state(lay, h, 1.4, lambda x, y, z: (f(x, y, z), *vel, 1.0)),
                    h, 1.4, 1)
    wb = I.Workload("tracer", lay, I._fill_state(lay, h, 1.4, lambda x, y, z: (1.0, *vel, 1.0)), h, 1.4, 1)
    rx = I.species(wb, 1, kind="const")
    V = I.species_view(lay, rx, 1, 0)
    V[0] = wa.layout.view(wa.arena, 0)[0]  # rho_b X = 1 * f
    dt = 0.4 * min(h) / (0.7 + math.sqrt(1.4 * 1.0 / 0.5))
    sa, sxa, _, fa = _advance(wa, I.species(wa, 1, kind="const"), 1, 3, dt=dt)
    sb, sxb, _, fb = _advance(wb, rx, 1, 3, dt=dt)
    assert fa == 0 and fb == 0
    rho_a = interior(sa[0])[0]
    err = np.abs(interior(sxb[0])[0] - rho_a).max() / rho_a.max()
    assert err <= 1e-13, err
    # and the flow itself is undisturbed by the contact (a check of the set-up)
    assert np.abs(interior(sa[0])[1] / rho_a - vel[0]).max() <= 1e-13


@pytest.mark.parametrize("d", [0, 1, 2])
def test_species_mirror_symmetry_bitwise(d):
    """Mirroring the flow and the species along an axis mirrors the new
    partial densities exactly (the upwind side flips with the mass flux)."""
    wl = _random_state(10, 37 + d, jump=True)
    ns = 2
    rx = I.species(wl, ns, kind="modes", seed=38 + d)
    lay = wl.layout
    st, sp = _level(wl, rx, ns)
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    O.fill_scalars(lay.boxes(), lay.domain(), lay.bc, sp)
    U, R = st[0], sp[0]
    p = O.params(gamma=wl.gamma)
    dt = p.cfl / O.max_wavespeed(U, wl.dx, p)[0]
    A, RA, _ = O.step_species(U, R, dt, wl.dx, p)
    Rm = np.flip(R, axis=3 - d).copy()
    B, RB, _ = O.step_species(_mirror(U, d), Rm, dt, wl.dx, p)
    assert np.array_equal(interior(B), interior(_mirror(A, d)))
    assert np.array_equal(interior(RB), interior(np.flip(RA, axis=3 - d)))


def test_species_step_leaves_the_hydro_step_unchanged():
    """The species ride along: the flow's new state is bitwise the plain
    step's."""
    wl = I.cfg5(2, 8, precision=0)
    rx = I.species(wl, 2, kind="density")
    st, sp, dts, fl = _advance(wl, rx, 2, 2)
    lay = wl.layout
    ref, dts2, fl2, _ = O.advance(lay.boxes(), lay.domain(), lay.bc,
                                 [lay.view(wl.arena, b).copy() for b in range(lay.nbox)], 2, wl.dx,
                                 O.params(gamma=wl.gamma, grav=wl.grav))
    assert dts == dts2 and fl == fl2
    for b in range(lay.nbox):
        assert np.array_equal(interior(st[b]), interior(ref[b]))


def test_fill_scalars_mirrors_without_sign_change():
    """The scalar ghost fill is the state fill applied to each component,
    with no sign flip at reflecting walls."""
    wl = I.cfg5(2, 8, precision=0)
    lay = wl.layout
    rx = I.species(wl, 2, kind="density")
    sp = [I.species_view(lay, rx, 2, b).copy() for b in range(lay.nbox)]
    O.fill_scalars(lay.boxes(), lay.domain(), lay.bc, sp)
    # the same fill through the state path: put each species in the density
    # slot (never sign-flipped) of a copy of the state
    for s in range(2):
        st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
        for b in range(lay.nbox):
            st[b][0] = I.species_view(lay, rx, 2, b)[s]
        O.fill(lay.boxes(), lay.domain(), lay.bc, st)
        for b in range(lay.nbox):
            assert np.array_equal(sp[b][s], st[b][0])

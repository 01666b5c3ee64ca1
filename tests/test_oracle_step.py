"""Pins of the oracle's whole step (O1-O11) against invariants, exact
solutions and symmetries.  CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import exact_riemann as X
from paper_1008_2801_amd import inputs as I
from tests.helpers import interior, oracle_level, field_errors, rescaled

NG = 4


def _filled(wl):
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    return st


def _random_state(n, seed, amp=0.3, jump=True, gamma=1.4):
    """Smooth random state plus (optionally) a pressure/density jump in x."""
    rng = np.random.default_rng(seed)
    lay = I.single_box(n)
    h = tuple(1.0 / v for v in ((n,) * 3 if np.isscalar(n) else n))
    S = [I.ModeSum(rng, 6, 3, (1.0, 1.0, 1.0)) for _ in range(5)]

    def prim(x, y, z):
        rj = np.where(x < 0.5, 1.0, 0.3) if jump else 1.0
        pj = np.where(x < 0.5, 1.0, 0.2) if jump else 1.0
        return (rj * (1.0 + amp * S[0](x, y, z)), 0.6 * S[1](x, y, z), 0.6 * S[2](x, y, z),
                0.6 * S[3](x, y, z), pj * (1.0 + amp * S[4](x, y, z)))
    return I.Workload("rand", lay, I._fill_state(lay, h, gamma, prim), h, gamma, 1)


# ------------------------------------------------------------------ P1 -----
@pytest.mark.parametrize("limiter,precision", [(1, 0), (0, 0), (1, 1)])
def test_uniform_state_preserved_bitwise(limiter, precision):
    rng = np.random.default_rng(5)
    for _ in range(3):
        wl = I.uniform(8, rho=rng.uniform(0.2, 3), vel=rng.uniform(-1, 1, 3), p=rng.uniform(0.1, 3))
        wl.precision = precision
        st0 = [wl.layout.view(wl.arena, 0).copy()]
        out, dts, fl, _ = oracle_level(O, wl, 3, limiter=limiter)
        assert fl == 0
        assert np.array_equal(interior(out[0]), interior(st0[0]))


# ------------------------------------------------------------------ P2 -----
@pytest.mark.parametrize("make,nsteps,precision", [
    (lambda: I.cfg1(16), 4, 0),
    (lambda: I.cfg2(16), 3, 0),
    (lambda: _random_state(12, 7), 3, 0),
    (lambda: I.cfg1(16), 3, 1),
])
def test_conservation_to_roundoff(make, nsteps, precision):
    wl = make()
    wl.precision = precision
    U0 = interior(wl.layout.view(wl.arena, 0))
    out, dts, fl, _ = oracle_level(O, wl, nsteps)
    assert fl == 0
    U1 = interior(out[0])
    for c in range(5):
        s0 = math.fsum(U0[c].ravel())
        s1 = math.fsum(U1[c].ravel())
        scale = math.fsum(np.abs(U0[c]).ravel())
        assert abs(s1 - s0) <= 1e-13 * scale, (c, s1 - s0, scale)


# ------------------------------------------------------------------ P3 -----
def _mirror(U, d):
    ax = 3 - d  # numpy axis of coordinate d in (c, z, y, x)
    V = np.flip(U, axis=ax).copy()
    V[1 + d] = -V[1 + d]
    return V


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("limiter", [1, 0])
def test_mirror_symmetry_bitwise(d, limiter):
    wl = _random_state(10, 11 + d, jump=True)
    U = _filled(wl)[0]
    p = O.params(gamma=wl.gamma, limiter=limiter)
    s, _ = O.max_wavespeed(U, wl.dx, p)
    dt = p.cfl / s
    A, _, _ = O.step(U, dt, wl.dx, p)
    B, _, _ = O.step(_mirror(U, d), dt, wl.dx, p)
    assert np.array_equal(interior(B), interior(_mirror(A, d)))


# ------------------------------------------------------------------ P4 -----
def _permute(U):
    """(x, y, z) -> new axes with new x = old y, new y = old z, new z = old x."""
    V = U.transpose(0, 3, 1, 2).copy()
    return V[[0, 2, 3, 1, 4]].copy()


def test_axis_permutation_symmetry():
    wl = _random_state((10, 12, 14), 21, jump=True)
    wl.dx = (0.1, 0.1, 0.1)
    U = _filled(wl)[0]
    p = O.params(gamma=wl.gamma)
    dt = 0.5 / O.max_wavespeed(U, wl.dx, p)[0]
    A, _, _ = O.step(U, dt, wl.dx, p)
    B, _, _ = O.step(_permute(U), dt, wl.dx, p)
    err = field_errors(interior(B), interior(_permute(A)))
    assert err.max() <= 1e-14, err


# ------------------------------------------------------------------ P5 -----
def test_planar_data_gives_planar_result_and_axis_independence():
    n = 24
    rng = np.random.default_rng(3)
    prof_r = 1.0 + 0.3 * np.sin(2 * np.pi * (np.arange(n) + 0.5) / n) + np.where(np.arange(n) < n // 2, 0.5, 0)
    prof_p = 1.0 + np.where(np.arange(n) < n // 3, 1.5, 0.0)
    un = 0.3 * np.cos(2 * np.pi * (np.arange(n) + 0.5) / n)
    vt = (0.2, -0.15)
    outs = []
    for axis in range(3):
        shape = [4, 4, 4]
        shape[axis] = n
        lay = I.single_box(tuple(shape))
        h = (1.0 / n,) * 3
        idx = [None, None, None]

        def prim(x, y, z, axis=axis):
            c = (x, y, z)[axis]
            i = np.rint(c * n - 0.5).astype(int)
            vel = [0.0, 0.0, 0.0]
            t = [a for a in range(3) if a != axis]
            vel[axis] = un[i]
            vel[t[0]] = vt[0]
            vel[t[1]] = vt[1]
            return (prof_r[i], vel[0], vel[1], vel[2], prof_p[i])
        wl = I.Workload("planar", lay, I._fill_state(lay, h, 1.4, prim), h, 1.4, 1)
        out, dts, fl, _ = oracle_level(O, wl, 2, dt=0.002)
        V = interior(out[0])
        # independent of the transverse indices, bit for bit
        ax = 3 - axis
        for t in (1, 2, 3):
            if t != ax:
                ref = np.take(V, [0], axis=t)
                assert np.array_equal(V, np.broadcast_to(ref, V.shape))
        line = np.moveaxis(V, ax, 3)[:, 0, 0, :]
        perm = [0, 1 + axis] + [1 + a for a in range(3) if a != axis] + [4]
        outs.append(line[perm])
    for k in (1, 2):
        np.testing.assert_allclose(outs[k], outs[0], rtol=0, atol=1e-14 * np.abs(outs[0]).max())


# ------------------------------------------------------------------ P6 -----
def _wave_error(n, nz, T, limiter):
    """L1 error of rho after advecting the density wave to time T."""
    lay = I.single_box((n, n, nz))
    h = (1.0 / n, 1.0 / n, 1.0 / nz)
    vel = (1.0, 0.5, 0.25)
    k = (1.0, 1.0, 0.0 if nz < n else 1.0)

    def prim(x, y, z):
        return (1.0 + 0.2 * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z)), *vel, 1.0)
    wl = I.Workload("wave", lay, I._fill_state(lay, h, 1.4, prim), h, 1.4, 1)
    nsteps = int(round(T / (0.25 / n)))
    dt = T / nsteps
    out, _, fl, _ = oracle_level(O, wl, nsteps, dt=dt, limiter=limiter)
    assert fl == 0
    V = interior(out[0])
    x = ((np.arange(n) + 0.5) / n)[None, None, :]
    y = ((np.arange(n) + 0.5) / n)[None, :, None]
    z = ((np.arange(nz) + 0.5) / nz)[:, None, None]
    exact = 1.0 + 0.2 * np.sin(2 * np.pi * (k[0] * (x - vel[0] * T) + k[1] * (y - vel[1] * T)
                                            + k[2] * (z - vel[2] * T)))
    rho = V[0]
    u = V[1] / rho
    pr = 0.4 * (V[4] - 0.5 * (V[1] ** 2 + V[2] ** 2 + V[3] ** 2) / rho)
    return np.abs(rho - exact).mean(), np.abs(u - 1.0).max(), np.abs(pr - 1.0).max()


@pytest.mark.parametrize("limiter", [1, 0])
def test_second_order_convergence_advected_wave(limiter):
    """Slab version (wave in x+y, uniform in z, nz = 4) at n = 16, 32, 64."""
    T = 0.25
    errs = []
    for n in (16, 32, 64):
        e, du, dp = _wave_error(n, 4, T, limiter)
        errs.append(e)
        assert du < 1e-13 and dp < 1e-13
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] >= 1.8, (errs, rates)


@pytest.mark.parametrize("limiter,n0,n1", [(1, 24, 32), (0, 16, 32)])
def test_second_order_convergence_3d_wave(limiter, n0, n1):
    """The full 3-D wave rho = 1 + 0.2 sin(2 pi (x+y+z)).  With the limiter the
    rate approaches 2 from below as the extremum clipping shrinks (1.6 at
    16 -> 24, 2.0 at 24 -> 32, 2.2 at 32 -> 48)."""
    T = 0.125
    e0 = _wave_error(n0, n0, T, limiter)[0]
    e1 = _wave_error(n1, n1, T, limiter)[0]
    assert math.log(e0 / e1) / math.log(n1 / n0) >= 1.9


# ------------------------------------------------------------------ P7 -----
def _sod_error(n, t_end=0.1):
    wl = I.shock_tube(n, axis=0)
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    p = O.params(gamma=1.4)
    t = 0.0
    while t < t_end - 1e-14:
        O.fill(lay.boxes(), lay.domain(), lay.bc, st)
        dt = p.cfl / O.max_wavespeed(st[0], wl.dx, p)[0]
        dt = min(dt, t_end - t)
        st[0], _, fl = O.step(st[0], dt, wl.dx, p)
        assert fl == 0
        t += dt
    rho = interior(st[0])[0]
    assert np.array_equal(rho, np.broadcast_to(rho[:1, :1, :], rho.shape))
    x = (np.arange(n) + 0.5) / n
    exact = np.array([X.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (xi - 0.5) / t_end)[0] for xi in x])
    return np.abs(rho[0, 0] - exact).mean()


def test_sod_shock_tube_converges_to_exact_solution():
    errs = [_sod_error(n) for n in (64, 128, 256)]
    assert errs[0] > errs[1] > errs[2]
    assert math.log2(errs[0] / errs[2]) / 2 >= 0.7, errs
    assert errs[2] < 0.01


# ------------------------------------------------------------------ P10 ----
def test_constant_gravity_closed_form():
    n = 8
    rho, vel, pr, g = 1.3, np.array([0.2, -0.1, 0.3]), 0.9, np.array([0.1, -0.2, -1.0])
    wl = I.uniform(n, rho=rho, vel=vel, p=pr)
    wl.grav = tuple(g)
    dt, nst = 0.01, 3
    out, _, fl, _ = oracle_level(O, wl, nst, dt=dt)
    assert fl == 0
    t = dt * nst
    V = interior(out[0])
    m0 = rho * vel
    E0 = pr / 0.4 + 0.5 * rho * vel @ vel
    for d in range(3):
        np.testing.assert_allclose(V[1 + d], m0[d] + rho * g[d] * t, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(V[4], E0 + (m0 @ g) * t + 0.5 * rho * (g @ g) * t * t, rtol=1e-14)
    np.testing.assert_array_equal(V[0], rho)


# ------------------------------------------------------------------ P11 ----
def _reference_fill(lay, arena_valid, bc):
    """Ghost fill by padding the assembled domain array with numpy: 'wrap'
    for periodic, 'edge' for outflow, 'symmetric' (mirror about the wall) for
    reflecting axes with the normal momentum negated."""
    L = np.array(lay.domain_hi) + 1
    dom = np.zeros((5, L[2], L[1], L[0]))
    for b in range(lay.nbox):
        (x0, y0, z0), (x1, y1, z1) = lay.boxes()[b]
        dom[:, z0:z1 + 1, y0:y1 + 1, x0:x1 + 1] = interior(lay.view(arena_valid, b))
    pad = dom
    for d in range(3):
        ax = 3 - d
        mode = {0: "wrap", 1: "edge", 2: "symmetric"}[bc[2 * d]]
        width = [(0, 0)] * 4
        width[ax] = (NG, NG)
        pad = np.pad(pad, width, mode=mode)
        if bc[2 * d] == 2:
            sl = [slice(None)] * 4
            sl[0] = 1 + d
            sl[ax] = slice(0, NG)
            pad[tuple(sl)] *= -1
            sl[ax] = slice(-NG, None)
            pad[tuple(sl)] *= -1
    out = []
    for b in range(lay.nbox):
        (x0, y0, z0), (x1, y1, z1) = lay.boxes()[b]
        out.append(pad[:, z0:z1 + 1 + 2 * NG, y0:y1 + 1 + 2 * NG, x0:x1 + 1 + 2 * NG])
    return out


@pytest.mark.parametrize("bc", [(0, 0, 0, 0, 0, 0), (0, 0, 0, 0, 2, 2), (1, 1, 0, 0, 2, 2),
                                (2, 2, 1, 1, 0, 0)])
def test_fill_matches_padded_domain(bc):
    rng = np.random.default_rng(8)
    lay = I.tensor_tiling(rng.integers(4, 9, 3), rng.integers(4, 9, 2), rng.integers(4, 9, 3), bc=bc)
    arena = rng.normal(size=lay.arena_len())
    st = [lay.view(arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    ref = _reference_fill(lay, arena, bc)
    for b in range(lay.nbox):
        assert np.array_equal(st[b], ref[b])


# ------------------------------------------------------- consistency -------
def test_window_reproduces_full_step():
    wl = _random_state(12, 31)
    U = _filled(wl)[0]
    p = O.params(gamma=1.4)
    A, FA, _ = O.step(U, 0.01, wl.dx, p, fluxes=True)
    for w in [((0, 0, 0), (0, 0, 0)), ((3, 5, 7), (6, 5, 11)), ((11, 0, 4), (11, 11, 4))]:
        B, FB, _ = O.step(U, 0.01, wl.dx, p, window=w, fluxes=True)
        (x0, y0, z0), (x1, y1, z1) = w
        sl = (slice(None), slice(z0 + NG, z1 + NG + 1), slice(y0 + NG, y1 + NG + 1), slice(x0 + NG, x1 + NG + 1))
        assert np.array_equal(A[sl], B[sl])
        assert np.array_equal(FA[0][:, z0:z1 + 1, y0:y1 + 1, x0:x1 + 2], FB[0][:, z0:z1 + 1, y0:y1 + 1, x0:x1 + 2])


def test_flux_output_reproduces_update():
    wl = _random_state(8, 41)
    U = _filled(wl)[0]
    p = O.params(gamma=1.4)
    dt = 0.004
    A, F, _ = O.step(U, dt, wl.dx, p, fluxes=True)
    h = wl.dx[0]
    div = (F[0][:, :, :, 1:] - F[0][:, :, :, :-1]) + (F[1][:, :, 1:, :] - F[1][:, :, :-1, :]) \
        + (F[2][:, 1:, :, :] - F[2][:, :-1, :, :])
    np.testing.assert_allclose(interior(A), interior(U) - dt / h * div, rtol=0, atol=1e-13)


def test_counted_step_follows_the_same_path():
    wl = _random_state(8, 51)
    U = _filled(wl)[0]
    p = O.params(gamma=1.4)
    A, _, _ = O.step(U, 0.01, wl.dx, p)
    B, counts, _ = O.step_count(U, 0.01, wl.dx, p)
    assert np.array_equal(A, B)
    assert counts[O.STAGES.index("riemann1")].sum() > 0


def test_fp32_reconstruction_close_to_fp64():
    wl = I.cfg1(16)
    o64, _, _, _ = oracle_level(O, wl, 2)
    wl.precision = 1
    o32, _, _, _ = oracle_level(O, wl, 2)
    err = field_errors(interior(o32[0]), interior(o64[0]))
    assert err.max() < 1e-5 and err.max() > 0


# ------------------------------------------------------------------ P12 ----
@pytest.mark.parametrize("limiter", [0])
def test_jvp_matches_central_differences(limiter):
    """Forward-mode tangent of one step vs central differences (dt frozen).
    With limiter = 0 the step is a smooth function of the state.  (With the
    limiter on, the CW84 clip at every smooth extremum and the min() of the MC
    slope are kinks that a 1e-6 perturbation crosses, so central differences
    differ from the frozen-branch derivative there.)"""
    wl = I.cfg4(8, amp=0.05)
    U = _filled(wl)[0]
    p = O.params(gamma=1.4, limiter=limiter)
    rng = np.random.default_rng(9)
    v = np.zeros_like(U)
    interior(v)[:] = rng.normal(size=interior(v).shape)
    lay = wl.layout
    vv = [v]
    O.fill(lay.boxes(), lay.domain(), lay.bc, vv)
    dt = 0.02
    A, J, _ = O.step_jvp(U, vv[0], dt, wl.dx, p)
    A0, _, _ = O.step(U, dt, wl.dx, p)
    assert np.array_equal(interior(A), interior(A0))
    eps = 1e-6
    Up, _, _ = O.step(U + eps * vv[0], dt, wl.dx, p)
    Um, _, _ = O.step(U - eps * vv[0], dt, wl.dx, p)
    fd = (interior(Up) - interior(Um)) / (2 * eps)
    err = np.abs(fd - interior(J)).max() / np.abs(interior(J)).max()
    assert err < 1e-6, err


def test_fp32_jvp_primal_is_the_fp32_step_and_tangent_its_derivative():
    """FP32-reconstruction tangent (float primal, double tangent): its primal
    is the FP32 step bit for bit (so every branch is the FP32 step's own), and
    its tangent is that step's derivative: central differences of the FP32
    step on the smooth unlimited step with a bulk flow (no characteristic
    speed near zero), eps = 3e-3 (float rounding of the quotient and the
    truncation error both near 1e-5); it also equals the FP64 tangent to
    float accuracy there (observed 1.1e-7)."""
    wl = I.cfg4(8, amp=0.05, bulk=(0.3, 0.2, 0.25))
    U = _filled(wl)[0]
    p32 = O.params(gamma=1.4, limiter=0, precision=1)
    p64 = O.params(gamma=1.4, limiter=0)
    rng = np.random.default_rng(19)
    v = np.zeros_like(U)
    interior(v)[:] = rng.normal(size=interior(v).shape)
    lay = wl.layout
    vv = [v]
    O.fill(lay.boxes(), lay.domain(), lay.bc, vv)
    dt = 0.02
    A, J, _ = O.step_jvp(U, vv[0], dt, wl.dx, p32)
    A0, _, _ = O.step(U, dt, wl.dx, p32)
    assert np.array_equal(interior(A), interior(A0))
    eps = 3e-3
    Up, _, _ = O.step(U + eps * vv[0], dt, wl.dx, p32)
    Um, _, _ = O.step(U - eps * vv[0], dt, wl.dx, p32)
    fd = (interior(Up) - interior(Um)) / (2 * eps)
    scale = np.abs(interior(J)).max()
    assert np.abs(fd - interior(J)).max() / scale < 1e-4
    _, J64, _ = O.step_jvp(U, vv[0], dt, wl.dx, p64)
    assert np.abs(interior(J64) - interior(J)).max() / scale < 1e-6


# ------------------------------------------------------ reflecting walls ----
def test_no_flow_through_reflecting_walls():
    """Faces on a reflecting wall carry no mass, no energy and no tangential
    momentum — exactly (the mirror state makes the solve land on u* = 0) —
    also with gravity, whose shift of the traced velocities is not mirror
    symmetric; the normal momentum flux is the wall pressure, positive."""
    wl = I.cfg5(2, 8, precision=0)
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    p = O.params(gamma=wl.gamma, grav=wl.grav)
    nchecked = 0
    for b in range(lay.nbox):
        walls = O.box_walls(lay.boxes(), lay.domain(), lay.bc, b)
        _, F, _ = O.step(st[b], 1e-3, wl.dx, p, fluxes=True, walls=walls)
        for side, k in ((0, 0), (1, -1)):
            if not walls[4 + side]:
                continue
            f = F[2][:, k]  # z-faces of the wall plane
            assert np.all(f[0] == 0) and np.all(f[1] == 0) and np.all(f[2] == 0) and np.all(f[4] == 0)
            assert np.all(f[3] > 0)
            nchecked += 1
    assert nchecked == 8


def test_walls_and_gravity_conserve_mass_and_transverse_momentum():
    """Rayleigh-Taylor set-up on 2x2x2 boxes, 3 steps: mass and the x, y
    momenta (gravity and the walls act along z only) are conserved to
    round-off (scale: the total mass times the sound speed, about 1)."""
    wl = I.cfg5(2, 8, precision=0)
    lay = wl.layout
    out, _, fl, _ = oracle_level(O, wl, 3)
    assert fl == 0
    mass = math.fsum(np.concatenate([interior(lay.view(wl.arena, b))[0].ravel() for b in range(lay.nbox)]))
    for c in range(3):
        s0 = math.fsum(np.concatenate([interior(lay.view(wl.arena, b))[c].ravel() for b in range(lay.nbox)]))
        s1 = math.fsum(np.concatenate([interior(out[b])[c].ravel() for b in range(lay.nbox)]))
        assert abs(s1 - s0) <= 1e-14 * mass, (c, s1 - s0)


def test_power_of_two_change_of_units_commutes_with_the_step():
    """Euler's equations carry no scale of their own: density times R and
    pressure times P (velocity times sqrt(P/R), time divided by it, lengths
    kept) maps solutions to solutions.  With R, P powers of two every
    floating-point operation of the FP64 step scales exactly, so the run in
    the new units is the scaled run in the old ones bit for bit, dt
    included.  A term that mixes dimensions (a constant added to a
    pressure, an absolute tolerance) breaks it."""
    wl = I.cfg2(16)
    wl.grav = (0.3, -0.2, 0.1)
    ws, sc, V = rescaled(wl)
    assert np.nanmax(np.abs(ws.arena)) > 1e21
    out, dts, fl, _ = oracle_level(O, wl, 3)
    outs, dtss, fls, _ = oracle_level(O, ws, 3)
    assert fl == fls == 0
    assert dtss == [d / V for d in dts]
    for b in range(wl.layout.nbox):
        assert np.array_equal(outs[b], out[b] * sc), b

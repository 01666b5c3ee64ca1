"""Pins of the oracle's building blocks against facts the mathematics fixes:
exact Riemann solutions, eigen-structure of the Euler equations, exact
polynomial reconstruction, closed-form index maps.  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import exact_riemann as X

HERE = os.path.dirname(os.path.abspath(__file__))


def euler_flux(q, d, g):
    """Flux of the 3-D Euler equations along d for primitive q = (rho, u, v, w, p)."""
    rho, p = q[0], q[4]
    v = np.array(q[1:4])
    E = p / (g - 1.0) + 0.5 * rho * (v @ v)
    F = np.zeros(5)
    F[0] = rho * v[d]
    F[1:4] = rho * v[d] * v
    F[1 + d] += p
    F[4] = v[d] * (E + p)
    return F


# ------------------------------------------------------------ exact solver --
def test_exact_solver_sod_matches_printed_values():
    vals = np.loadtxt(os.path.join(HERE, "golden", "sod_star.txt"))
    L, R, g = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4
    ps, us = X.star(L, R, g)
    rl = X.sample(L, R, g, us - 1e-9)[0]
    rr = X.sample(L, R, g, us + 1e-9)[0]
    assert abs(ps - vals[0]) < 5e-6
    assert abs(us - vals[1]) < 5e-6
    assert abs(rl - vals[2]) < 5e-6
    assert abs(rr - vals[3]) < 5e-6


@pytest.mark.parametrize("case", [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4),
    ((1.0, 2.0, 1.0), (0.5, -1.0, 0.3), 5.0 / 3.0),
    ((0.4, -0.5, 0.2), (1.5, 0.8, 2.0), 1.4),
])
def test_exact_solver_jump_conditions(case):
    """Rankine-Hugoniot across each shock; isentropy and the Riemann invariant
    across each rarefaction; continuity of p and u at the contact."""
    L, R, g = case
    ps, us = X.star(L, R, g)
    sl, sr = X.shock_speeds(L, R, g)
    for side, (st, S) in (("L", (L, sl)), ("R", (R, sr))):
        rk, uk, pk = st
        if S is not None:
            eps = 1e-9
            a = X.sample(L, R, g, S - eps) if side == "L" else X.sample(L, R, g, S + eps)
            b = X.sample(L, R, g, S + eps) if side == "L" else X.sample(L, R, g, S - eps)

            def cons_flux(q):
                r, u, p = q
                E = p / (g - 1) + 0.5 * r * u * u
                return np.array([r, r * u, E]), np.array([r * u, r * u * u + p, u * (E + p)])
            Ua, Fa = cons_flux(a)
            Ub, Fb = cons_flux(b)
            np.testing.assert_allclose(Fb - Fa, S * (Ub - Ua), rtol=0, atol=1e-10)
        else:
            # rarefaction: entropy p/rho^g and u +/- 2c/(g-1) constant through the fan
            star_r = X.sample(L, R, g, us - 1e-9 if side == "L" else us + 1e-9)[0]
            assert abs(ps / star_r ** g - pk / rk ** g) < 1e-12 * pk / rk ** g
            sgn = 1.0 if side == "L" else -1.0
            inv0 = uk + sgn * 2 * math.sqrt(g * pk / rk) / (g - 1)
            inv1 = us + sgn * 2 * math.sqrt(g * ps / star_r) / (g - 1)
            assert abs(inv0 - inv1) < 1e-12


# ---------------------------------------------------------- O6: Riemann ----
@pytest.mark.parametrize("d", [0, 1, 2])
def test_riemann_equal_states_give_physical_flux(d):
    rng = np.random.default_rng(10 + d)
    for _ in range(50):
        q = np.array([rng.uniform(0.2, 3), *rng.uniform(-2, 2, 3), rng.uniform(0.1, 4)])
        g = rng.choice([1.4, 5.0 / 3.0])
        p = O.params(gamma=g)
        F, fl = O.riemann(q, q, d, p)
        assert fl == 0
        np.testing.assert_allclose(F, euler_flux(q, d, g), rtol=1e-13,
                                   atol=1e-14 * np.abs(euler_flux(q, d, g)).max())


@pytest.mark.parametrize("L,R", [
    ((1.0, 2.0, 0.0, 0.0, 1.0), (1.0, -2.0, 0.0, 0.0, 1.0)),
    ((1.2, 1.5, 0.3, -0.2, 0.8), (0.7, -0.9, -0.4, 0.6, 1.3)),
    ((0.5, 0.3, 0.1, 0.2, 2.0), (2.0, -1.7, 0.0, 0.9, 0.4)),
])
def test_two_shock_collision_equals_exact_solution(L, R):
    """When both nonlinear waves are shocks the two-shock curves are exact; the
    iteration converges to the exact star state, and the Godunov flux is the
    exact one (sampled at x/t = 0)."""
    g = 1.4
    L, R = np.array(L), np.array(R)
    ps, us = X.star((L[0], L[1], L[4]), (R[0], R[1], R[4]), g)
    assert ps > L[4] and ps > R[4]
    r, u, pp = X.sample((L[0], L[1], L[4]), (R[0], R[1], R[4]), g, 0.0)
    side = L if us > 0 else R
    q = np.array([r, u, side[2], side[3], pp])
    for it in (8, 12):
        F, fl = O.riemann(L, R, 0, O.params(gamma=g, riemann_iters=it))
        np.testing.assert_allclose(F, euler_flux(q, 0, g), rtol=1e-12, atol=1e-12)
    # the default 3 iterations already land within 1e-4 of the exact flux
    F3, _ = O.riemann(L, R, 0, O.params(gamma=g))
    np.testing.assert_allclose(F3, euler_flux(q, 0, g), rtol=1e-4, atol=1e-6)


def test_riemann_newton_residual_decreases():
    g = 1.4
    L = np.array([1.0, 1.0, 0.0, 0.0, 1.0])
    R = np.array([0.6, -1.2, 0.0, 0.0, 0.7])
    ps, us = X.star((1.0, 1.0, 1.0), (0.6, -1.2, 0.7), g)
    errs = []
    for it in range(0, 6):
        F, _ = O.riemann(L, R, 0, O.params(gamma=g, riemann_iters=it))
        errs.append(abs(F[1] - F[0] * us - ps))  # momentum flux minus rho u* u* = p*
    assert errs[5] < 1e-10 and errs[3] < errs[1] < errs[0] + 1e-30


@pytest.mark.parametrize("d", [0, 1, 2])
def test_riemann_mirror_symmetry_bitwise(d):
    """Swapping sides and reversing the normal velocity reverses the odd flux
    components and keeps the even ones, bit for bit."""
    rng = np.random.default_rng(20 + d)
    p = O.params(gamma=1.4)
    for _ in range(200):
        L = np.array([rng.uniform(0.1, 3), *rng.uniform(-3, 3, 3), rng.uniform(0.05, 4)])
        R = np.array([rng.uniform(0.1, 3), *rng.uniform(-3, 3, 3), rng.uniform(0.05, 4)])
        F, _ = O.riemann(L, R, d, p)
        Lm, Rm = R.copy(), L.copy()
        Lm[1 + d] = -Lm[1 + d]
        Rm[1 + d] = -Rm[1 + d]
        Fm, _ = O.riemann(Lm, Rm, d, p)
        sgn = -np.ones(5)
        sgn[1 + d] = 1.0
        assert np.array_equal(Fm, sgn * F)


def test_riemann_sod_two_shock_approximation_close():
    """On Sod data (rarefaction + shock, pressure ratio 10) the two-shock
    approximation is not exact; its mass flux lies within 6 percent."""
    g = 1.4
    L = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
    R = np.array([0.125, 0.0, 0.0, 0.0, 0.1])
    F, _ = O.riemann(L, R, 0, O.params(gamma=g, riemann_iters=20))
    ps, us = X.star((1, 0, 1), (0.125, 0, 0.1), g)
    r, u, pp = X.sample((1, 0, 1), (0.125, 0, 0.1), g, 0.0)
    assert abs(F[0] - r * u) < 0.06 * abs(r * u)


# --------------------------------------------------------------- O4: PPM ----
def test_ppm_unlimited_edges_exact_for_cubics():
    """Edge values from cell averages reproduce any cubic exactly."""
    rng = np.random.default_rng(1)
    h = 0.1
    m = 24
    for _ in range(10):
        c = rng.normal(size=4)
        P = np.polynomial.Polynomial(c)
        Pi = P.integ()
        xe = (np.arange(m + 1) - 0.5) * h
        avg = (Pi(xe[1:]) - Pi(xe[:-1])) / h
        aL, aR, a6 = O.ppm_line(avg, O.params(limiter=0))
        i = np.arange(2, m - 2)
        scale = np.abs(avg).max()
        np.testing.assert_allclose(aL[i], P(xe[i]), atol=1e-13 * scale)
        np.testing.assert_allclose(aR[i], P(xe[i + 1]), atol=1e-13 * scale)


def test_ppm_integrals_over_the_cell_give_the_average():
    """I+(1) and I-(1) average the parabola over the whole zone: the zone value."""
    rng = np.random.default_rng(2)
    a = rng.normal(size=40).cumsum()
    for lim in (0, 1):
        aL, aR, a6 = O.ppm_line(a, O.params(limiter=lim))
        for i in range(2, 38):
            ip, im = O.ppm_integrals(aL[i], aR[i], a6[i], 1.0)
            assert abs(ip - a[i]) <= 1e-13 * max(1, abs(a[i]))
            assert abs(im - a[i]) <= 1e-13 * max(1, abs(a[i]))
            ip0, im0 = O.ppm_integrals(aL[i], aR[i], a6[i], 0.0)
            assert ip0 == aR[i] and im0 == aL[i]


def test_ppm_parabola_is_the_quadratic_through_edges_and_mean():
    """a6 makes the zone mean of aL + (aR-aL) x + a6 x (1-x) equal to a_i."""
    rng = np.random.default_rng(3)
    a = rng.uniform(0, 1, 30)
    aL, aR, a6 = O.ppm_line(a, O.params(limiter=1))
    i = np.arange(2, 28)
    mean = aL[i] + 0.5 * (aR[i] - aL[i]) + a6[i] / 6.0
    np.testing.assert_allclose(mean, a[i], atol=1e-14)


def test_ppm_limited_monotone_data_gives_monotone_parabolas():
    rng = np.random.default_rng(4)
    for _ in range(20):
        a = np.cumsum(rng.exponential(1.0, 40)) * rng.choice([-1, 1])
        aL, aR, a6 = O.ppm_line(a, O.params(limiter=1))
        for i in range(2, 38):
            lo, hi = sorted((a[i - 1], a[i + 1]))
            assert lo - 1e-12 <= aL[i] <= hi + 1e-12 and lo - 1e-12 <= aR[i] <= hi + 1e-12
            # a parabola aL + da x + a6 x(1-x) is monotone on [0,1] iff |a6| <= |da|
            assert abs(a6[i]) <= abs(aR[i] - aL[i]) + 1e-14 * abs(a[i])


def test_ppm_limited_flat_at_extrema_and_flattening_blend():
    a = np.array([0.0, 1.0, 2.0, 5.0, 2.0, 1.0, 0.0])
    aL, aR, a6 = O.ppm_line(a, O.params(limiter=1))
    assert aL[3] == 5.0 and aR[3] == 5.0 and a6[3] == 0.0
    # full flattening (phi = 0) reduces every zone to a constant
    b = np.array([0.0, 0.5, 1.5, 2.0, 3.5, 4.0, 4.1, 6.0])
    aL, aR, a6 = O.ppm_line(b, O.params(limiter=1), phi=np.zeros(8))
    i = np.arange(2, 6)
    assert np.array_equal(aL[i], b[i]) and np.array_equal(aR[i], b[i]) and np.all(a6[i] == 0)


# ------------------------------------------------------------ O5: tracing --
def _wave_parabolas(q, r, amp_l, amp_r, amp_6):
    """Parabolas whose variation lies along the primitive vector r."""
    q = np.asarray(q, dtype=np.float64)
    aL = q[:5] + amp_l * r
    aR = q[:5] + amp_r * r
    a6 = amp_6 * r
    return aL, aR, a6


def _eigvecs(q, d):
    rho, p = q[0], q[4]
    c = math.sqrt(1.4 * p / rho)
    r1 = np.zeros(5); r1[0] = 1; r1[1 + d] = -c / rho; r1[4] = c * c
    r2 = np.zeros(5); r2[0] = 1
    r3 = np.zeros(5); r3[0] = 1; r3[1 + d] = c / rho; r3[4] = c * c
    return c, r1, r2, r3


@pytest.mark.parametrize("d", [0, 1, 2])
def test_trace_constant_parabolas_give_cell_state(d):
    q = np.array([1.3, 0.2, -0.4, 0.1, 0.9])
    c = math.sqrt(1.4 * q[4] / q[0])
    cell = np.append(q, c)
    qp, qm, _ = O.trace(q, q, np.zeros(5), cell, d, 0.3, O.params())
    assert np.array_equal(qp, q) and np.array_equal(qm, q)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_trace_pure_acoustic_wave_keeps_its_own_characteristic(d):
    """Subsonic flow, data along r3 only: at the high face the reference state
    I+(sigma3) is already the answer (waves 1 and 2 carry nothing of r3)."""
    q = np.array([1.1, 0.15, -0.3, 0.25, 0.8])
    q[1 + d] = 0.2
    c, r1, r2, r3 = _eigvecs(q, d)
    cell = np.append(q, c)
    aL, aR, a6 = _wave_parabolas(q, r3, -0.01, 0.02, 0.004)
    dtdx = 0.4
    qp, qm, _ = O.trace(aL, aR, a6, cell, d, dtdx, O.params())
    s3 = (q[1 + d] + c) * dtdx
    expect = np.array([O.ppm_integrals(aL[m], aR[m], a6[m], s3)[0] for m in range(5)])
    np.testing.assert_allclose(qp, expect, rtol=0, atol=1e-14)
    # at the low face only wave 1 arrives and the data carry none of it: the
    # reference I-(sigma1) is the answer
    s1 = (c - q[1 + d]) * dtdx
    expect = np.array([O.ppm_integrals(aL[m], aR[m], a6[m], s1)[1] for m in range(5)])
    np.testing.assert_allclose(qm, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_trace_supersonic_slow_wave_removed_from_reference(d):
    """Supersonic flow to the high side (all lambdas > 0), data along r1: the
    high-face state is the average swept by wave 1, I+(sigma1); the entropy
    and shear waves see no r1 content."""
    q = np.array([0.9, 0.0, 0.05, -0.1, 0.6])
    c, r1, r2, r3 = _eigvecs(q, d)
    q[1 + d] = 1.8 * c
    c, r1, r2, r3 = _eigvecs(q, d)
    cell = np.append(q, c)
    aL, aR, a6 = _wave_parabolas(q, r1, 0.02, -0.015, 0.006)
    dtdx = 0.2
    qp, qm, _ = O.trace(aL, aR, a6, cell, d, dtdx, O.params())
    s1 = (q[1 + d] - c) * dtdx
    expect = np.array([O.ppm_integrals(aL[m], aR[m], a6[m], s1)[0] for m in range(5)])
    np.testing.assert_allclose(qp, expect, rtol=0, atol=2e-14)
    # nothing reaches the low face: its state is the low edge value
    np.testing.assert_array_equal(qm, aL)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_trace_entropy_and_shear_waves(d):
    """Supersonic flow; density and a transverse velocity vary, p and u_n do
    not: the high face takes I+(sigma2) of those fields, the rest stays."""
    q = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
    c = math.sqrt(1.4)
    q[1 + d] = 1.5 * c
    cell = np.append(q, c)
    t1 = 1 + (1 if d == 0 else 0)
    r = np.zeros(5); r[0] = 1.0; r[t1] = 0.5
    aL, aR, a6 = _wave_parabolas(q, r, -0.03, 0.05, 0.01)
    dtdx = 0.15
    qp, qm, _ = O.trace(aL, aR, a6, cell, d, dtdx, O.params())
    s2 = q[1 + d] * dtdx
    for m in range(5):
        e = O.ppm_integrals(aL[m], aR[m], a6[m], s2)[0]
        assert abs(qp[m] - e) <= 1e-14

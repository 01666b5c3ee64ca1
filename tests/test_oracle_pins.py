"""Pins of oracle parts that the invariants and exact solutions do not reach:
the shock-flattening coefficient (O3) on designed pressure and velocity
profiles, the CFL signal speed (O11) on a hand-made state of an anisotropic
grid, and the operation counts of one Riemann solve and one state
conversion (the counts the roofline's algorithmic flops come from).

Every expected value below is worked out by hand from the definitions in
the comments next to it; all inputs are dyadic and gamma = 2 (gamma - 1 = 1),
so the oracle's arithmetic on them is exact and the comparisons are exact.

Flattening (Colella-Woodward 1984 appendix, eps 0.33, omega1 0.75, omega2
10), per axis at zone i:
  dp1 = p[i+1] - p[i-1], dp2 = p[i+2] - p[i-2], zeta = |dp1| / |dp2|,
  chi~_i = min(max(10 (zeta - 0.75), 0), 1) if u[i-1] - u[i+1] > 0 and
           |dp1| > 0.33 min(p[i+1], p[i-1]), else 0,
  chi_i = max(chi~_i, chi~ of the lower-pressure neighbour) (both
          neighbours when dp1 = 0),
  phi_i = min over axes of (1 - chi_i).
"""
import numpy as np
import pytest

from oracle import oracle as O

NG = 4
GAMMA = 2.0


def _box(n, rho, u, p):
    """Conserved state of one box (5, nz+8, ny+8, nx+8) from primitive
    arrays over the stored grid (each of shape (nz+8, ny+8, nx+8))."""
    U = np.zeros((5,) + rho.shape)
    U[0] = rho
    for d in range(3):
        U[1 + d] = rho * u[d]
    U[4] = p / (GAMMA - 1.0) + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    return U


def _line_box(px, ux):
    """A box of valid extents (len(px) - 8, 1, 1) whose pressure and
    x-velocity vary along x only (rho = 1)."""
    nx = len(px) - 2 * NG
    shape = (1 + 2 * NG, 1 + 2 * NG, len(px))
    rho = np.ones(shape)
    p = np.broadcast_to(np.asarray(px, dtype=float), shape).copy()
    u = [np.broadcast_to(np.asarray(ux, dtype=float), shape).copy(), np.zeros(shape), np.zeros(shape)]
    return _box((nx, 1, 1), rho, u, p)


def _phi_x(px, ux, i):
    """phi at valid zone i of a line profile."""
    phi, fl = O.flatten(_line_box(px, ux), O.params(gamma=GAMMA))
    assert fl == 0
    return phi[1, 1, i + 1]


# Stored index s = i + 4 of valid zone i; the line has 12 valid zones and the
# profiles below are built around valid zone I0 = 6 (stored index 10).
I0 = 6
S0 = I0 + NG
NS = 12 + 2 * NG


def _profile(vals, left, right):
    """Pressure along the line: vals[k] at stored index S0 - 3 + k (k = 0..6,
    zones i0-3 .. i0+3), `left` before, `right` after."""
    p = np.full(NS, float(right))
    p[:S0 - 3] = left
    p[S0 - 3:S0 + 4] = vals
    return p


# x-velocity decreasing by 1/16 per zone: u[i-1] - u[i+1] = 1/8 > 0
# (compression) at every zone.
U_COMP = -0.0625 * (np.arange(NS) - S0)
U_EXP = -U_COMP


def _ramp(dp1):
    """Zones i0-3 .. i0+3: 1, 1, 1.125, 1.5, 1.125 + dp1, 2, 2.  At i0:
    dp1 as given, dp2 = 2 - 1 = 1, so zeta = dp1.  At i0 - 1: dp1 = 1.5 - 1
    = 0.5, dp2 = (1.125 + dp1) - 1 <= 1 with zeta < 0.75 for dp1 > 0.55, so
    chi~ = 0 there; dp1 > 0 at i0, so chi = chi~_i0."""
    return _profile([1.0, 1.0, 1.125, 1.5, 1.125 + dp1, 2.0, 2.0], 1.0, 2.0)


@pytest.mark.parametrize("dp1,phi", [
    (0.734375, 1.0),      # zeta = 0.75 - 1/64: z = 0
    (0.765625, 0.84375),  # zeta = 0.75 + 1/64: z = 10/64 = 0.15625
    (0.84375, 0.0625),    # zeta = 0.75 + 3/32: z = 0.9375
    (0.859375, 0.0),      # zeta = 0.75 + 7/64: 10 (zeta - 0.75) = 1.09375 -> 1
])
def test_flattening_coefficient_at_the_zeta_thresholds(dp1, phi):
    # strong: dp1 > 0.33 min(1.125 + dp1, 1.125) = 0.37125 in every case
    assert _phi_x(_ramp(dp1), U_COMP, I0) == phi


def test_flattening_needs_compression():
    # the same ramp as zeta = 0.765625 in an expansion (u[i-1] - u[i+1] < 0)
    assert _phi_x(_ramp(0.765625), U_EXP, I0) == 1.0


@pytest.mark.parametrize("offset,phi", [
    (1.0, 0.84375),   # min(p[i+1], p[i-1]) = 2.125: 0.33 * 2.125 = 0.70125 < 0.765625, strong
    (1.25, 1.0),      # min = 2.375: 0.33 * 2.375 = 0.78375 > 0.765625, not strong
])
def test_flattening_strength_test(offset, phi):
    # a constant offset leaves dp1, dp2 and zeta unchanged
    assert _phi_x(_ramp(0.765625) + offset, U_COMP, I0) == phi


def test_flattening_takes_the_lower_pressure_neighbour():
    """Zones i0-3 .. i0+4: 1, 1, 1, 1, 1.0625, 2, 2, 2.
    i0:   dp1 = 1.0625 - 1 = 1/16 > 0, dp2 = 2 - 1 = 1: zeta = 1/16, chi~ = 0;
    i0+1: dp1 = 2 - 1 = 1, dp2 = 2 - 1 = 1: zeta = 1, strong (1 > 0.33):
          chi~ = 1;
    i0-1: dp1 = 1 - 1 = 0: chi~ = 0.
    dp1 > 0 at i0, so the lower-pressure neighbour is i0 - 1: chi = 0,
    phi = 1 (the higher-pressure neighbour would give phi = 0).  At i0+1
    and i0+2 chi = 1, phi = 0.  The mirror image (p reversed, u reversed
    and negated, still a compression) takes the dp1 < 0 branch: the same
    values at the mirrored zones."""
    px = _profile([1.0, 1.0, 1.0, 1.0, 1.0625, 2.0, 2.0], 1.0, 2.0)
    phi, fl = O.flatten(_line_box(px, U_COMP), O.params(gamma=GAMMA))
    assert fl == 0
    assert phi[1, 1, I0 + 1] == 1.0
    assert phi[1, 1, I0 + 2] == 0.0 and phi[1, 1, I0 + 3] == 0.0
    phim, fl = O.flatten(_line_box(px[::-1].copy(), -U_COMP[::-1]), O.params(gamma=GAMMA))
    assert fl == 0
    # valid zone i <-> 11 - i; traced slot i + 1 <-> 12 - i
    assert phim[1, 1, 12 - I0] == 1.0
    assert phim[1, 1, 12 - (I0 + 1)] == 0.0 and phim[1, 1, 12 - (I0 + 2)] == 0.0


def test_flattening_tie_takes_both_neighbours():
    """Zones i0-3 .. i0+3: 1, 1, 1, 1, 1, 2, 2: dp1 = p[i0+1] - p[i0-1] = 0
    at i0 (chi~ = 0, zeta = 0); i0+1: dp1 = 2 - 1 = 1, dp2 = 2 - 1 = 1,
    chi~ = 1; i0-1: chi~ = 0.  The tie takes max(chi~_{i0-1}, chi~_i0,
    chi~_{i0+1}) = 1: phi = 0 (the left neighbour alone would give 1)."""
    px = _profile([1.0, 1.0, 1.0, 1.0, 1.0, 2.0, 2.0], 1.0, 2.0)
    assert _phi_x(px, U_COMP, I0) == 0.0


def test_flattening_is_the_minimum_over_axes():
    """p(i, j) = P(i) + Q(j) + 1/8 on a 12 x 12 x 1 box, u_x = U_COMP(i),
    u_y = U_COMP(j).  P: the zeta = 0.765625 ramp minus 1 along x (chi_x =
    0.15625 at i0); Q: the zeta = 0.84375 ramp minus 1 along y (chi_y =
    0.9375 at j0 = i0).  At (i0, i0): along x min(p[i+1], p[i-1]) =
    0.125 + 0.5 + 0.125 = 0.75, 0.33 * 0.75 < 0.765625 (strong); along y
    likewise 0.75 (strong).  phi = min(0.84375, 0.0625) = 0.0625."""
    P = _ramp(0.765625) - 1.0
    Q = _ramp(0.84375) - 1.0
    shape = (1 + 2 * NG, NS, NS)
    p = np.broadcast_to(P[None, None, :], shape) + np.broadcast_to(Q[None, :, None], shape) + 0.125
    ux = np.broadcast_to(U_COMP[None, None, :], shape).copy()
    uy = np.broadcast_to(U_COMP[None, :, None], shape).copy()
    U = _box((12, 12, 1), np.ones(shape), [ux, uy, np.zeros(shape)], p.copy())
    phi, fl = O.flatten(U, O.params(gamma=GAMMA))
    assert fl == 0
    assert phi[1, I0 + 1, I0 + 1] == 0.0625
    # along x alone at (i0, j far from the y ramp): 1 - 0.15625
    assert phi[1, 1, I0 + 1] == 0.84375


def test_flattening_off_gives_one():
    phi, _ = O.flatten(_line_box(_ramp(0.859375), U_COMP), O.params(gamma=GAMMA, flattening=0))
    assert np.all(phi == 1.0)


# ---------------------------------------------------------------- O11 -----
def _speed_box(extra=()):
    """Box of valid extents (3, 2, 2), rho = 1, p = 2 (c = sqrt(2 * 2 / 1) =
    2), u = 0, with `extra` = [(stored index (s_z, s_y, s_x), rho, u, p)]
    overrides."""
    shape = (2 + 2 * NG, 2 + 2 * NG, 3 + 2 * NG)
    rho, p = np.ones(shape), np.full(shape, 2.0)
    u = [np.zeros(shape), np.zeros(shape), np.zeros(shape)]
    for idx, r, vel, pr in extra:
        rho[idx] = r
        p[idx] = pr
        for d in range(3):
            u[d][idx] = vel[d]
    return _box((3, 2, 2), rho, u, p)


H = (0.5, 0.25, 0.125)


@pytest.mark.parametrize("extra,s", [
    # at rest: max over axes of c / h_d = 2 / 0.125
    ((), 16.0),
    # zone (0, 1, 1): u_x = -7.5: (|-7.5| + 2) / 0.5 = 19; zone (2, 0, 1):
    # v = 2.5: (2.5 + 2) / 0.25 = 18; a ghost zone with u_x = 100 is not a
    # valid zone.  (|u| over all components with the smallest h would give
    # 76; u_x without the absolute value 18; the ghost 204.)
    ((((1 + NG, 1 + NG, 0 + NG), 1.0, (-7.5, 0.0, 0.0), 2.0),
      ((1 + NG, 0 + NG, 2 + NG), 1.0, (0.0, 2.5, 0.0), 2.0),
      ((1 + NG, 1 + NG, NG - 1), 1.0, (100.0, 0.0, 0.0), 2.0)), 19.0),
    # zone (1, 1, 0): rho = 1/4, p = 1/2, w = -1: c = sqrt(2 * 0.5 / 0.25) =
    # 2, (1 + 2) / 0.125 = 24; zone (2, 1, 1): p = 8, c = 4, 4 / 0.125 = 32
    ((((0 + NG, 1 + NG, 1 + NG), 0.25, (0.0, 0.0, -1.0), 0.5),
      ((1 + NG, 1 + NG, 2 + NG), 1.0, (0.0, 0.0, 0.0), 8.0)), 32.0),
])
def test_cfl_signal_speed_on_an_anisotropic_grid(extra, s):
    got, fl = O.max_wavespeed(_speed_box(extra), H, O.params(gamma=GAMMA))
    assert fl == 0
    assert got == s


# ---------------------------------------------------- operation counts -----
# One two-shock solve with N Newton iterations, counted from the definition
# (add = add/sub, min/max separately; unary minus and |x| are free):
#   C_L, C_R = sqrt(gamma p rho):          mul 4, sqrt 2
#   acoustic guess ((C_R p_L + C_L p_R) + C_L C_R (u_L - u_R)) / (C_L + C_R):
#                                          mul 4, add 4, div 1; floor: minmax 1
#   per iteration, per side W_s = C_s sqrt(1 + beta (p/p_s - 1)):
#                                          div 1, add 2, mul 2, sqrt 1
#     Z_s = 2 W_s^3 / (W_s^2 + C_s^2):     mul 5, add 1, div 1
#     u*_s = u_s -/+ (p - p_s)/W_s:        add 2, div 1
#     p <- p - Z_L Z_R (u*_R - u*_L)/(Z_L + Z_R): mul 2, add 3, div 1;
#                                          floor: minmax 1
#     -> per iteration div 7, add 13, mul 16, sqrt 2, minmax 1
#   final W_L, W_R:                        div 2, add 4, mul 4, sqrt 2
#   u* = ((W_L u_L + W_R u_R) + (p_L - p_R)) / (W_L + W_R): mul 2, add 4, div 1
#   flux of the Godunov state (m = rho u; e = p/(gamma-1) + rho/2 |u|^2;
#     (m, m u + p, m v, m w, u (e + p))): mul 10, add 5, div 1
#   sampling one side: rho* = 1/(1/rho_s - (p* - p_s)/W_s^2): div 3, add 2,
#     mul 1; c* = sqrt(gamma p*/rho*), c_s = sqrt(gamma p_s/rho_s):
#     mul 2, div 2, sqrt 2; then
#       shock, S = u_s -/+ W_s/rho_s:      add 1, div 1
#       fan, w = -H/(T - H) and three blends (1 - w) a + w b:
#         H, T: add 2; w: add 1, div 1; blends: add 6, mul 6
# Totals with N = 3:
#   shock side: div 5 + 21 + 6 = 32, add 17 + 39 + 3 = 59,
#               mul 24 + 48 + 3 = 75, sqrt 4 + 6 + 2 = 12, minmax 4
#   fan side:   div 32, add 17 + 39 + 11 = 67, mul 24 + 48 + 9 = 81,
#               sqrt 12, minmax 4
# and with N = 0 (shock side): div 5 + 6 = 11, add 20, mul 27, sqrt 6, minmax 1.
@pytest.mark.parametrize("L,R,iters,want", [
    # colliding streams (both waves shocks; u* > 0, left side sampled)
    ((1.0, 2.0, 0.0, 0.0, 1.0), (1.0, -1.0, 0.0, 0.0, 1.0), 3,
     {"div": 32, "add": 59, "mul": 75, "sqrt": 12, "minmax": 4}),
    ((1.0, 2.0, 0.0, 0.0, 1.0), (1.0, -1.0, 0.0, 0.0, 1.0), 0,
     {"div": 11, "add": 20, "mul": 27, "sqrt": 6, "minmax": 1}),
    # Toro's first test (sonic left rarefaction): the fan at x/t = 0
    ((1.0, 0.75, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.0, 0.1), 3,
     {"div": 32, "add": 67, "mul": 81, "sqrt": 12, "minmax": 4}),
])
def test_riemann_solve_operation_count(L, R, iters, want):
    _, got, fl = O.count_ops("riemann", list(L) + list(R), O.params(gamma=1.4, riemann_iters=iters))
    assert fl == 0
    assert got == want


def test_state_conversion_operation_count():
    """Primitive -> conserved (rho u_d: mul 3; p/(gamma-1) + rho/2 |u|^2:
    div 1, mul 5, add 3) -> primitive with floors (rho floor: minmax 1;
    u_d = (rho u_d)/rho: div 3; rho/2 |u|^2: mul 5, add 2;
    p = (gamma-1)(rho E - ke): mul 1, add 1; p floor: minmax 1)."""
    q = (1.0, 0.3, 0.2, 0.1, 1.0)
    out, got, fl = O.count_ops("conversion", q, O.params(gamma=1.4))
    assert fl == 0
    assert got == {"div": 4, "add": 6, "mul": 14, "sqrt": 0, "minmax": 2}
    assert np.allclose(out, q, rtol=1e-15, atol=0)


def test_flux_output_tangent_matches_central_differences():
    """The tangents of the step's flux outputs (the dual-number evaluation
    with flux output) against central differences of the plain step's
    fluxes on smooth data with the unlimited scheme (no kinks)."""
    from paper_1008_2801_amd import inputs as I
    wl = I.cfg4(10, amp=0.05, bulk=(0.3, 0.2, 0.25))
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    dv = [np.random.default_rng(0).normal(size=st[0].shape)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, dv)
    p = O.params(gamma=wl.gamma, limiter=0)
    U1, _, F, dF, fl = O.step_jvp_flux(st[0], dv[0], 1e-3, wl.dx, p)
    U2, F2, _ = O.step(st[0], 1e-3, wl.dx, p, fluxes=True)
    assert fl == 0 and np.array_equal(U1, U2)
    eps = 1e-6
    _, Fp, _ = O.step(st[0] + eps * dv[0], 1e-3, wl.dx, p, fluxes=True)
    _, Fm, _ = O.step(st[0] - eps * dv[0], 1e-3, wl.dx, p, fluxes=True)
    for d in range(3):
        assert np.array_equal(F[d], F2[d])
        err = np.abs((Fp[d] - Fm[d]) / (2 * eps) - dF[d]).max() / np.abs(dF[d]).max()
        assert err < 1e-8, (d, err)

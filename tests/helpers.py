"""Shared helpers of the test suite (inputs and comparisons only)."""
import copy
import math

import numpy as np

NG = 4


def interior(U):
    g = NG
    return U[:, g:-g, g:-g, g:-g]


def oracle_level(O, wl, nsteps, dt=None, fluxes=False, **pk):
    """Run the oracle on a Workload for nsteps; returns (states, dts, flags, F)."""
    lay = wl.layout
    states = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    p = O.params(gamma=wl.gamma, grav=wl.grav, precision=wl.precision, **pk)
    return O.advance(lay.boxes(), lay.domain(), lay.bc, states, nsteps, wl.dx, p, dt=dt, fluxes=fluxes)


def field_errors(A, B):
    """Per-field max |A - B| / max |B| over valid zones (fields with max |B| = 0
    are normalised by max |rho E| instead)."""
    e = []
    scale4 = np.abs(B[4]).max()
    for c in range(A.shape[0]):
        s = np.abs(B[c]).max()
        e.append(np.abs(A[c] - B[c]).max() / (s if s > 0 else scale4))
    return np.array(e)


# Density and pressure factors of a change of units (velocity: their ratio's
# square root, 2^26; lengths unchanged).  Powers of two, so that every
# floating-point operation of a dimensionally consistent step scales exactly.
# They take unit-scale states to rho ~ 1e6 and p ~ 5e21, the magnitudes of a
# white dwarf's outer layers in cgs units.
UNIT_R, UNIT_P = 2.0 ** 20, 2.0 ** 72


def rescaled(wl, R=UNIT_R, P=UNIT_P):
    """A copy of a Workload in units where density is R times and pressure P
    times larger: momentum scales by R V, energy by P, gravity by V^2 (V =
    sqrt(P / R)).  Returns (workload, per-field factors, V)."""
    V = math.sqrt(P / R)
    w = copy.deepcopy(wl)
    sc = np.array([R, R * V, R * V, R * V, P])
    for b in range(w.layout.nbox):
        w.layout.view(w.arena, b)[...] *= sc[:, None, None, None]
    w.grav = tuple(g * V * V for g in wl.grav)
    return w, sc[:, None, None, None], V


def dts_close(got, ref, rtol=1e-12):
    """Time-step sequences equal to rtol (the first step's dt is computed
    from the same state on both sides; later ones from states that agree
    to rounding)."""
    return len(got) == len(ref) and all(abs(a - b) <= rtol * abs(b) for a, b in zip(got, ref))


def parity_report(tag, pairs, tol, state=None):
    """Per-field parity of GPU arrays against reference arrays: pairs is a
    list of (gpu, ref) arrays of shape (ncomp, ...).  Each field's error is
    max |gpu - ref| over all pairs divided by the field's scale: its largest
    reference magnitude, except that for a conserved state (ncomp == 5,
    state not False) the three momenta are scaled by at least
    M = max over zones of sqrt(rho rho E), the momentum of the matter moving
    at about its sound speed.  The momentum fluxes of every face carry the
    pressure, so their rounding error is a fraction of rho c whatever the
    flow speed; a momentum component that is nearly zero (matter at rest, a
    flow along one axis) would otherwise turn rounding of the pressure terms
    into large relative errors.  Prints the errors (and, where the floor
    applies, the errors relative to the field's own maximum) and how many
    values differ in their bits; asserts every field error <= tol and names
    the worst value's pair and position if not."""
    ncomp = pairs[0][1].shape[0]
    state = (ncomp == 5) if state is None else state
    num = np.zeros(ncomp)
    den = np.zeros(ncomp)
    mscale = 0.0
    nbits = 0
    total = 0
    where = [None] * ncomp
    for k, (g, r) in enumerate(pairs):
        d = np.abs(g - r)
        for c in range(ncomp):
            m = float(np.nanmax(d[c])) if d[c].size else 0.0
            if not (m <= num[c]):
                num[c] = m
                where[c] = (k, np.unravel_index(int(np.nanargmax(d[c])), d[c].shape))
            den[c] = max(den[c], float(np.abs(r[c]).max()) if r[c].size else 0.0)
        if state and r[0].size:
            mscale = max(mscale, float(np.sqrt(np.abs(r[0] * r[4])).max()))
        nbits += int(np.count_nonzero(g != r))
        total += g.size
    own = np.where(den > 0, den, den.max() if den.max() > 0 else 1.0)
    scale = own.copy()
    if state:
        scale[1:4] = np.maximum(scale[1:4], mscale)
    err = num / scale
    extra = ""
    if state and np.any(scale != own):
        extra = f" (momenta against their own maxima {np.array2string(num[1:4] / own[1:4], precision=2)})"
    print(f"{tag}: per-field error {np.array2string(err, precision=2)}{extra}, "
          f"{nbits} of {total} values differ in their bits", flush=True)
    bad = [c for c in range(ncomp) if not err[c] <= tol]
    assert not bad, (tag, [(c, err[c], where[c]) for c in bad])
    return err, nbits

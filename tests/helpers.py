"""Shared helpers of the test suite (inputs and comparisons only)."""
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

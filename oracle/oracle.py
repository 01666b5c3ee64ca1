"""TEST INFRASTRUCTURE -- Python wrapper of the oracle (``ppm_oracle.cpp``).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads the serial C++ oracle with
ctypes and adds a multi-step driver.  It imports nothing from the product
package.

State layout (shared with the product by definition of the data, not by
code): one box is a float64 array of shape (5, n_z+8, n_y+8, n_x+8) holding
(rho, rho u, rho v, rho w, rho E) with 4 ghost zones on each side.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppm_oracle.cpp")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "liboracle.so")
NG = 4
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_COARSE_FINE, BC_INFLOW = 0, 1, 2, 3, 4
FLAG_NONPHYS, FLAG_FLOOR = 1, 2
STAGES = ("prim", "flatten", "trace", "riemann1", "transverse1", "riemann2",
          "transverse2", "riemann3", "update")
OPKINDS = ("add", "mul", "div", "sqrt", "minmax")


def build(force=True):
    """Compile the oracle with g++: -O2, no contraction, no fast-math."""
    os.makedirs(_LIBDIR, exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared",
           "-fPIC", _SRC, "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("small_dens", ctypes.c_double), ("small_pres", ctypes.c_double),
                ("grav", ctypes.c_double * 3), ("limiter", ctypes.c_int),
                ("flattening", ctypes.c_int), ("riemann_iters", ctypes.c_int),
                ("precision", ctypes.c_int)]


def params(gamma=1.4, cfl=0.5, small_dens=1e-12, small_pres=1e-12, grav=(0.0, 0.0, 0.0),
           limiter=1, flattening=1, riemann_iters=3, precision=0):
    p = OParams()
    p.gamma, p.cfl, p.small_dens, p.small_pres = gamma, cfl, small_dens, small_pres
    for d in range(3):
        p.grav[d] = grav[d]
    p.limiter, p.flattening, p.riemann_iters, p.precision = limiter, flattening, riemann_iters, precision
    return p


_lib_handle = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step.argtypes = [_dp, _ip, _ip, _ip, ctypes.c_double, _dp,
                                  ctypes.POINTER(OParams), _ip, _dp, ctypes.POINTER(_dp)]
        L.oracle_step_count.restype = ctypes.c_int
        L.oracle_step_count.argtypes = [_dp, _ip, _ip, _ip, ctypes.c_double, _dp,
                                        ctypes.POINTER(OParams), _ip, _dp,
                                        ctypes.POINTER(ctypes.c_ulonglong)]
        L.oracle_step_species.restype = ctypes.c_int
        L.oracle_step_species.argtypes = [_dp, _dp, ctypes.c_int, _ip, _ip, _ip, ctypes.c_double, _dp,
                                          ctypes.POINTER(OParams), _ip, _dp, _dp]
        L.oracle_fill_inflow.restype = ctypes.c_int
        L.oracle_fill_inflow.argtypes = [ctypes.c_int, _ip, _ip, _ip, _ip, _ip, _dp,
                                         ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_dp)]
        L.oracle_fill_scalars.restype = ctypes.c_int
        L.oracle_fill_scalars.argtypes = [ctypes.c_int, _ip, _ip, _ip, _ip, _ip, _dp,
                                          ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        L.oracle_step_jvp.restype = ctypes.c_int
        L.oracle_step_jvp.argtypes = [_dp, _dp, _ip, _ip, _ip, ctypes.c_double, _dp,
                                      ctypes.POINTER(OParams), _ip, _dp, _dp]
        L.oracle_step_jvp_flux.restype = ctypes.c_int
        L.oracle_step_jvp_flux.argtypes = [_dp, _dp, _ip, _ip, _ip, ctypes.c_double, _dp,
                                           ctypes.POINTER(OParams), _ip, _dp, _dp, ctypes.POINTER(_dp),
                                           ctypes.POINTER(_dp)]
        L.oracle_max_wavespeed.restype = ctypes.c_double
        L.oracle_max_wavespeed.argtypes = [_dp, _ip, _dp, ctypes.POINTER(OParams), _ip]
        L.oracle_riemann.restype = ctypes.c_int
        L.oracle_riemann.argtypes = [_dp, _dp, ctypes.c_int, ctypes.POINTER(OParams), _dp]
        L.oracle_flatten.restype = ctypes.c_int
        L.oracle_flatten.argtypes = [_dp, _ip, ctypes.POINTER(OParams), _dp]
        L.oracle_count_ops.restype = ctypes.c_int
        L.oracle_count_ops.argtypes = [ctypes.c_int, _dp, ctypes.POINTER(OParams), _dp,
                                       ctypes.POINTER(ctypes.c_ulonglong)]
        L.oracle_ppm_line.restype = ctypes.c_int
        L.oracle_ppm_line.argtypes = [_dp, ctypes.c_int, _dp, ctypes.POINTER(OParams), _dp, _dp, _dp]
        L.oracle_ppm_integrals.restype = None
        L.oracle_ppm_integrals.argtypes = [ctypes.c_double] * 4 + [_dp, _dp]
        L.oracle_trace.restype = ctypes.c_int
        L.oracle_trace.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                   ctypes.POINTER(OParams), _dp, _dp]
        L.oracle_fill.restype = ctypes.c_int
        L.oracle_fill.argtypes = [ctypes.c_int, _ip, _ip, _ip, _ip, _ip, _dp,
                                  ctypes.POINTER(ctypes.c_longlong)]
        _lib_handle = L
    return _lib_handle


def _d(a):
    return a.ctypes.data_as(_dp)


def _i3(v):
    return (ctypes.c_int * 3)(*[int(x) for x in v])


def _d3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def _box_n(U):
    assert U.dtype == np.float64 and U.flags.c_contiguous and U.ndim == 4 and U.shape[0] == 5
    return (U.shape[3] - 2 * NG, U.shape[2] - 2 * NG, U.shape[1] - 2 * NG)


def _walls(walls):
    """Six wall flags (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi) as a C array, or None."""
    if walls is None:
        return None
    return (ctypes.c_int * 6)(*[int(bool(w)) for w in walls])


def box_walls(boxes, domain, bc, b):
    """The faces of box b that lie on a reflecting domain boundary, as six
    flags (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi)."""
    lo, hi = boxes[b]
    dlo, dhi = domain
    out = []
    for d in range(3):
        out.append(int(lo[d] == dlo[d] and bc[2 * d] == BC_REFLECT))
        out.append(int(hi[d] == dhi[d] and bc[2 * d + 1] == BC_REFLECT))
    return tuple(out)


def step(U, dt, dx, p, window=None, fluxes=False, out=None, walls=None):
    """One step of one box (ghosts of U already filled).

    Returns (Unew, F, flags).  Unew has U's shape; only the window's valid
    zones are written (others copy U).  F is None or a list of three
    face-centred arrays, F[d] of shape (5, nz', ny', nx') with n_d + 1 faces
    along d.  window: ((x0, y0, z0), (x1, y1, z1)) inclusive valid indices.
    walls: the box's faces on a reflecting domain boundary (box_walls).
    """
    n = _box_n(U)
    wlo, whi = ((0, 0, 0), tuple(x - 1 for x in n)) if window is None else window
    Unew = U.copy() if out is None else out
    F = None
    Fp = None
    if fluxes:
        F = []
        for d in range(3):
            e = list(n)
            e[d] += 1
            F.append(np.zeros((5, e[2], e[1], e[0])))
        Fp = (_dp * 3)(*[_d(f) for f in F])
    fl = lib().oracle_step(_d(U), _i3(n), _i3(wlo), _i3(whi), float(dt), _d3(dx),
                           ctypes.byref(p), _walls(walls), _d(Unew), Fp)
    if fl < 0:
        raise ValueError("oracle_step: invalid arguments")
    return Unew, F, fl


def step_species(U, RX, dt, dx, p, window=None, walls=None):
    """One step of one box with passive species (ghosts of U and RX filled).
    RX: (ns, nz+8, ny+8, nx+8) partial densities rho X_s.  Returns
    (Unew, RXnew, flags); only the window's valid zones are written."""
    n = _box_n(U)
    assert RX.dtype == np.float64 and RX.flags.c_contiguous and RX.shape[1:] == U.shape[1:]
    wlo, whi = ((0, 0, 0), tuple(x - 1 for x in n)) if window is None else window
    Unew = U.copy()
    RXnew = RX.copy()
    fl = lib().oracle_step_species(_d(U), _d(RX), int(RX.shape[0]), _i3(n), _i3(wlo), _i3(whi), float(dt),
                                   _d3(dx), ctypes.byref(p), _walls(walls), _d(Unew), _d(RXnew))
    if fl < 0:
        raise ValueError("oracle_step_species: invalid arguments")
    return Unew, RXnew, fl


def step_count(U, dt, dx, p, window=None, walls=None):
    """Step with operation counting.  Returns (Unew, counts[stage][kind], flags)."""
    n = _box_n(U)
    wlo, whi = ((0, 0, 0), tuple(x - 1 for x in n)) if window is None else window
    Unew = U.copy()
    cnt = (ctypes.c_ulonglong * (len(STAGES) * len(OPKINDS)))()
    fl = lib().oracle_step_count(_d(U), _i3(n), _i3(wlo), _i3(whi), float(dt), _d3(dx),
                                 ctypes.byref(p), _walls(walls), _d(Unew), cnt)
    if fl < 0:
        raise ValueError("oracle_step_count: invalid arguments")
    counts = np.array(list(cnt), dtype=np.int64).reshape(len(STAGES), len(OPKINDS))
    return Unew, counts, fl


def step_jvp(U, dU, dt, dx, p, window=None, walls=None):
    """(step(U), J dU) with frozen dt and branches.  Ghosts of U and dU must be filled."""
    n = _box_n(U)
    assert dU.shape == U.shape and dU.dtype == np.float64 and dU.flags.c_contiguous
    wlo, whi = ((0, 0, 0), tuple(x - 1 for x in n)) if window is None else window
    Unew = U.copy()
    dUnew = np.zeros_like(U)
    fl = lib().oracle_step_jvp(_d(U), _d(dU), _i3(n), _i3(wlo), _i3(whi), float(dt), _d3(dx),
                               ctypes.byref(p), _walls(walls), _d(Unew), _d(dUnew))
    if fl < 0:
        raise ValueError("oracle_step_jvp: invalid arguments")
    return Unew, dUnew, fl


def step_jvp_flux(U, dU, dt, dx, p, walls=None):
    """(step(U), J dU, F, J_F dU): the new state and the face-centred flux
    outputs of one box with their tangents (FP64 mode; ghosts of U and dU
    filled).  F[d], dF[d]: arrays (5, nz', ny', nx') with n_d + 1 faces
    along d."""
    n = _box_n(U)
    assert dU.shape == U.shape and dU.dtype == np.float64 and dU.flags.c_contiguous
    Unew = U.copy()
    dUnew = np.zeros_like(U)
    F, dF = [], []
    for d in range(3):
        e = list(n)
        e[d] += 1
        F.append(np.zeros((5, e[2], e[1], e[0])))
        dF.append(np.zeros((5, e[2], e[1], e[0])))
    fl = lib().oracle_step_jvp_flux(_d(U), _d(dU), _i3(n), _i3((0, 0, 0)), _i3(tuple(x - 1 for x in n)),
                                    float(dt), _d3(dx), ctypes.byref(p), _walls(walls), _d(Unew), _d(dUnew),
                                    (_dp * 3)(*[_d(f) for f in F]), (_dp * 3)(*[_d(f) for f in dF]))
    if fl < 0:
        raise ValueError("oracle_step_jvp_flux: invalid arguments")
    return Unew, dUnew, F, dF, fl


def max_wavespeed(U, dx, p):
    """max over valid zones and axes of (|u_d| + c)/h_d; returns (s, flags)."""
    n = _box_n(U)
    fl = ctypes.c_int(0)
    s = lib().oracle_max_wavespeed(_d(U), _i3(n), _d3(dx), ctypes.byref(p), ctypes.byref(fl))
    return s, fl.value


def riemann(L, R, d, p):
    L = np.ascontiguousarray(L, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    F = np.zeros(5)
    fl = lib().oracle_riemann(_d(L), _d(R), int(d), ctypes.byref(p), _d(F))
    return F, fl


def flatten(U, p):
    """O3 alone: the flattening coefficient of every traced zone [-1, n]^3 of
    one box (O2 on its stored zones first; ghosts as given).  Returns
    (phi of shape (nz+2, ny+2, nx+2), flags)."""
    n = _box_n(U)
    phi = np.zeros((n[2] + 2, n[1] + 2, n[0] + 2))
    fl = lib().oracle_flatten(_d(U), _i3(n), ctypes.byref(p), _d(phi))
    if fl < 0:
        raise ValueError("oracle_flatten: invalid arguments")
    return phi, fl


def count_ops(what, inp, p):
    """Operation counts of one piece of the method: what = "riemann" (inp =
    L[5] + R[5], a face normal to x) or "conversion" (inp = q[5]: primitive
    -> conserved -> primitive with floors).  Returns (output, {kind: count},
    flags)."""
    code = {"riemann": 0, "conversion": 1}[what]
    a = np.ascontiguousarray(inp, dtype=np.float64)
    out = np.zeros(5)
    cnt = (ctypes.c_ulonglong * len(OPKINDS))()
    fl = lib().oracle_count_ops(code, _d(a), ctypes.byref(p), _d(out), cnt)
    if fl < 0:
        raise ValueError("oracle_count_ops: invalid arguments")
    return out, dict(zip(OPKINDS, (int(c) for c in cnt))), fl


def ppm_line(a, p, phi=None):
    """Parabolas (aL, aR, a6) of a 1-D line at indices 2..m-3 (NaN elsewhere)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    m = a.shape[0]
    aL, aR, a6 = np.full(m, np.nan), np.full(m, np.nan), np.full(m, np.nan)
    ph = None if phi is None else _d(np.ascontiguousarray(phi, dtype=np.float64))
    lib().oracle_ppm_line(_d(a), m, ph, ctypes.byref(p), _d(aL), _d(aR), _d(a6))
    return aL, aR, a6


def ppm_integrals(aL, aR, a6, sigma):
    ip, im = ctypes.c_double(), ctypes.c_double()
    lib().oracle_ppm_integrals(aL, aR, a6, sigma, ctypes.byref(ip), ctypes.byref(im))
    return ip.value, im.value


def trace(aL, aR, a6, cell, d, dtdx, p):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (aL, aR, a6, cell)]
    qp, qm = np.zeros(5), np.zeros(5)
    fl = lib().oracle_trace(_d(arr[0]), _d(arr[1]), _d(arr[2]), _d(arr[3]), int(d), float(dtdx),
                            ctypes.byref(p), _d(qp), _d(qm))
    return qp, qm, fl


def fill(boxes, domain, bc, states, inflow=None):
    """Ghost fill (O1) of a level, in place.

    boxes: list of (lo, hi) inclusive global index triples; domain: (lo, hi);
    bc: six face codes (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi); states: list of
    per-box arrays (5, nz+8, ny+8, nx+8), modified in place.  inflow: for a
    layout with an inflow face, {face: array (5, E_t2, E_t1)} of the
    prescribed conserved state over the domain's extents of the two other
    axes (t1 < t2).
    """
    nb = len(boxes)
    lo = (ctypes.c_int * (3 * nb))(*[int(v) for b in boxes for v in b[0]])
    hi = (ctypes.c_int * (3 * nb))(*[int(v) for b in boxes for v in b[1]])
    sizes = [s.size for s in states]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    arena = np.concatenate([s.ravel() for s in states])
    if inflow:
        keep = {f: np.ascontiguousarray(a, dtype=np.float64) for f, a in inflow.items()}
        ptrs = (_dp * 6)(*[_d(keep[f]) if f in keep else None for f in range(6)])
        rc = lib().oracle_fill_inflow(nb, lo, hi, _i3(domain[0]), _i3(domain[1]), (ctypes.c_int * 6)(*bc),
                                      _d(arena), off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), ptrs)
    else:
        rc = lib().oracle_fill(nb, lo, hi, _i3(domain[0]), _i3(domain[1]), (ctypes.c_int * 6)(*bc),
                               _d(arena), off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    if rc != 0:
        raise ValueError("oracle_fill: ghost image without an owning box")
    for s, o, z in zip(states, off, sizes):
        s.ravel()[:] = arena[o:o + z]
    return states


def fill_scalars(boxes, domain, bc, states):
    """Ghost fill of per-box scalar arrays (ncomp, nz+8, ny+8, nx+8) (passive
    species): like fill, with no sign change at reflecting walls."""
    nb = len(boxes)
    ncomp = int(states[0].shape[0])
    lo = (ctypes.c_int * (3 * nb))(*[int(v) for b in boxes for v in b[0]])
    hi = (ctypes.c_int * (3 * nb))(*[int(v) for b in boxes for v in b[1]])
    sizes = [s.size for s in states]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    arena = np.concatenate([s.ravel() for s in states])
    rc = lib().oracle_fill_scalars(nb, lo, hi, _i3(domain[0]), _i3(domain[1]), (ctypes.c_int * 6)(*bc),
                                   _d(arena), off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), ncomp)
    if rc != 0:
        raise ValueError("oracle_fill_scalars: ghost image without an owning box")
    for s, o, z in zip(states, off, sizes):
        s.ravel()[:] = arena[o:o + z]
    return states


def advance_species(boxes, domain, bc, states, rx, nsteps, dx, p, dt=None):
    """advance with passive species: rx is a list of per-box (ns, ...) arrays
    of partial densities.  Returns (states, rx, dts, flags)."""
    states = [s.copy() for s in states]
    rx = [r.copy() for r in rx]
    dts, flags = [], 0
    for _ in range(nsteps):
        fill(boxes, domain, bc, states)
        fill_scalars(boxes, domain, bc, rx)
        if dt is None:
            s = 0.0
            for U in states:
                sb, fl = max_wavespeed(U, dx, p)
                flags |= fl
                s = max(s, sb)
            dtn = p.cfl / s
        else:
            dtn = dt
        dts.append(dtn)
        new, newx = [], []
        for b, (U, R) in enumerate(zip(states, rx)):
            Un, Rn, fl = step_species(U, R, dtn, dx, p, walls=box_walls(boxes, domain, bc, b))
            flags |= fl
            new.append(Un)
            newx.append(Rn)
        states, rx = new, newx
    return states, rx, dts, flags


def advance(boxes, domain, bc, states, nsteps, dx, p, dt=None, fluxes=False, inflow=None):
    """Run nsteps full steps of a level: fill, dt = cfl / max signal speed
    (unless dt is given), step every box.  Returns (states, dts, flags, F)
    where F holds the last step's per-box fluxes if requested.  inflow: the
    inflow-face data of fill()."""
    states = [s.copy() for s in states]
    dts, flags, F = [], 0, None
    for _ in range(nsteps):
        fill(boxes, domain, bc, states, inflow=inflow)
        if dt is None:
            s = 0.0
            for U in states:
                sb, fl = max_wavespeed(U, dx, p)
                flags |= fl
                s = max(s, sb)
            dtn = p.cfl / s
        else:
            dtn = dt
        dts.append(dtn)
        new, F = [], []
        for b, U in enumerate(states):
            Un, Fb, fl = step(U, dtn, dx, p, fluxes=fluxes, walls=box_walls(boxes, domain, bc, b))
            flags |= fl
            new.append(Un)
            F.append(Fb)
        states = new
    return states, dts, flags, (F if fluxes else None)

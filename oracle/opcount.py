"""TEST INFRASTRUCTURE -- algorithmic operation counts per unit of work.

Runs the op-counting instantiation of the oracle on windows of a workload's
initial state and divides each stage's floating-point operation count by the
number of units that stage processes on the window, giving the per-unit
figures used for the arithmetic roofline of the step's kernels.  A flop is
one add/sub, mul, div or sqrt (min/max/abs/compare are not counted).

Units (window of valid extents w, traced region w + 2 per axis):
  prim      zones of the primitive region, prod(w + 8)
  flatten   traced zones, prod(w + 2)
  trace     traced (zone, axis) pairs, 3 prod(w + 2)
  riemann1  normal-predictor faces, sum_d (w_d + 1) prod_{t != d} (w_t + 2)
  riemann2  single-transverse faces, sum over (d, t) of (w_d + 1) w_t (w_r + 2)
  riemann3  final faces, sum_d (w_d + 1) w_t1 w_t2
  update    valid zones, prod(w)
The GPU kernel riemann2 also forms the corrected states (oracle stage
"transverse1"), riemann3 likewise ("transverse2"); their counts are merged.

Usage: python oracle/opcount.py [cfg2|cfg3|cfg4|cfg5] -> JSON on stdout.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path = [q for q in sys.path if os.path.abspath(q or ".") != HERE]
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402


def _load_inputs():
    """The seeded input generators (paper_1008_2801_amd/inputs.py, which
    imports only numpy and the standard library), loaded from their file
    alone: the package's __init__, and with it the HIP binding, is never
    imported."""
    import importlib.util
    path = os.path.join(ROOT, "paper_1008_2801_amd", "inputs.py")
    spec = importlib.util.spec_from_file_location("ppm_workload_inputs", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod  # dataclasses look their module up by name
    spec.loader.exec_module(mod)
    return mod


I = _load_inputs()

KERNELS = {"prim": ["prim"], "flatten": ["flatten"], "trace": ["trace"], "riemann1": ["riemann1"],
           "riemann2": ["transverse1", "riemann2"], "riemann3": ["transverse2", "riemann3"],
           "update": ["update"]}


def units(w):
    w = np.asarray(w, dtype=np.int64)
    e = w + 2
    r1 = sum((w[d] + 1) * np.prod([e[t] for t in range(3) if t != d]) for d in range(3))
    r2 = 0
    for d in range(3):
        for t in range(3):
            if t != d:
                r = 3 - d - t
                r2 += (w[d] + 1) * w[t] * e[r]
    r3 = sum((w[d] + 1) * np.prod([w[t] for t in range(3) if t != d]) for d in range(3))
    return {"prim": int(np.prod(w + 8)), "flatten": int(np.prod(e)), "trace": int(3 * np.prod(e)),
            "riemann1": int(r1), "riemann2": int(r2), "riemann3": int(r3), "update": int(np.prod(w))}


def per_unit(states, dx, p, windows, walls=None):
    """Flops per unit of each stage over windows [(box, lo, hi)] of the
    boxes' filled states."""
    tot = {k: 0 for k in KERNELS}
    cnt = {k: 0 for k in KERNELS}
    kinds = {k: np.zeros(len(O.OPKINDS), dtype=np.int64) for k in KERNELS}
    for b, lo, hi in windows:
        _, counts, _ = O.step_count(states[b], 1e-3, dx, p, window=(lo, hi),
                                    walls=walls[b] if walls else None)
        u = units(np.array(hi) - np.array(lo) + 1)
        for k, stages in KERNELS.items():
            c = sum(counts[O.STAGES.index(s)] for s in stages)
            kinds[k] += c
            tot[k] += int(c[:4].sum())
            cnt[k] += u[k]
    return ({k: tot[k] / cnt[k] for k in KERNELS},
            {k: {O.OPKINDS[i]: kinds[k][i] / cnt[k] for i in range(len(O.OPKINDS))} for k in KERNELS})


def measure(name="cfg2"):
    """(flops per unit, ops per unit by kind, windows) of a workload's step:
    six 12^3 windows of the initial state (in six different boxes of a
    multi-box level)."""
    if name == "cfg2":
        wl = I.cfg2(64)  # same recipe (seed, modes, jump, velocity draws) on a 64^3 box
    elif name == "cfg3":
        wl = I.cfg3()
    elif name == "cfg4":
        wl = I.cfg4(64)
    else:
        # the 512^3 Rayleigh-Taylor recipe on 4^3 boxes of 32^3 (interface
        # width 2 zones as in the full level; the sampled boxes include the
        # walls and the interface)
        wl = I.cfg5(4, 32, precision=0)
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    walls = [O.box_walls(lay.boxes(), lay.domain(), lay.bc, b) for b in range(lay.nbox)]
    rng = np.random.default_rng(0)
    w = 12
    boxes = rng.choice(lay.nbox, min(6, lay.nbox), replace=False) if lay.nbox > 1 else [0] * 6
    windows = []
    for b in boxes:
        n = lay.n(int(b))
        lo = [int(rng.integers(0, n[d] - w + 1)) for d in range(3)]
        windows.append((int(b), tuple(lo), tuple(v + w - 1 for v in lo)))
    p = O.params(gamma=wl.gamma, grav=wl.grav)
    flops, kinds = per_unit(st, wl.dx, p, windows, walls)
    return flops, kinds, windows


def main(name="cfg2"):
    flops, kinds, windows = measure(name)
    print(json.dumps({"workload": name, "windows": windows, "flops_per_unit": flops,
                      "ops_per_unit_by_kind": kinds}, indent=1))


if __name__ == "__main__":
    main(*sys.argv[1:])

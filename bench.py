#!/usr/bin/env python3
"""Throughput of the unsplit PPM step on one MI355X.

A step is one pass of the hot path over the level: ghost fill, CFL time step
on the device, and the step itself (primitive conversion, flattening, PPM
reconstruction, characteristic tracing, 12 two-shock Riemann solves per zone
with corner-transport corrections, conservative update).  The default
workload is the 256^3 single-box FP64 problem (gamma 5/3, random-mode density
times a planar Sod jump, constant random velocity, periodic); inputs are
synthetic and seeded and are resident in HBM before timing starts.

Prints one JSON line.  `value` is zone-updates/s (valid zones x steps / s).
`roofline` reports the stage kernel that takes the most time, with its
algorithmic FP64 flops per launch divided by its mean launch time (HIP events
on the stream the kernels run on) against the FP64 vector peak.
`cpu_baseline` times the serial CPU reference evaluation on a bounded window
of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zone-updates/s per PPM step: batched vs plain per-box; adjoint/forward cost"

# Algorithmic FP64 flops (add/sub, mul, div, sqrt; min/max not counted) per
# unit of work of each stage kernel, counted by the op-counting instantiation
# of the reference evaluation on windows of this workload's state
# (oracle/opcount.py cfg2).  Units: see stage_units().
FLOPS_PER_UNIT = {"prim": 15.0, "flatten": 64.99, "trace": 389.27, "riemann1": 178.06,
                  "riemann2": 256.06, "riemann3": 286.06, "update": 45.0}
# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
FP64_VECTOR_PEAK_TFLOPS = 78.6
# MI355X FP32 vector peak (packed FP32 FMA), the peak of the FP32-reconstruction
# mode's stage kernels.
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


# Tilings picked by the autotuner on this device, keyed by architecture,
# precision and box-size histogram (see ppm_autotune); a level whose key is
# present is set up without timing, so the timed configuration is stable.
AUTOTUNE_CACHE = os.path.join(ROOT, "paper_1008_2801_amd", "autotune_cache.jsonl")

# Sources whose change invalidates recorded counter traffic (kernels, their
# arithmetic and the tile lists that shape the launches).
TRAFFIC_SOURCES = ("paper_1008_2801_amd/csrc/ppm_kernels.hip", "paper_1008_2801_amd/csrc/ppm_math.h",
                   "paper_1008_2801_amd/csrc/ppm_device.h", "paper_1008_2801_amd/csrc/ppm_internal.h",
                   "paper_1008_2801_amd/csrc/ppm_api.hip")


def sources_digest():
    """SHA-256 of the traffic sources' code: comments and blank lines are
    dropped first, so that only a change of the code itself invalidates a
    record."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def traffic_record_path(kernel, workload):
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")


def record_traffic(fetch_csv, write_csv, kernel, workload, tiling, fetch_factor, write_factor):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the kernel from two
    rocprofv3 --pmc runs, times the factors a plain copy of known size gives,
    stored with the digest of the kernel sources and the tiling."""
    import csv

    def mean_kib(path, counter):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                if r["Counter_Name"] == counter and f"k_{kernel}<double>" in r["Kernel_Name"]]
        if not vals:
            raise SystemExit(f"no {counter} records of k_{kernel}<double> in {path}")
        return sum(vals) / len(vals), len(vals)
    f_kib, nf = mean_kib(fetch_csv, "FETCH_SIZE")
    w_kib, nw = mean_kib(write_csv, "WRITE_SIZE")

    def step_bytes(path, counter, factor):
        # every stage kernel of the step (not the one dt pass before the
        # first step), per step: the counted dispatches over the step count,
        # which the kernel's own dispatches give
        tot = sum(float(r["Counter_Value"]) for r in csv.DictReader(open(path))
                  if r["Counter_Name"] == counter and "ppm::" in r["Kernel_Name"]
                  and "k_wavespeed" not in r["Kernel_Name"])
        return tot * 1024 * factor
    steps = nf  # one dispatch of the kernel per step
    rec = {"kernel": f"k_{kernel}<double>", "workload": workload, "tiling": list(tiling),
           "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib, "dispatches": [nf, nw],
           "fetch_factor": fetch_factor, "write_factor": write_factor,
           "read_bytes_per_launch": f_kib * 1024 * fetch_factor,
           "write_bytes_per_launch": w_kib * 1024 * write_factor,
           "sources_sha256": sources_digest()}
    rec["traffic_bytes_per_launch"] = rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    rec["step_traffic_bytes"] = (step_bytes(fetch_csv, "FETCH_SIZE", fetch_factor) +
                                 step_bytes(write_csv, "WRITE_SIZE", write_factor)) / steps
    with open(traffic_record_path(kernel, workload), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def recorded_traffic(kernel, workload, tiling, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of the kernel (key "step_traffic_bytes": of the
    whole step) from the recorded counters, or None when there is no record
    or the kernels or tiling changed since it was taken."""
    try:
        with open(traffic_record_path(kernel, workload)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != sources_digest() or list(rec.get("tiling", [])) != list(tiling):
        return None
    return rec.get(key)


def stage_units(n):
    """Units each stage kernel processes on one box of valid extents n."""
    import numpy as np
    w = np.asarray(n, dtype=np.int64)
    e = w + 2
    r1 = sum((w[d] + 1) * np.prod([e[t] for t in range(3) if t != d]) for d in range(3))
    r2 = sum((w[d] + 1) * w[t] * e[3 - d - t] for d in range(3) for t in range(3) if t != d)
    r3 = sum((w[d] + 1) * np.prod([w[t] for t in range(3) if t != d]) for d in range(3))
    return {"prim": int(np.prod(w + 8)), "flatten": int(np.prod(e)), "trace": int(3 * np.prod(e)),
            "riemann1": int(r1), "riemann2": int(r2), "riemann3": int(r3), "update": int(np.prod(w))}


def make_workload(name):
    from paper_1008_2801_amd import inputs as I
    if name == "cfg2":
        return I.cfg2()
    if name == "cfg2-small":
        return I.cfg2(64)
    if name == "cfg2-fp32":
        wl = I.cfg2()  # the same level and state, FP32 reconstruction, FP64 update
        wl.precision = 1
        return wl
    raise SystemExit(f"unknown workload {name}")


def level_rates(wl, steps, warmup, precision, per_box=True):
    """zone-updates/s of one workload in three launch forms: batched eager
    (one launch per stage over all boxes), per-box eager (one launch per
    stage per box) and a HIP graph of `steps` batched steps.  In all three
    each step's dt comes from the update of the step before it."""
    import torch
    from paper_1008_2801_amd import ppm as P
    lay = wl.layout
    lev = P.Level(lay)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    lev.ensure_workspace(precision)
    U0 = torch.from_numpy(wl.arena).to("cuda")
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    zones = lay.valid_zones()
    Uf = U0.clone()
    lev.fill_boundary(Uf)
    tile, strip, _ = lev.autotune(Uf, wl.dx, p, reps=2, cache_path=AUTOTUNE_CACHE)
    del Uf
    out = {"tiling": {"tile": tile, "strip_rows": strip}}
    forms = (("batched", P.BATCHED), ("per_box", P.PER_BOX)) if per_box else (("batched", P.BATCHED),)
    for name, mode in forms:
        U = U0.clone()
        V = lev.new_state()
        lev.compute_dt(U, wl.dx, p, out=dtv)
        for k in range(warmup + steps):
            if k == warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            # each step's dt left in dtv by the update of the step before
            lev.fill_boundary(U, mode)
            lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, mode=mode, dt_next=dtv)
            U, V = V, U
        torch.cuda.synchronize()
        out[name] = zones * steps / (time.perf_counter() - t0)
    A = U0.clone()
    B = lev.new_state()
    g = lev.graph(A, B, wl.dx, p, steps)
    g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch()
    torch.cuda.synchronize()
    out["graph"] = zones * steps / (time.perf_counter() - t0)
    out["flags"] = lev.check_status()
    g.close()
    lev.close()
    lev._work = None
    del A, B, U0, U, V, g, lev
    torch.cuda.empty_cache()
    return out


def adjoint_costs(wl, nsteps, every, reps=3, precision=0, rollout=True):
    """Per-step forward and adjoint times (the adjoint includes its own
    recompute of the forward intermediates) and the whole checkpointed
    roll-out, forward vs backward."""
    import torch
    from paper_1008_2801_amd import ppm as P
    lay = wl.layout
    lev = P.Level(lay)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    U = torch.from_numpy(wl.arena).to("cuda")
    lev.fill_boundary(U)
    V = lev.new_state()
    dtv = lev.compute_dt(U, wl.dx, p)
    W = torch.randn_like(U)
    Ub = torch.empty_like(U)
    lev.ensure_workspace(precision)
    lev.ensure_adjoint_workspace(precision)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    t_fwd = timed(lambda: lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv))
    t_adj = timed(lambda: lev.hydro_step_adjoint(U, W, Ub, wl.dx, p, dt_dev=dtv))
    # the adjoint on the intermediates the forward step left in its workspace
    acc = 0.0
    for r in range(reps + 1):
        lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lev.hydro_step_adjoint(U, W, Ub, wl.dx, p, dt_dev=dtv, saved=True)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            acc += e0.elapsed_time(e1)
    t_sav = acc / reps
    res = {"precision": "f64" if precision == 0 else "f32 reconstruction + f64 update",
           "forward_step_ms": t_fwd, "adjoint_step_ms": t_adj, "adjoint_over_forward": t_adj / t_fwd,
           "adjoint_step_saved_ms": t_sav, "adjoint_saved_over_forward": t_sav / t_fwd}
    if not rollout:
        res["flags"] = lev.check_status()
        lev.close()
        return res
    del W, Ub, V
    res.update({"rollout_steps": nsteps, "checkpoint_every": every})
    for saved, tag in ((False, ""), (True, "_saved_segments")):
        t_f, t_b = [], []
        for _ in range(3):  # the first backward also starts autograd's device thread
            U0 = torch.from_numpy(wl.arena).to("cuda").requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            UT = P.rollout(U0, lev, nsteps, wl.dx, p, checkpoint_every=every, saved=saved)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            UT.backward(torch.ones_like(UT))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            t_f.append(t1 - t0)
            t_b.append(t2 - t1)
            del UT, U0
        res.update({"rollout_forward_s" + tag: min(t_f), "rollout_backward_s" + tag: min(t_b),
                    "backward_over_forward" + tag: min(t_b) / min(t_f)})
    lev.release_workspace_slots()
    res["flags"] = lev.check_status()
    lev.close()
    return res


# Per species and traced zone, the bytes each staged species kernel must move
# at least (every plane it reads or writes touched once, FP64): fractions
# 8 + 8, trace 3 x 8 read + 6 x 8 written, stage 1 6 x 8 + 3 x 8, stage 2
# (6 + 3) x 8 + 6 x 8, stage 3 (6 + 6) x 8 + 3 x 8, update 3 x 8 + 8 + 8;
# plus the hydro planes the stages read once per zone for all species
# (density for the fractions; flattening, normal velocity and sound speed
# per axis; stage mass fluxes and traced densities).
SPECIES_BYTES_PER_ZONE_SPECIES = 16 + 72 + 72 + 120 + 120 + 40
SPECIES_SHARED_BYTES_PER_ZONE = 8 + 72 + 24 + 120 + 120


def species_costs(wl, ns, steps, warmup, precision=0):
    """Time of the step with ns passive species against the plain step on
    the same level (HIP events on the launch stream), and the species part's
    rate against the HBM roofline of its staged kernels' minimum traffic."""
    import numpy as np
    import torch
    from paper_1008_2801_amd import inputs as I
    from paper_1008_2801_amd import ppm as P
    lay = wl.layout
    lev = P.Level(lay)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    lev.ensure_workspace(precision)
    lev.ensure_species_workspace(ns, precision)
    U0 = torch.from_numpy(wl.arena).to("cuda")
    R0 = torch.from_numpy(I.species(wl, ns, seed=80)).to("cuda")
    Uf = U0.clone()
    lev.fill_boundary(Uf)
    lev.autotune(Uf, wl.dx, p, reps=2, cache_path=AUTOTUNE_CACHE)
    del Uf
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")

    def run(with_species):
        U, V = U0.clone(), lev.new_state()
        R, Rn = R0.clone(), lev.new_species(ns)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for k in range(warmup + steps):
            if k == warmup:
                e0.record()
            lev.fill_boundary(U)
            lev.compute_dt(U, wl.dx, p, out=dtv)
            if with_species:
                lev.fill_species(R, ns)
                lev.hydro_step_species(U, V, R, Rn, ns, wl.dx, p, dt_dev=dtv)
                R, Rn = Rn, R
            else:
                lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv)
            U, V = V, U
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    plain = min(run(False) for _ in range(2))
    with_sp = min(run(True) for _ in range(2))
    zones = lay.valid_zones()
    ezones = sum(int(np.prod(np.asarray(lay.n(b)) + 2)) for b in range(lay.nbox))
    sp_ms = with_sp - plain
    size = 8 if precision == 0 else 4
    # the fractions, fluxes and traces are in the reconstruction precision;
    # rho X and its update stay FP64
    nbytes = ezones * (ns * SPECIES_BYTES_PER_ZONE_SPECIES * size / 8 + SPECIES_SHARED_BYTES_PER_ZONE * size / 8)
    out = {"species": ns, "ms_per_step_plain": plain, "ms_per_step_with_species": with_sp,
           "species_ms_per_step": sp_ms, "species_ms_per_species": sp_ms / ns,
           "zone_species_updates_per_s": zones * ns / (sp_ms / 1e3) if sp_ms > 0 else None,
           "species_min_traffic_GB": nbytes / 1e9,
           "species_hbm_GBps": nbytes / (sp_ms / 1e3) / 1e9 if sp_ms > 0 else None,
           "flags": lev.check_status()}
    lev.close()
    del U0, R0, lev
    torch.cuda.empty_cache()
    return out


def amr_costs(n, cbox, fbox, steps, warmup, precision=0):
    """One coarse step of the two-level hierarchy (inner 12.5% refined by 2,
    so the fine level has as many zones as the coarse one) against the
    single-level steps it contains.  The paper's overhead measure compares
    it with three single-level coarse steps; the second measure compares it
    with the level steps actually run (one coarse and two fine)."""
    import torch
    from paper_1008_2801_amd import inputs as I
    from paper_1008_2801_amd import ppm as P
    t = I.amr_cfg2(n, cbox=cbox, fbox=fbox)
    H = P.TwoLevel(t.coarse.layout, t.fine.layout)
    p = P.params(gamma=t.coarse.gamma, precision=precision)
    for lev in (H.coarse, H.fine):
        lev.ensure_workspace(precision)
    Uc0 = torch.from_numpy(t.coarse.arena).to("cuda")
    Uf0 = torch.from_numpy(t.fine.arena).to("cuda")
    for lev, U in ((H.coarse, Uc0), (H.fine, Uf0)):
        Ut = U.clone()
        if lev is H.coarse:
            lev.fill_boundary(Ut)
        else:
            Uc = Uc0.clone()
            H.coarse.fill_boundary(Uc)
            H.fill_fine(Uc, Uc, 0, Ut)
            del Uc
        lev.autotune(Ut, t.coarse.dx if lev is H.coarse else t.fine.dx, p, reps=2, cache_path=AUTOTUNE_CACHE)
        del Ut
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")

    def timed(fn, nst, nwarm):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for k in range(nwarm + nst):
            if k == nwarm:
                e0.record()
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / nst

    # single-level steps: the coarse level alone (periodic) and the fine
    # level alone (its coarse-fine ghosts filled once, then left as they are)
    st = {"Uc": Uc0.clone(), "Vc": H.coarse.new_state()}

    def coarse_single():
        H.coarse.fill_boundary(st["Uc"])
        H.coarse.compute_dt(st["Uc"], t.coarse.dx, p, out=dtv)
        H.coarse.hydro_step(st["Uc"], st["Vc"], t.coarse.dx, p, dt_dev=dtv)
        st["Uc"], st["Vc"] = st["Vc"], st["Uc"]
    t_c = min(timed(coarse_single, steps, warmup) for _ in range(2))
    Uc = Uc0.clone()
    H.coarse.fill_boundary(Uc)
    fs = {"Uf": Uf0.clone(), "Vf": H.fine.new_state()}
    H.fill_fine(Uc, Uc, 0, fs["Uf"])
    H.fill_fine(Uc, Uc, 0, fs["Vf"])

    def fine_single():
        H.fine.fill_boundary(fs["Uf"])
        H.fine.compute_dt(fs["Uf"], t.fine.dx, p, out=dtv)
        H.fine.hydro_step(fs["Uf"], fs["Vf"], t.fine.dx, p, dt_dev=dtv)
        fs["Uf"], fs["Vf"] = fs["Vf"], fs["Uf"]
    t_f = min(timed(fine_single, steps, warmup) for _ in range(2))
    del Uc, fs, st
    # the hierarchy
    am = {"Uc": Uc0.clone(), "Vc": H.coarse.new_state(), "Uf": Uf0.clone(), "Tf": H.fine.new_state()}

    def amr_step():
        H.step(am["Uc"], am["Vc"], am["Uf"], am["Tf"], t.coarse.dx, p)
        am["Uc"], am["Vc"] = am["Vc"], am["Uc"]
    t_a = min(timed(amr_step, steps, warmup) for _ in range(2))
    flags = H.coarse.check_status() | H.fine.check_status()
    sizes = H.sizes()
    zc, zf = t.coarse.layout.valid_zones(), t.fine.layout.valid_zones()
    H.close()
    del am, Uc0, Uf0, H
    torch.cuda.empty_cache()
    return {"coarse_zones": zc, "fine_zones": zf, "coarse_boxes": t.coarse.layout.nbox,
            "fine_boxes": t.fine.layout.nbox, "ms_single_level_coarse_step": t_c,
            "ms_single_level_fine_step": t_f, "ms_two_level_coarse_step": t_a,
            "overhead_vs_3_coarse_steps": t_a / (3.0 * t_c) - 1.0,
            "overhead_vs_level_steps": t_a / (t_c + 2.0 * t_f) - 1.0,
            "zone_updates_per_s": (zc + 2 * zf) / (t_a / 1e3), "sizes": sizes, "flags": flags}


def jet_costs(n=256, nz=4, graph_steps=250):
    """The inflowing jet on n^2 x nz zones to t = 300 us: the eager loop
    (fill, CFL dt read back every step, step) timed over the whole run, and
    HIP graphs of graph_steps steps (dt from the CFL rule on the device)."""
    import numpy as np
    import torch
    from paper_1008_2801_amd import inputs as I
    from paper_1008_2801_amd import ppm as P
    wl = I.jet(n, nz=nz)
    lev = P.Level(wl.layout)
    lev.set_inflow(2, torch.from_numpy(np.ascontiguousarray(wl.meta["inflow"][2])).to("cuda"))
    p = P.params(gamma=wl.gamma)
    lev.ensure_workspace(0)
    U = torch.from_numpy(wl.arena).to("cuda")
    V = lev.new_state()
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, t_end, nsteps = 0.0, wl.meta["t_end"], 0
    while t < t_end * (1 - 1e-12):
        lev.fill_boundary(U)
        lev.compute_dt(U, wl.dx, p, out=dtv)
        dt = min(float(dtv[0].item()), t_end - t)
        lev.hydro_step(U, V, wl.dx, p, dt=dt)
        U, V = V, U
        t += dt
        nsteps += 1
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0
    A = U.clone()
    B = lev.new_state()
    g = lev.graph(A, B, wl.dx, p, graph_steps)
    g.launch()
    torch.cuda.synchronize()
    reps = 4
    t0 = time.perf_counter()
    for _ in range(reps):
        g.launch()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / (reps * graph_steps)
    flags = lev.check_status()
    g.close()
    lev.close()
    zones = wl.layout.valid_zones()
    del U, V, A, B, lev
    torch.cuda.empty_cache()
    return {"zones": zones, "steps_to_300us": nsteps, "eager_run_s": eager_s,
            "eager_ms_per_step": eager_s / nsteps * 1e3, "graph_ms_per_step": graph_s * 1e3,
            "graph_zone_updates_per_s": zones / graph_s, "graph_run_s_estimate": graph_s * nsteps,
            "flags": flags}


def copy_bandwidth(gib=2, reps=5):
    """Measured HBM bandwidth of a plain device-to-device copy (bytes read +
    written per second), the practical ceiling next to the 8 TB/s spec."""
    import torch
    n = gib * (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * n * 8 / sec / 1e9


def cpu_baseline(wl, window_edge, gamma):
    """Serial oracle on one step of a cubic window of the workload."""
    import numpy as np
    from oracle import oracle as O
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    p = O.params(gamma=gamma)
    s, _ = O.max_wavespeed(st[0], wl.dx, p)
    dt = p.cfl / s
    lo = (0, 0, 0)
    hi = (window_edge - 1,) * 3
    t0 = time.perf_counter()
    O.step(st[0], dt, wl.dx, p, window=(lo, hi))
    sec = time.perf_counter() - t0
    zones = window_edge ** 3
    return {"value": zones / sec, "unit": "zone-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one step of the same workload on the {window_edge}^3 window of valid zones "
                      f"at the box corner (serial C++ reference, -O2, 1 thread), {sec:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--cpu-window", type=int, default=160)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiling")
    ap.add_argument("--autotune-cache", default=None,
                    help="autotuner cache file (default: the package's autotune_cache.jsonl)")
    ap.add_argument("--tiling", default=None, help="'tile,strip_rows': use this tiling instead of autotuning")
    ap.add_argument("--fused", action="store_true",
                    help="run the final fluxes and the update in the brick kernel (fluxes in LDS)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 512-box batched / per-box / graph measurements")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only measure the adjoint/forward cost on the 128^3 differentiation workload")
    ap.add_argument("--amr-only", action="store_true",
                    help="with --no-extras: still measure the two-level hierarchy")
    ap.add_argument("--jet-only", action="store_true",
                    help="with --no-extras: still run the inflowing jet to 300 us")
    ap.add_argument("--species-only", action="store_true",
                    help="with --no-extras: still measure the passive-species step")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record of the dominant kernel from two rocprofv3 --pmc "
                         "counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--record-kernel", default="riemann2")
    ap.add_argument("--counter-factors", default="2.0,1.0",
                    help="FETCH_SIZE and WRITE_SIZE scale factors from the copy calibration")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU box distribution is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    if args.autotune_cache:
        global AUTOTUNE_CACHE
        AUTOTUNE_CACHE = args.autotune_cache
    if args.record_traffic:
        ff, wf = (float(v) for v in args.counter_factors.split(","))
        t_, s_ = (int(v) for v in args.tiling.split(","))
        record_traffic(args.record_traffic[0], args.record_traffic[1], args.record_kernel, args.workload,
                       (t_, s_), ff, wf)
        return

    import torch
    from paper_1008_2801_amd import ppm as P

    if args.calibrate_copy:
        n = (1 << 30) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                          "copies": 3}))
        return

    if args.adjoint_only:
        from paper_1008_2801_amd import inputs as I
        a = adjoint_costs(I.cfg4(), 20, 5)
        a32 = adjoint_costs(I.cfg4(), 20, 5, precision=1)
        print(json.dumps({"adjoint": a, "adjoint_fp32_reconstruction": a32}))
        return

    wl = make_workload(args.workload)
    lay = wl.layout
    print(f"bench: workload {wl.name} {lay.n(0)} x {lay.nbox} box(es), building state", file=sys.stderr,
          flush=True)
    lev = P.Level(lay)
    lev.set_step_form(args.fused)
    U = torch.from_numpy(wl.arena).to("cuda")
    V = lev.new_state()
    p = P.params(gamma=wl.gamma, precision=wl.precision)
    lev.ensure_workspace(p.precision)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    if args.tiling:
        t_, s_ = (int(v) for v in args.tiling.split(","))
        lev.set_tiling(t_, s_)
        tiling = lev.get_tiling()
    elif not args.no_autotune:
        Uf = U.clone()
        lev.fill_boundary(Uf)
        tiling = lev.autotune(Uf, wl.dx, p, reps=2, cache_path=AUTOTUNE_CACHE)[:2]
        del Uf
    else:
        tiling = lev.get_tiling()

    # Each step reads its dt from dtv and leaves the next step's there: the
    # CFL maximum of the state it writes, computed by its update kernel
    # (ppm_hydro_step_dt), the same bits as a separate pass over it.
    def step(a, b):
        lev.fill_boundary(a)
        lev.hydro_step(a, b, wl.dx, p, dt_dev=dtv, dt_next=dtv)
        return b, a

    lev.compute_dt(U, wl.dx, p, out=dtv)
    for _ in range(args.warmup):
        U, V = step(U, V)
    torch.cuda.synchronize()
    lev.profile_read()
    lev.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        U, V = step(U, V)
    e1.record()
    torch.cuda.synchronize()
    lev.profile_enable(False)
    ms = e0.elapsed_time(e1)
    prof = lev.profile_read()
    flags = lev.check_status()
    zones = lay.valid_zones()
    value = zones * args.steps / (ms / 1e3)

    # dominant stage kernel and its arithmetic roofline
    units = {k: 0 for k in FLOPS_PER_UNIT}
    for b in range(lay.nbox):
        for k, v in stage_units(lay.n(b)).items():
            units[k] += v
    stages = {k: prof[k] for k in FLOPS_PER_UNIT}
    dom = max(stages, key=lambda k: stages[k][0])
    t_ms, cnt = stages[dom]
    mean_s = t_ms / cnt / 1e3
    flops = FLOPS_PER_UNIT[dom] * units[dom]
    achieved = flops / mean_s / 1e12
    step_flops = sum(FLOPS_PER_UNIT[k] * units[k] for k in FLOPS_PER_UNIT)
    # the FP32 mode's stage kernels compute in FP32 (the counts are those of
    # the same algorithm; the FP32 forms differ by a few operations per solve)
    peak = FP64_VECTOR_PEAK_TFLOPS if p.precision == 0 else FP32_VECTOR_PEAK_TFLOPS
    # HBM bytes of a whole step from the same counter record (all its
    # kernels), against the step's live time: the staged step's traffic rate
    step_traffic = (recorded_traffic(dom, args.workload, tiling, "step_traffic_bytes")
                    if p.precision == 0 else None)
    out = {
        "metric": METRIC, "value": value, "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if p.precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {lay.n(0)[0]}^3 single box, "
                               f"{'FP64' if p.precision == 0 else 'FP32 reconstruction + FP64 update'}, "
                               f"gamma {wl.gamma:.4g}, "
                               "random-mode density x planar Sod jump, periodic, CFL 0.5, plain step "
                               "(fill + step; each step's CFL dt computed by the previous step's update)",
                   "valid_zones": zones, "boxes": lay.nbox,
                   "tiling": {"tile": tiling[0], "strip_rows": tiling[1]}},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": recorded_traffic(dom, args.workload, tiling) if p.precision == 0 else None,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "mean_launch_ms": mean_s * 1e3, "flops_per_launch": flops,
                     "step_traffic": step_traffic,
                     "step_traffic_GBps": (step_traffic / (ms / args.steps / 1e3) / 1e9
                                           if step_traffic else None)},
        "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items()},
        "step_flop_rate_tflops": step_flops * args.steps / (ms / 1e3) / 1e12,
        "hbm_copy_GBps": copy_bandwidth(),
        "status_flags": flags,
    }
    if not args.no_extras:
        del lev, U, V
        torch.cuda.empty_cache()
        from paper_1008_2801_amd import inputs as I
        print("bench: 512-box level (batched / per-box / graph)", file=sys.stderr, flush=True)
        w3 = I.cfg3()
        extra = {"workload": f"cfg3: 512 boxes, edges from {{16,24,32,48,64}} (seed 3), "
                             f"{w3.layout.valid_zones()} valid zones, gamma 1.4, periodic, 20 steps",
                 "unit": "zone-updates/s"}
        for prec, tag in ((0, "fp64"), (1, "fp32_reconstruction")):
            r = level_rates(w3, 20, 2, prec)
            extra[tag] = r
            extra[tag]["batched_over_per_box"] = r["batched"] / r["per_box"]
        out["multibox"] = extra
        print("bench: adjoint cost on the 128^3 differentiation workload", file=sys.stderr, flush=True)
        w4 = I.cfg4()
        a = adjoint_costs(w4, 20, 5)
        a["workload"] = "cfg4: 128^3 single box, FP64, gamma 1.4, smooth modes of amplitude 0.05, periodic"
        out["adjoint"] = a
        a = adjoint_costs(w4, 20, 5, precision=1)
        a["workload"] = "cfg4 with the FP32-reconstruction step and its FP32 reverse"
        out["adjoint_fp32_reconstruction"] = a
        del w4
        print("bench: adjoint cost on a 2x2x2-box instance of the Rayleigh-Taylor set-up", file=sys.stderr,
              flush=True)
        a5 = adjoint_costs(I.cfg5(nb=2, m=64, precision=0), 10, 5)
        a5["workload"] = ("cfg5 instance: 8 boxes of 64^3 (128^3), Rayleigh-Taylor, g = (0,0,-1), walls in z, "
                          "FP64, 10 steps")
        out["adjoint_rayleigh_taylor"] = a5
        a5 = adjoint_costs(I.cfg5(nb=2, m=64, precision=1), 10, 5, precision=1)
        a5["workload"] = "the same instance with the FP32-reconstruction step and its FP32 reverse"
        out["adjoint_rayleigh_taylor_fp32_reconstruction"] = a5
        print("bench: 512^3 Rayleigh-Taylor level (512 boxes of 64^3)", file=sys.stderr, flush=True)
        w5 = I.cfg5()
        rt = {"workload": "cfg5: 512 boxes of 64^3 (512^3), Rayleigh-Taylor, g = (0,0,-1), walls in z, "
                          "10 steps", "unit": "zone-updates/s"}
        for prec, tag in ((1, "fp32_reconstruction"), (0, "fp64")):
            r = level_rates(w5, 10, 1, prec, per_box=False)
            rt[tag] = r
        print("bench: adjoint step of the 512^3 Rayleigh-Taylor level (FP32 reconstruction)", file=sys.stderr,
              flush=True)
        torch.cuda.empty_cache()
        a5 = adjoint_costs(w5, 0, 1, precision=1, rollout=False)
        a5["workload"] = "cfg5: 512 boxes of 64^3, FP32 reconstruction, one forward step vs one adjoint step"
        rt["adjoint"] = a5
        out["rayleigh_taylor"] = rt
        del w5
    if not args.no_extras or args.amr_only:
        print("bench: two-level hierarchy (256^3 coarse, inner 12.5% refined)", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        am = {"workload": "cfg2's state on 256^3 coarse zones with the inner 12.5% of the domain refined by 2 "
                          "(256^3 fine zones); one coarse step = coarse step + two fine steps + fill, "
                          "interpolation, flux register, reflux, average down; 5 timed steps",
              "one_box_per_level": amr_costs(256, 256, 256, 5, 1),
              "boxes_of_64": amr_costs(256, 64, 64, 5, 1)}
        out["amr"] = am
    if not args.no_extras or args.jet_only:
        print("bench: inflowing jet to 300 us", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["jet"] = {"workload": "inflowing jet: 1 cm square of sea-level air, tanh inflow of peak Mach 0.1 "
                                  "and half density at y = 0, outflow elsewhere, 4 zones periodic in z, "
                                  "FP64, to t = 300 us",
                      "n256": jet_costs(256), "n512": jet_costs(512)}
    if not args.no_extras or args.species_only:
        from paper_1008_2801_amd import inputs as I
        print("bench: passive species on the 256^3 workload", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        w2 = make_workload(args.workload)
        sp = {"workload": f"{w2.name} with passive species (mode-sum mass fractions summing to one), "
                          "fill + dt + step, 10 steps"}
        for ns in (1, 4):
            sp[f"fp64_ns{ns}"] = species_costs(w2, ns, 10, 2, precision=0)
        sp["fp32_reconstruction_ns4"] = species_costs(w2, 4, 10, 2, precision=1)
        out["species"] = sp
        del w2
    if not args.no_cpu_baseline:
        print("bench: timing the CPU reference on a window", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_window, wl.gamma)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

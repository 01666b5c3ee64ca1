#!/usr/bin/env python3
"""Throughput of the unsplit PPM step on one MI355X.

A step is one pass of the hot path over a level: ghost fill, CFL time step
on the device, and the step itself (primitive conversion, flattening, PPM
reconstruction, characteristic tracing, 12 two-shock Riemann solves per zone
with corner-transport corrections, conservative update).  The default
workload is the largest level: the 512^3 Rayleigh-Taylor set-up as 512 boxes
of 64^3 (walls in z, constant gravity, gamma 1.4), FP64, in the batched form
(every stage one launch over all boxes' tiles, whole steps captured in a HIP
graph); inputs are synthetic and seeded and are resident in HBM before
timing starts.

Prints one JSON line.  `value` is zone-updates/s (valid zones x steps / s)
of the graph form; the same level is also timed with one launch per stage
per box (`per_box`), and the ratio is `batched_over_per_box`.  `roofline`
reports the stage kernel that takes the most time, with its algorithmic FP64
flops per launch divided by its mean launch time (HIP events on the stream
the kernels run on) against the FP64 vector peak.  `cpu_baseline` times the
serial CPU reference evaluation on boxes of the same level, on one core and
on all the cores the process may use (one box per thread at a time).
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
# of the reference evaluation on windows of each workload's recipe
# (`python oracle/opcount.py cfg2|cfg5`).  Units: see stage_units().
FLOPS_PER_UNIT = {
    "cfg2": {"prim": 15.0, "flatten": 64.98, "trace": 389.28, "riemann1": 178.06,
             "riemann2": 256.06, "riemann3": 286.06, "update": 45.0},
    "cfg5": {"prim": 15.0, "flatten": 62.0, "trace": 362.75, "riemann1": 194.0,
             "riemann2": 266.86, "riemann3": 291.62, "update": 81.0},
}
STAGES = ("prim", "flatten", "trace", "riemann1", "riemann2", "riemann3", "update")
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


def record_traffic(fetch_csv, write_csv, kernel, workload, tiling, fetch_factor, write_factor, valu_csv=None):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the kernel from two
    rocprofv3 --pmc runs, times the factors a plain copy of known size gives,
    stored with the digest of the kernel sources and the tiling.  With
    valu_csv (a third run with SQ_INSTS_VALU and GRBM_GUI_ACTIVE): the
    kernel's VALU issue utilisation, SQ_INSTS_VALU x 4 cycles (a wave64 FP64
    instruction holds a 16-lane SIMD for 4 cycles) over 1024 SIMDs x the
    kernel's cycles (GRBM_GUI_ACTIVE / 8 XCDs), and the sustained clock,
    those cycles over the dispatch's duration."""
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
        # every kernel of the steps, per step: the counted dispatches over
        # the step count, which the kernel's own dispatches give.  A
        # stand-alone dt pass (k_zero_u64, k_wavespeed, k_finish_dt) is not
        # part of a step; the speed pass that the brick form runs after its
        # update is.
        rows = sorted((r for r in csv.DictReader(open(path))
                       if r["Counter_Name"] == counter and "ppm::" in r["Kernel_Name"]),
                      key=lambda r: int(r["Dispatch_Id"]))
        tot = 0.0
        for i, r in enumerate(rows):
            if "k_wavespeed" in r["Kernel_Name"] and i > 0 and "k_zero_u64" in rows[i - 1]["Kernel_Name"]:
                continue
            tot += float(r["Counter_Value"])
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
    if valu_csv:
        rows = [r for r in csv.DictReader(open(valu_csv)) if f"k_{kernel}<double>" in r["Kernel_Name"]]
        by = {}
        for r in rows:
            by.setdefault(r["Dispatch_Id"], {})[r["Counter_Name"]] = (float(r["Counter_Value"]), r)
        utils, clocks = [], []
        for d in by.values():
            if "SQ_INSTS_VALU" in d and "GRBM_GUI_ACTIVE" in d:
                cyc = d["GRBM_GUI_ACTIVE"][0] / 8.0
                utils.append(d["SQ_INSTS_VALU"][0] * 4.0 / (1024.0 * cyc))
                r0 = d["GRBM_GUI_ACTIVE"][1]
                if r0.get("Start_Timestamp") and r0.get("End_Timestamp"):
                    ns = float(r0["End_Timestamp"]) - float(r0["Start_Timestamp"])
                    if ns > 0:
                        clocks.append(cyc / ns)
        if utils:
            rec["valu_util"] = sum(utils) / len(utils)
        if clocks:
            rec["clock_ghz"] = sum(clocks) / len(clocks)
    with open(traffic_record_path(kernel, workload), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def recorded_record(kernel, workload, tiling):
    """The counter record of the kernel and workload, or None when there is
    none or the kernels or tiling changed since it was taken."""
    try:
        with open(traffic_record_path(kernel, workload)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != sources_digest() or list(rec.get("tiling", [])) != list(tiling):
        return None
    return rec


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


WORKLOADS = {
    "cfg5": "512^3 Rayleigh-Taylor level, 512 boxes of 64^3, walls in z, g = (0,0,-1), gamma 1.4, FP64",
    "cfg5-fp32": "512^3 Rayleigh-Taylor level, 512 boxes of 64^3, walls in z, g = (0,0,-1), gamma 1.4, "
                 "FP32 reconstruction + FP64 fluxes and update",
    "cfg2": "256^3 single box, gamma 5/3, random-mode density x planar Sod jump, constant velocity, periodic, FP64",
    "cfg2-fp32": "256^3 single box as cfg2, FP32 reconstruction + FP64 fluxes and update",
    "cfg2-small": "64^3 single box with cfg2's recipe, FP64",
}


def stage_units_axis(n, d):
    """riemann1's units (faces) along axis d of one box of valid extents n."""
    import numpy as np
    w = np.asarray(n, dtype=np.int64)
    e = w + 2
    return int((w[d] + 1) * np.prod([e[t] for t in range(3) if t != d]))


def make_workload(name):
    from paper_1008_2801_amd import inputs as I
    if name == "cfg5":
        return I.cfg5(precision=0)
    if name == "cfg5-fp32":
        return I.cfg5(precision=1)
    if name == "cfg2":
        return I.cfg2()
    if name == "cfg2-small":
        return I.cfg2(64)
    if name == "cfg2-fp32":
        wl = I.cfg2()  # the same level and state, FP32 reconstruction, FP64 update
        wl.precision = 1
        return wl
    raise SystemExit(f"unknown workload {name}")


def flops_table(name):
    return FLOPS_PER_UNIT["cfg5" if name.startswith("cfg5") else "cfg2"]


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


def adjoint_costs(wl, nsteps, every, reps=10, precision=0, rollout=True):
    """Per-step forward and adjoint times (the adjoint includes its own
    recompute of the forward intermediates) and the whole checkpointed
    roll-out, forward vs backward.  Per-step times are medians over `reps`
    calls, each bracketed by its own events, after two untimed calls; they
    are taken with the level's default launch configuration and again with
    the autotuned one (the headline's), which is the one the roll-out uses."""
    import numpy as np
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

    def timed(fn, before=None):
        ts = []
        for r in range(reps + 2):
            if before is not None:
                before()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if r >= 2:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def costs():
        t_fwd = timed(lambda: lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv))
        t_adj = timed(lambda: lev.hydro_step_adjoint(U, W, Ub, wl.dx, p, dt_dev=dtv))
        # the adjoint on the intermediates the forward step left in its workspace
        t_sav = timed(lambda: lev.hydro_step_adjoint(U, W, Ub, wl.dx, p, dt_dev=dtv, saved=True),
                      before=lambda: lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv))
        return t_fwd, t_adj, t_sav

    d_fwd, d_adj, d_sav = costs()
    Uf = U.clone()
    _, _, from_cache = lev.autotune(Uf, wl.dx, p, reps=2, cache_path=AUTOTUNE_CACHE)
    del Uf
    t_fwd, t_adj, t_sav = costs()
    res = {"precision": "f64" if precision == 0 else "f32 reconstruction + f64 update",
           "launch_config": launch_config(lev), "autotune_from_cache": bool(from_cache),
           "forward_step_ms": t_fwd, "adjoint_step_ms": t_adj, "adjoint_over_forward": t_adj / t_fwd,
           "adjoint_step_saved_ms": t_sav, "adjoint_saved_over_forward": t_sav / t_fwd,
           "default_launch_config": {"forward_step_ms": d_fwd, "adjoint_step_ms": d_adj,
                                     "adjoint_over_forward": d_adj / d_fwd, "adjoint_step_saved_ms": d_sav,
                                     "adjoint_saved_over_forward": d_sav / d_fwd}}
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
# (density for the fractions; flattening, normal velocity, density and
# pressure per axis, the last two for the sound speed; stage mass fluxes and
# traced densities).
SPECIES_BYTES_PER_ZONE_SPECIES = 16 + 72 + 72 + 120 + 120 + 40
SPECIES_SHARED_BYTES_PER_ZONE = 8 + 96 + 24 + 120 + 120


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, single_s=10.0, per_thread=2):
    """The serial CPU oracle on whole boxes of the same level (one box's step
    per call, each call single-threaded), first on one core for about
    single_s seconds, then on every core of the process's affinity set, one
    box per thread at a time (ctypes releases the GIL during each call).
    The ghost fill and the level's dt are the oracle's own, outside the
    timing.  A box stepped in both phases must come out bit for bit the
    same."""
    import concurrent.futures as cf
    import numpy as np
    from oracle import oracle as O
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    p = O.params(gamma=wl.gamma, grav=wl.grav, precision=wl.precision)
    dt = p.cfl / max(O.max_wavespeed(u, wl.dx, p)[0] for u in st)
    walls = [O.box_walls(lay.boxes(), lay.domain(), lay.bc, b) for b in range(lay.nbox)]
    order = [int(b) for b in np.random.default_rng(7).permutation(lay.nbox)]

    def one(b):
        out, _, _ = O.step(st[b], dt, wl.dx, p, walls=walls[b])
        return b, out

    t0 = time.perf_counter()
    k, zones1, first = 0, 0, None
    while k < lay.nbox and (k == 0 or time.perf_counter() - t0 < single_s):
        b, out = one(order[k])
        if first is None:
            first = (b, out)
        zones1 += int(np.prod(lay.n(b)))
        k += 1
    sec1 = time.perf_counter() - t0
    ncores = len(os.sched_getaffinity(0))
    nb = min(lay.nbox, ncores * per_thread)
    todo = [first[0]] + [order[(k + i) % lay.nbox] for i in range(nb - 1)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(ncores) as ex:
        res = list(ex.map(one, todo))
    secn = time.perf_counter() - t0
    zonesn = sum(int(np.prod(lay.n(b))) for b in todo)
    same = bool(np.array_equal(res[0][1], first[1]))
    return {"value": zonesn / secn, "unit": "zone-updates/s", "cores": ncores, "kind": "oracle",
            "sample": f"one step of {nb} boxes of the same level ({zonesn} zones), one box per thread on "
                      f"{ncores} threads, {secn:.1f} s wall; serial C++ reference (-O2, no contraction)",
            "single_core": {"value": zones1 / sec1, "cores": 1,
                            "sample": f"one step of {k} boxes ({zones1} zones) on one thread, {sec1:.1f} s"},
            "threads_bitwise_equal_to_serial": same, "cpu_model": cpu_model()}


def child_processes():
    """Child processes of this process still alive (none are started)."""
    try:
        import psutil
        return [c.pid for c in psutil.Process().children(recursive=True)]
    except Exception:
        return []


def algorithmic_bytes_per_step(lay):
    """HBM bytes a step must move at least: read every stored zone of U (5
    FP64 values, ghosts included), write every valid zone of U'."""
    import numpy as np
    stored = sum(int(np.prod(np.asarray(lay.n(b)) + 8)) for b in range(lay.nbox))
    return 40 * stored + 40 * lay.valid_zones()


# The final stage's launch forms (ppm_set_step_form): the staged riemann3 +
# update kernels, the brick kernel, the streamed kernel; the front end's
# (ppm_set_front_form): staged trace + riemann1, streamed along z, the x
# axis fused, every axis fused.
FINAL_FORMS = ("staged", "brick", "streamed")
FRONT_FORMS = ("staged", "streamed", "x_fused", "xyz_fused")


def launch_config(lev):
    """[tile, strip_rows, final-stage form, front-end form], then the
    streamed final stage's tile extents [x, y, z run] when that form is on
    and the streamed front end's when that one is: what the counter records
    are tied to."""
    t, s = lev.get_tiling()
    form, front = lev.get_step_form(), lev.get_front_form()
    return [t, s, form, front] + (list(lev.get_stream_tiling()) if form == 2 else []) + \
        (list(lev.get_front_tiling()) if front == 1 else [])


def apply_launch_config(lev, cfg):
    """The inverse of launch_config (a prefix of it is enough)."""
    lev.set_tiling(*cfg[:2])
    k = 4
    if len(cfg) > 2 and cfg[2] == 2 and len(cfg) >= k + 3:
        lev.set_stream_tiling(*cfg[k:k + 3])
        k += 3
    if len(cfg) > 3 and cfg[3] == 1 and len(cfg) >= k + 3:
        lev.set_front_tiling(*cfg[k:k + 3])
    if len(cfg) > 2:
        lev.set_step_form(cfg[2])
    if len(cfg) > 3:
        lev.set_front_form(cfg[3])


def headline(wl, wname, steps, warmup, per_box=True, tiling=None, autotune=True):
    """The timed level: batched eager steps with stage profiling (the
    roofline's kernel times), the same steps as one HIP-graph launch (the
    value), and one launch per stage per box."""
    import torch
    from paper_1008_2801_amd import ppm as P
    lay = wl.layout
    lev = P.Level(lay)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=wl.precision)
    lev.ensure_workspace(p.precision)
    U0 = torch.from_numpy(wl.arena).to("cuda")
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    from_cache = None
    if tiling:
        apply_launch_config(lev, tiling)
    elif autotune:
        Uf = U0.clone()
        lev.fill_boundary(Uf)
        t_, s_, from_cache = lev.autotune(Uf, wl.dx, p, reps=2, cache_path=AUTOTUNE_CACHE)
        del Uf
    tiling = launch_config(lev)
    zones = lay.valid_zones()
    out = {"tiling": {"tile": tiling[0], "strip_rows": tiling[1], "final_stage_form": FINAL_FORMS[tiling[2]],
                      "front_end_form": FRONT_FORMS[tiling[3]], "extents": tiling[4:] or None},
           "autotune": {"from_cache": None if from_cache is None else bool(from_cache),
                        "cache": os.path.relpath(AUTOTUNE_CACHE, ROOT) if from_cache is not None else None}}

    def eager(mode, prof):
        U = U0.clone()
        V = lev.new_state()
        lev.compute_dt(U, wl.dx, p, out=dtv)
        for _ in range(warmup):
            lev.fill_boundary(U, mode)
            lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, mode=mode, dt_next=dtv)
            U, V = V, U
        torch.cuda.synchronize()
        if prof:
            lev.profile_read()
            lev.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            lev.fill_boundary(U, mode)
            lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, mode=mode, dt_next=dtv)
            U, V = V, U
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        st = None
        if prof:
            lev.profile_enable(False)
            st = lev.profile_read()
        del U, V
        return sec, st

    sec_b, prof = eager(P.BATCHED, True)
    out["batched_eager"] = zones * steps / sec_b
    # the graph of `steps` whole steps [fill, step], each dt from the update
    # before it (the first from a dt pass), replayed once untimed, then timed
    A = U0.clone()
    B = lev.new_state()
    g = lev.graph(A, B, wl.dx, p, steps)
    for _ in range(max(1, warmup // max(1, steps))):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch()
    torch.cuda.synchronize()
    sec_g = time.perf_counter() - t0
    out["graph"] = zones * steps / sec_g
    out["ms_per_step"] = sec_g / steps * 1e3
    g.close()
    del A, B
    if per_box:
        sec_p, _ = eager(P.PER_BOX, False)
        out["per_box"] = zones * steps / sec_p
        out["batched_over_per_box"] = out["graph"] / out["per_box"]
    out["flags"] = lev.check_status()
    lev.close()
    lev._work = None
    del U0, lev
    torch.cuda.empty_cache()
    return out, prof, tiling


def roofline(wname, lay, prof, ms_step, precision, tiling):
    """The dominant stage kernel's algorithmic flop rate against the vector
    peak of its precision, with the recorded counter figures of the same
    kernel and workload (null once the kernel sources or the tiling
    changed since the counters were taken), and the step's HBM figures."""
    units = {k: 0 for k in STAGES}
    for b in range(lay.nbox):
        for k, v in stage_units(lay.n(b)).items():
            units[k] += v
    table = flops_table(wname)
    # with a fused final stage (brick or streamed form) one kernel does the
    # riemann3 and update work, timed in the riemann3 slot.  The fused front
    # ends are timed in the trace slot: form 2 (x fused) holds the x axis's
    # riemann1 work there, the riemann1 slot the y and z axes'; forms 1 and 3
    # hold all of it there
    fused = len(tiling) > 2 and tiling[2] != 0
    front = tiling[3] if len(tiling) > 3 else 0
    stages = {k: prof[k] for k in STAGES if not (fused and k == "update") and not (front in (1, 3) and k == "riemann1")}
    flops_of = {k: table[k] * units[k] for k in stages}
    if fused:
        flops_of["riemann3"] += table["update"] * units["update"]
    if front in (1, 3):
        flops_of["trace"] += table["riemann1"] * units["riemann1"]
    elif front == 2:
        ux = sum(stage_units_axis(lay.n(b), 0) for b in range(lay.nbox))
        flops_of["trace"] += table["riemann1"] * ux
        flops_of["riemann1"] -= table["riemann1"] * ux
    dom = max(stages, key=lambda k: stages[k][0])
    t_ms, cnt = stages[dom]
    mean_s = t_ms / cnt / 1e3
    flops = flops_of[dom]
    achieved = flops / mean_s / 1e12
    peak = FP64_VECTOR_PEAK_TFLOPS if precision == 0 else FP32_VECTOR_PEAK_TFLOPS
    rec = recorded_record(dom, wname, tiling) if precision == 0 else None
    step_flops = sum(table[k] * units[k] for k in STAGES)
    alg = algorithmic_bytes_per_step(lay)
    name = dom
    if fused and dom == "riemann3":
        name = ("final_update (riemann3 + update, brick form)" if tiling[2] == 1 else
                "final_stream (riemann3 + update, streamed form)")
    elif front and dom == "trace":
        name = f"trace slot ({FRONT_FORMS[front]} front end: its fused kernels and any staged trace)"
    elif front == 2 and dom == "riemann1":
        name = "riemann1 (y and z axes)"
    r = {"bound": "alu", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
         "frac": achieved / peak,
         "traffic": rec.get("traffic_bytes_per_launch") if rec else None,
         "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
         "mean_launch_ms": mean_s * 1e3, "flops_per_launch": flops,
         "flops_per_unit": table[dom] if name == dom else None,
         "units_per_launch": units[dom] if name == dom else None,
         "clock_ghz": rec.get("clock_ghz") if rec else None,
         "valu_issue_util": rec.get("valu_util") if rec else None,
         "step_traffic": rec.get("step_traffic_bytes") if rec else None,
         "step_traffic_GBps": (rec["step_traffic_bytes"] / (ms_step / 1e3) / 1e9
                               if rec and rec.get("step_traffic_bytes") else None),
         "step_flop_rate_tflops": step_flops / (ms_step / 1e3) / 1e12,
         "hbm": {"algorithmic_bytes_per_step": alg, "achieved_GBps": alg / (ms_step / 1e3) / 1e9,
                 "peak_GBps": HBM_PEAK_GBS, "frac": alg / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS}}
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="single-core oracle sample length")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiling")
    ap.add_argument("--no-per-box", action="store_true", help="skip the one-launch-per-box timing")
    ap.add_argument("--autotune-cache", default=None,
                    help="autotuner cache file (default: the package's autotune_cache.jsonl)")
    ap.add_argument("--tiling", default=None,
                    help="'tile,strip_rows[,final[,front[,x,y,z[,x,y,z]]]]': use this launch configuration "
                         "(tiling; final-stage form 0 staged / 1 brick / 2 streamed; front-end form 0 staged / "
                         "1 streamed / 2 x fused / 3 all fused; the streamed forms' tile extents) instead of "
                         "autotuning")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (single box, 512-box tiling, adjoint, two-level, jet, species)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only measure the adjoint/forward cost on the 128^3 differentiation workload")
    ap.add_argument("--amr-only", action="store_true",
                    help="with --no-extras: still measure the two-level hierarchy")
    ap.add_argument("--jet-only", action="store_true",
                    help="with --no-extras: still run the inflowing jet to 300 us")
    ap.add_argument("--species-only", action="store_true",
                    help="with --no-extras: still measure the passive-species step")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter record of the dominant kernel from two rocprofv3 --pmc "
                         "counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--record-valu", default=None, metavar="VALU_CSV",
                    help="with --record-traffic: a counter_collection.csv with SQ_INSTS_VALU, "
                         "SQ_BUSY_CYCLES and GRBM_GUI_ACTIVE of the same command")
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
        record_traffic(args.record_traffic[0], args.record_traffic[1], args.record_kernel, args.workload,
                       [int(v) for v in args.tiling.split(",")], ff, wf, args.record_valu)
        return

    import torch

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
    print(f"bench: workload {args.workload}: {lay.nbox} box(es), {lay.valid_zones()} valid zones", file=sys.stderr,
          flush=True)
    tiling = tuple(int(v) for v in args.tiling.split(",")) if args.tiling else None
    h, prof, tiling = headline(wl, args.workload, args.steps, args.warmup, per_box=not args.no_per_box,
                               tiling=tiling, autotune=not args.no_autotune)
    zones = lay.valid_zones()
    print(f"bench: {args.workload} graph {h['graph']:.4g} zone-updates/s ({h['ms_per_step']:.3f} ms/step)",
          file=sys.stderr, flush=True)
    rf = roofline(args.workload, lay, prof, h["ms_per_step"], wl.precision, tiling)
    out = {
        "metric": METRIC, "value": h["graph"], "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if wl.precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}; batched step (one launch per "
                               "stage over all boxes' tiles), [fill, step] x steps captured in one HIP graph, "
                               "each step's CFL dt left on the device by the previous step's update",
                   "valid_zones": zones, "boxes": lay.nbox, "tiling": h["tiling"], "autotune": h["autotune"]},
        "batched_eager": h["batched_eager"],
        "per_box": h.get("per_box"), "batched_over_per_box": h.get("batched_over_per_box"),
        "roofline": rf,
        "stage_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items()},
        "hbm_copy_GBps": copy_bandwidth(),
        "status_flags": h["flags"],
    }
    if not args.no_extras:
        from paper_1008_2801_amd import inputs as I
        print("bench: 256^3 single box (FP64)", file=sys.stderr, flush=True)
        w2 = I.cfg2()
        r2, p2, t2 = headline(w2, "cfg2", 20, 2, per_box=False)
        r2["roofline"] = roofline("cfg2", w2.layout, p2, r2["ms_per_step"], 0, t2)
        r2["workload"] = "cfg2: " + WORKLOADS["cfg2"]
        out["single_box_256"] = r2
        del w2
        print("bench: 512-box tensor tiling (batched / per-box / graph)", file=sys.stderr, flush=True)
        w3 = I.cfg3()
        extra = {"workload": f"cfg3: 512 boxes, edges from {{16,24,32,48,64}} (seed 3), "
                             f"{w3.layout.valid_zones()} valid zones, gamma 1.4, periodic, 20 steps",
                 "unit": "zone-updates/s"}
        for prec, tag in ((0, "fp64"), (1, "fp32_reconstruction")):
            r = level_rates(w3, 20, 2, prec)
            extra[tag] = r
            extra[tag]["batched_over_per_box"] = r["batched"] / r["per_box"]
        out["multibox"] = extra
        print("bench: the same 512^3 level, FP32 reconstruction", file=sys.stderr, flush=True)
        w5 = I.cfg5(precision=1)
        r5, p5, t5 = headline(w5, "cfg5-fp32", args.steps, args.warmup, per_box=False)
        r5["workload"] = "cfg5-fp32: " + WORKLOADS["cfg5-fp32"]
        out["fp32_reconstruction"] = r5
        print("bench: adjoint step of the 512^3 level (FP32 reconstruction)", file=sys.stderr, flush=True)
        a5 = adjoint_costs(w5, 0, 1, precision=1, rollout=False)
        a5["workload"] = "cfg5: 512 boxes of 64^3, FP32 reconstruction, one forward step vs one adjoint step"
        out["adjoint_512cubed_fp32"] = a5
        del w5
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
        a5["workload"] = ("Rayleigh-Taylor instance: 8 boxes of 64^3 (128^3), g = (0,0,-1), walls in z, "
                          "FP64, 10 steps")
        out["adjoint_rayleigh_taylor"] = a5
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
        w2 = I.cfg2()
        sp = {"workload": "cfg2 with passive species (mode-sum mass fractions summing to one), "
                          "fill + dt + step, 10 steps"}
        for ns in (1, 4):
            sp[f"fp64_ns{ns}"] = species_costs(w2, ns, 10, 2, precision=0)
        sp["fp32_reconstruction_ns4"] = species_costs(w2, 4, 10, 2, precision=1)
        out["species"] = sp
        del w2
    if not args.no_cpu_baseline:
        print("bench: timing the CPU reference on boxes of the level", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, single_s=args.cpu_seconds)
    kids = child_processes()
    if kids:
        print(f"bench: child processes still alive: {kids}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

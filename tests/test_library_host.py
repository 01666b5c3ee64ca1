"""Host-side logic of the library (no GPU): the C ABI loads and exports every
declared symbol; the hash-sorted fill plan equals the all-pairs plan and,
executed on the host, reproduces the oracle's ghost fill (inflow faces
included); the plan cache is hit on repeated layouts; invalid layouts are
rejected."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1008_2801_amd import inputs as I
from paper_1008_2801_amd import ppm as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="ppm.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ppm_[a-z_0-9]+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 17
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.SYMBOLS)


def test_diagnostics_library_exports_its_declared_symbols():
    """The arithmetic diagnostics live in a library of their own
    (include/ppm_diag.h, libppm_diag.so), outside the step's ABI."""
    names = declared_functions("ppm_diag.h")
    assert set(names) == set(P.DIAG_SYMBOLS)
    L = P.diag_lib()
    for n in names:
        assert hasattr(L, n), n
    assert not set(names) & set(P.SYMBOLS)


def _layouts():
    rng = np.random.default_rng(3)
    out = [I.cfg3_layout()[0],
           I.tensor_tiling([16] * 4, [16] * 4, [16] * 4, bc=(0, 0, 0, 0, 2, 2)),
           I.single_box(8)]
    for bc in [(1, 1, 0, 0, 2, 2), (2, 2, 1, 1, 0, 0), (1, 1, 1, 1, 1, 1)]:
        out.append(I.tensor_tiling(rng.integers(4, 9, 3), rng.integers(4, 9, 4), rng.integers(4, 9, 2), bc=bc))
    return out


@pytest.mark.parametrize("k", range(6))
def test_hash_sorted_plan_equals_all_pairs_plan(k):
    lay = _layouts()[k]
    a = P.plan_build(lay)
    b = P.plan_build(lay, brute=True)
    assert np.array_equal(a, b)
    # every ghost zone of every box is written exactly once
    assert a[:, 15].sum() == lay.stored_zones() - lay.valid_zones()


@pytest.mark.parametrize("k", range(1, 6))
def test_plan_executed_on_host_equals_oracle_fill(k):
    lay = _layouts()[k]
    rng = np.random.default_rng(k)
    arena = np.full(lay.arena_len(), np.nan)
    for b in range(lay.nbox):
        v = lay.view(arena, b)
        g = 4
        v[:, g:-g, g:-g, g:-g] = rng.normal(size=v[:, g:-g, g:-g, g:-g].shape)
    mine = P.fill_boundary_host(lay, arena.copy())
    st = [lay.view(arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    for b in range(lay.nbox):
        assert np.array_equal(lay.view(mine, b), st[b])


def test_plan_cache_hits_on_repeated_layout():
    lay = I.tensor_tiling([5, 6], [7, 4], [4, 9])
    l0, h0, _ = P.plan_cache_stats()
    P.plan_build(lay)
    P.plan_build(lay)
    l1, h1, e1 = P.plan_cache_stats()
    # plan_build queries twice (count, then descriptors): 4 lookups, 3 hits
    assert l1 - l0 == 4 and h1 - h0 == 3 and e1 >= 1


@pytest.mark.parametrize("lo,hi,dom,bc", [
    ([[0, 0, 0], [2, 0, 0]], [[3, 3, 3], [5, 3, 3]], ((0, 0, 0), (5, 3, 3)), (0,) * 6),   # overlap
    ([[0, 0, 0]], [[3, 3, 3]], ((0, 0, 0), (4, 3, 3)), (0,) * 6),                          # gap
    ([[0, 0, 0]], [[3, 3, 3]], ((0, 0, 0), (3, 3, 3)), (0, 1, 0, 0, 0, 0)),                # half periodic
    ([[0, 0, 0]], [[2, 3, 3]], ((0, 0, 0), (2, 3, 3)), (0,) * 6),                          # extent < 4
])
def test_invalid_layouts_rejected(lo, hi, dom, bc):
    lay = I.Layout(np.array(lo), np.array(hi), dom[0], dom[1], bc)
    with pytest.raises(P.PPMError):
        P.plan_build(lay)


def test_box_beyond_32_bit_zone_indices_rejected():
    """Zone indices within a box, ghost layers included, are 32-bit: a box
    of 1283^3 zones (1291^3 > 2^31 with its ghosts) is refused before any
    work, while a thinner box of the same face area passes."""
    big = I.Layout(np.array([[0, 0, 0]]), np.array([[1282, 1282, 1282]]), (0, 0, 0), (1282, 1282, 1282), (0,) * 6)
    with pytest.raises(P.PPMError):
        P.plan_build(big)
    thin = I.Layout(np.array([[0, 0, 0]]), np.array([[1282, 1282, 7]]), (0, 0, 0), (1282, 1282, 7), (0,) * 6)
    P.plan_build(thin)


def test_empty_layout_rejected():
    """A level without boxes has nothing to advance: the library refuses it
    (PPM_EINVAL, "no boxes") rather than building an empty plan."""
    none = np.zeros((0, 3), dtype=np.int64)
    lay = I.Layout(none, none, (0, 0, 0), (3, 3, 3), (0,) * 6)
    with pytest.raises(P.PPMError):
        P.plan_build(lay)


def _apply_plan(lay, desc, arena, inflow):
    """Execute fill descriptors (ndesc, 20) in numpy: copies between boxes,
    and for src < 0 the prescribed state of the inflow face -1 - src."""
    g = 4
    ext = [lay.domain_hi[d] - lay.domain_lo[d] + 1 for d in range(3)]
    for D in desc:
        dst, src = int(D[0]), int(D[1])
        lo, hi, a, c, sign = D[2:5], D[5:8], D[8:11], D[11:14], int(D[14])
        rng = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
        s = [a[d] * rng[d] + c[d] for d in range(3)]
        dv = lay.view(arena, dst)
        di = np.ix_(rng[2] + g, rng[1] + g, rng[0] + g)
        if src >= 0:
            sv = lay.view(arena, src)
            vals = sv[(slice(None),) + np.ix_(s[2] + g, s[1] + g, s[0] + g)]
        else:
            f = -1 - src
            d = f // 2
            t1, t2 = [x for x in range(3) if x != d]
            F = inflow[f].reshape(5, ext[t2], ext[t1])
            # broadcast the face state over the region (constant along d)
            grids = np.meshgrid(s[2], s[1], s[0], indexing="ij")
            vals = F[:, grids[2 - t2], grids[2 - t1]]
        vals = vals.copy()
        for m in range(3):
            if (sign >> m) & 1:
                vals[1 + m] = -vals[1 + m]
        dv[(slice(None),) + di] = vals
    return arena


@pytest.mark.parametrize("which", ["jet", "boxes_reflect"])
def test_inflow_plan_equals_oracle_fill(which):
    """The plan's inflow descriptors (negative source), executed on the host,
    reproduce the oracle's fill of an inflow face, edges and corners
    included (outflow clamp, reflecting mirror with sign, periodic wrap)."""
    if which == "jet":
        wl = I.jet(16, nz=4)
        lay, inflow = wl.layout, wl.meta["inflow"]
        arena = wl.arena.copy()
    else:
        lay = I.tensor_tiling([5, 7], [6, 4, 5], [4, 6],
                              bc=(I.BC_REFLECT, I.BC_OUTFLOW, I.BC_INFLOW, I.BC_OUTFLOW, I.BC_PERIODIC,
                                  I.BC_PERIODIC))
        rng = np.random.default_rng(9)
        arena = np.full(lay.arena_len(), np.nan)
        for b in range(lay.nbox):
            v = lay.view(arena, b)
            v[:, 4:-4, 4:-4, 4:-4] = rng.normal(size=v[:, 4:-4, 4:-4, 4:-4].shape)
        inflow = {2: rng.normal(size=(5, 10, 12))}
    desc = P.plan_build(lay)
    assert (desc[:, 1] < 0).any()
    assert desc[:, 15].sum() == lay.stored_zones() - lay.valid_zones()
    mine = _apply_plan(lay, desc, arena.copy(), inflow)
    st = [lay.view(arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st, inflow=inflow)
    for b in range(lay.nbox):
        assert np.array_equal(lay.view(mine, b), st[b])
    # the host executor of the library refuses a layout with an inflow face
    with pytest.raises(P.PPMError):
        P.fill_boundary_host(lay, arena.copy())


def test_traffic_record_follows_the_code_not_the_comments(tmp_path, monkeypatch):
    """bench.py reports recorded counter traffic only while the kernel
    sources' code and the tiling are those it was taken with: a changed
    comment keeps the record, a changed line of code or another tiling
    drops it."""
    import shutil
    import bench
    for f in bench.TRAFFIC_SOURCES:
        (tmp_path / os.path.dirname(f)).mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), tmp_path / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.sources_digest()
    rec = {"tiling": [256, 32], "sources_sha256": d0, "traffic_bytes_per_launch": 123.0}
    with open(bench.traffic_record_path("riemann2", "cfg2"), "w") as fh:
        json.dump(rec, fh)
    assert bench.recorded_traffic("riemann2", "cfg2", (256, 32)) == 123.0
    assert bench.recorded_traffic("riemann2", "cfg2", (128, 0)) is None
    src = tmp_path / bench.TRAFFIC_SOURCES[1]
    text = src.read_text()
    src.write_text("// a new comment line\n" + text.replace("\n", "\n/* block */\n", 1) + "\n\n")
    assert bench.sources_digest() == d0
    assert bench.recorded_traffic("riemann2", "cfg2", (256, 32)) == 123.0
    src.write_text(text + "\nconstexpr int unused_value = 1;\n")
    assert bench.sources_digest() != d0
    assert bench.recorded_traffic("riemann2", "cfg2", (256, 32)) is None


def test_roofline_flop_figures_are_the_op_counting_oracles():
    """bench.py prices the stage kernels with per-unit flop counts; they
    must be the op-counting oracle's on the 256^3 and 512^3 workloads'
    recipes (to the two decimals stored), and bench's units per stage must
    be the oracle's definitions, so that the reported roofline rests on
    counted work."""
    import bench
    from oracle import opcount
    for wl in ("cfg2", "cfg5"):
        flops, _, _ = opcount.measure(wl)
        assert set(bench.FLOPS_PER_UNIT[wl]) == set(bench.STAGES)
        for k, v in bench.FLOPS_PER_UNIT[wl].items():
            assert abs(v - flops[k]) <= 0.006, (wl, k, v, flops[k])
    for n in ((256, 256, 256), (16, 24, 8), (1, 3, 5)):
        assert bench.stage_units(n) == opcount.units(n), n


def test_roofline_prices_fused_slots_by_their_kernels_work():
    """bench.py's roofline: with the x-fused front end the trace slot holds
    the tracing plus the x axis's stage-1 solves and the riemann1 slot the y
    and z solves; with a fused final stage the riemann3 slot holds the
    update's work too; the staged forms price each slot by its own stage."""
    import bench
    from paper_1008_2801_amd import inputs as I
    lay = I.cfg5(nb=2, m=8).layout
    table = bench.flops_table("cfg5")
    units = {k: 0 for k in bench.STAGES}
    ux = 0
    for b in range(lay.nbox):
        for k, v in bench.stage_units(lay.n(b)).items():
            units[k] += v
        ux += bench.stage_units_axis(lay.n(b), 0)
    assert ux * 3 == units["riemann1"]  # cubes: the same faces per axis

    def prof(**ms):
        return {k: (ms.get(k, 1.0), 1) for k in bench.STAGES}
    # staged: riemann2 dominant, priced alone
    r = bench.roofline("cfg5", lay, prof(riemann2=9.0), 20.0, 0, [256, 0, 0, 0])
    assert r["kernel"] == "riemann2" and r["flops_per_launch"] == table["riemann2"] * units["riemann2"]
    # x-fused front end, its slot dominant: tracing + the x axis's solves
    r = bench.roofline("cfg5", lay, prof(trace=9.0), 20.0, 0, [256, 0, 0, 2])
    assert r["kernel"].startswith("trace slot")
    assert abs(r["flops_per_launch"] - (table["trace"] * units["trace"] + table["riemann1"] * ux)) < 1e-3
    # x-fused front end, the riemann1 slot dominant: the y and z solves only
    r = bench.roofline("cfg5", lay, prof(riemann1=9.0), 20.0, 0, [256, 0, 0, 2])
    assert r["kernel"].startswith("riemann1")
    assert abs(r["flops_per_launch"] - table["riemann1"] * (units["riemann1"] - ux)) < 1e-3
    # brick final stage dominant: riemann3 + update
    r = bench.roofline("cfg5", lay, prof(riemann3=9.0), 20.0, 0, [256, 0, 1, 2])
    assert r["kernel"].startswith("final_update")
    assert abs(r["flops_per_launch"] - (table["riemann3"] * units["riemann3"] +
                                        table["update"] * units["update"])) < 1e-3


def test_zone_index_division_multipliers_give_integer_division():
    """The kernels decode zone indices (below 2^31) by a high multiply and a
    shift with multipliers the library forms per divisor; checked against
    Python's integer division for small, random, power-of-two-adjacent and
    the largest divisors, at dividends around every multiple's edge."""
    rng = np.random.default_rng(31)
    divisors = list(range(2, 600)) + [2 ** k + e for k in range(1, 31) for e in (-1, 0, 1) if 2 <= 2 ** k + e < 2 ** 31]
    divisors += [int(v) for v in rng.integers(2, 2 ** 31, size=300)] + [2 ** 31 - 1]
    top = 2 ** 31 - 1
    for d in divisors:
        m, sh = P.div31_params(d)
        assert 0 < m < 2 ** 32 and sh >= 0
        ns = {0, 1, d - 1, d, d + 1, top, top - 1, top // d * d, top // d * d - 1}
        ns.update(int(v) for v in rng.integers(0, 2 ** 31, size=40))
        ns.update(k * d + e for k in (1, 2, 3, 7, 1000, top // d) for e in (-1, 0, 1))
        for n in ns:
            if 0 <= n <= top:
                assert ((n * m) >> 32) >> sh == n // d, (d, n, m, sh)
    for bad in (0, 1, 2 ** 31):
        with pytest.raises(P.PPMError):
            P.div31_params(bad)

"""GPU parity: the HIP path through the C ABI against the oracle on the same
seeded inputs.  FP64 bar: per-field max |gpu - oracle| / max |oracle| <= 1e-12.
The kernels evaluate reciprocal forms of the method's divisions and the
oracle the plain definition, so the two agree to rounding; every comparison
prints its per-field errors and how many values differ in their bits."""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1008_2801_amd import inputs as I  # noqa: E402
from paper_1008_2801_amd import ppm as P  # noqa: E402
from tests.helpers import dts_close, interior, field_errors, parity_report, rescaled  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12
# FP32-reconstruction mode against the oracle's FP32 mode: both round every
# reconstruction, tracing and Riemann operation to FP32 (unit roundoff
# 6e-8) in differently arranged formulas, and the update adds dt/h times
# flux differences of that accuracy to the FP64 state.  Where the step
# cancels large terms (a hydrostatic column) or starts from rest (the
# tracing then picks waves by the sign of FP32 rounding noise), the two
# differ by as much as the FP32 mode differs from FP64 itself: a few 1e-6.
FP32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def gpu_run(wl, nsteps, mode=P.BATCHED, fluxes=False, dt=None, tiling=None, **pk):
    """nsteps of [fill, dt, step] on the GPU; returns (level, host arena, dts, flags, last fluxes)."""
    lev = P.Level(wl.layout)
    if tiling is not None:
        lev.set_tiling(*tiling)
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=wl.precision, **pk)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    dts, F = [], None
    for _ in range(nsteps):
        lev.fill_boundary(U, mode)
        if dt is None:
            lev.compute_dt(U, wl.dx, p, out=dtv)
        else:
            dtv[0] = dt
        F = lev.new_fluxes() if fluxes else None
        lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, fluxes=F, mode=mode)
        dts.append(float(dtv[0].item()))
        U, V = V, U
    flags = lev.check_status()
    return lev, U.cpu().numpy(), dts, flags, F


def oracle_run(wl, nsteps, dt=None, fluxes=False, **pk):
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    p = O.params(gamma=wl.gamma, grav=wl.grav, precision=wl.precision, **pk)
    return O.advance(lay.boxes(), lay.domain(), lay.bc, st, nsteps, wl.dx, p, dt=dt, fluxes=fluxes)


def compare_level(wl, arena, ostates, tol=TOL, tag=None):
    """Parity of a whole level's valid zones against the oracle's states,
    per field over all boxes; returns (worst field error, differing values)."""
    pairs = [(interior(wl.layout.view(arena, b)), interior(ostates[b])) for b in range(wl.layout.nbox)]
    err, nbits = parity_report(tag or wl.name, pairs, tol)
    return float(err.max()), nbits


def test_cfg1_full_run_matches_oracle():
    """32^3 advected wave, 10 steps at CFL 0.5 (the small configuration)."""
    wl = I.cfg1()
    _, arena, dts, flags, _ = gpu_run(wl, 10)
    ost, odts, ofl, _ = oracle_run(wl, 10)
    assert flags == 0 and ofl == 0
    assert dts_close(dts, odts)
    compare_level(wl, arena, ost, tag="cfg1 32^3, 10 steps")


@pytest.mark.parametrize("limiter,iters", [(1, 3), (0, 3), (1, 0), (1, 8)])
def test_scheme_options_match_oracle(limiter, iters):
    # the unlimited scheme is for smooth data (at the Sod jump it overshoots
    # into negative pressures and the run collapses): the smooth state of
    # the differentiation workload for limiter 0, the Sod recipe otherwise
    wl = I.cfg4(24) if limiter == 0 else I.cfg2(24)
    _, arena, dts, flags, _ = gpu_run(wl, 3, limiter=limiter, riemann_iters=iters)
    ost, odts, ofl, _ = oracle_run(wl, 3, limiter=limiter, riemann_iters=iters)
    assert dts_close(dts, odts) and flags == ofl
    compare_level(wl, arena, ost, tag=f"24^3, limiter {limiter}, {iters} Newton steps, 3 steps")


def test_fluxes_match_oracle():
    wl = I.cfg2(20)
    lev, arena, dts, flags, F = gpu_run(wl, 1, fluxes=True)
    ost, odts, ofl, OF = oracle_run(wl, 1, fluxes=True)
    for d in range(3):
        parity_report(f"20^3 fluxes along axis {d}", [(lev.flux_view(F[d], d, 0).cpu().numpy(), OF[0][d])], TOL,
                      state=False)


@pytest.mark.parametrize("bc", [(0, 0, 0, 0, 0, 0), (0, 0, 0, 0, 2, 2), (1, 1, 2, 2, 0, 0)])
def test_fill_matches_oracle_fill_bitwise(bc):
    rng = np.random.default_rng(12)
    lay = I.tensor_tiling(rng.integers(4, 11, 3), rng.integers(4, 11, 2), rng.integers(4, 11, 3), bc=bc)
    arena = rng.normal(size=lay.arena_len())
    lev = P.Level(lay)
    for mode in (P.BATCHED, P.PER_BOX):
        U = torch.from_numpy(arena).cuda()
        lev.fill_boundary(U, mode)
        g = U.cpu().numpy()
        st = [lay.view(arena, b).copy() for b in range(lay.nbox)]
        O.fill(lay.boxes(), lay.domain(), lay.bc, st)
        for b in range(lay.nbox):
            assert np.array_equal(lay.view(g, b), st[b])


def _uneven_level(seed=5, bc=(0, 0, 0, 0, 0, 0), sizes=(8, 12, 16)):
    rng = np.random.default_rng(seed)
    lay = I.tensor_tiling(rng.choice(sizes, 3), rng.choice(sizes, 2), rng.choice(sizes, 2), bc=bc)
    L = tuple((np.array(lay.domain_hi) + 1) / 64.0)
    S = [I.ModeSum(rng, 6, 3, L) for _ in range(5)]

    def prim(x, y, z):
        return (1.25 + 0.75 * S[0](x, y, z), 0.5 * S[1](x, y, z), 0.5 * S[2](x, y, z), 0.5 * S[3](x, y, z),
                1.25 + 0.75 * S[4](x, y, z))
    h = (1.0 / 64,) * 3
    return I.Workload("uneven", lay, I._fill_state(lay, h, 1.4, prim), h, 1.4, 2)


def test_multibox_batched_and_per_box_match_oracle_and_each_other():
    wl = _uneven_level()
    _, a_b, dts_b, fl_b, _ = gpu_run(wl, 2, mode=P.BATCHED)
    _, a_p, dts_p, fl_p, _ = gpu_run(wl, 2, mode=P.PER_BOX)
    assert np.array_equal(a_b, a_p) or np.array_equal(np.nan_to_num(a_b), np.nan_to_num(a_p))
    ost, odts, ofl, _ = oracle_run(wl, 2)
    assert dts_close(dts_b, odts)
    compare_level(wl, a_b, ost, tag="uneven multi-box level, 2 steps")


def test_reflecting_walls_and_gravity_match_oracle():
    wl = _uneven_level(seed=7, bc=(0, 0, 0, 0, 2, 2))
    wl.grav = (0.0, 0.0, -1.0)
    _, arena, dts, flags, _ = gpu_run(wl, 2)
    ost, odts, ofl, _ = oracle_run(wl, 2)
    assert dts_close(dts, odts) and flags == ofl == 0
    compare_level(wl, arena, ost, tag="walls + gravity, 2 steps")


def test_fp32_reconstruction_matches_oracle_fp32_mode():
    wl = I.cfg1(16)
    wl.precision = 1
    _, arena, dts, flags, _ = gpu_run(wl, 3)
    ost, odts, ofl, _ = oracle_run(wl, 3)
    compare_level(wl, arena, ost, tol=FP32_TOL, tag="FP32 mode vs the oracle's FP32 mode, 3 steps")
    wl.precision = 0
    o64, _, _, _ = oracle_run(wl, 3)
    err = max(field_errors(interior(wl.layout.view(arena, 0)), interior(o64[0])))
    assert err < 1e-5
    print(f"fp32 mode vs fp64 oracle: {err:.3e}")


def test_uniform_state_preserved_bitwise_on_gpu():
    wl = I.uniform(12, rho=1.7, vel=(0.4, -0.3, 0.2), p=0.6)
    _, arena, _, flags, _ = gpu_run(wl, 3)
    assert flags == 0
    assert np.array_equal(interior(wl.layout.view(arena, 0)), interior(wl.layout.view(wl.arena, 0)))


def test_conservation_on_gpu():
    wl = _uneven_level(seed=9)
    _, arena, _, flags, _ = gpu_run(wl, 3)
    for c in range(5):
        s0 = math.fsum(np.concatenate([interior(wl.layout.view(wl.arena, b))[c].ravel()
                                       for b in range(wl.layout.nbox)]))
        s1 = math.fsum(np.concatenate([interior(wl.layout.view(arena, b))[c].ravel()
                                       for b in range(wl.layout.nbox)]))
        sc = math.fsum(np.abs(np.concatenate([interior(wl.layout.view(wl.arena, b))[c].ravel()
                                              for b in range(wl.layout.nbox)])))
        assert abs(s1 - s0) <= 1e-13 * sc


def test_graph_replay_matches_eager_steps():
    """Two captured steps A -> B -> A, replayed three times with eager work and
    synchronisation in between; every replay equals two eager steps."""
    wl = I.cfg2(16)
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma)
    A = torch.from_numpy(wl.arena).cuda()
    B = lev.new_state()
    g = lev.graph(A, B, wl.dx, p, 2)
    cur = wl.arena.copy()
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        got = A.cpu().numpy()
        ref = gpu_run(I.Workload(wl.name, wl.layout, cur.copy(), wl.dx, wl.gamma, 2), 2)[1]
        assert np.array_equal(interior(wl.layout.view(got, 0)), interior(wl.layout.view(ref, 0))), rep
        cur = got.copy()
    g.close()


def test_nan_poisoned_workspace_does_not_leak():
    wl = I.cfg2(16)
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma)
    lev.ensure_workspace(0)
    lev._work.view(torch.uint8).fill_(0xFF)  # all-ones bytes: NaN doubles everywhere
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    lev.fill_boundary(U)
    dtv = lev.compute_dt(U, wl.dx, p)
    lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv)
    got = V.cpu().numpy()
    _, ref, _, _, _ = gpu_run(wl, 1)
    assert np.array_equal(interior(wl.layout.view(got, 0)), interior(wl.layout.view(ref, 0)))
    assert lev.check_status() == 0


def test_runs_are_deterministic():
    wl = _uneven_level(seed=11)
    a = gpu_run(wl, 2)[1]
    b = gpu_run(wl, 2)[1]
    assert np.array_equal(np.nan_to_num(a), np.nan_to_num(b))


def test_invalid_arguments_are_rejected():
    wl = I.cfg1(8)
    lev = P.Level(wl.layout)
    p = P.params(gamma=1.4)
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    with pytest.raises(P.PPMError):
        lev.hydro_step(U, U, wl.dx, p, dt=0.01)          # in place
    with pytest.raises(P.PPMError):
        lev.hydro_step(U, V, wl.dx, p, dt=-1.0)          # dt <= 0
    with pytest.raises(P.PPMError):
        lev.hydro_step(U, V, wl.dx, P.params(gamma=1.0), dt=0.01)
    with pytest.raises(P.PPMError):
        lev.hydro_step(U, V, (0.1, 0.0, 0.1), p, dt=0.01)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PPMError):                       # the next dt needs a cfl in (0, 1)
        lev.hydro_step(U, V, wl.dx, P.params(gamma=1.4, cfl=1.5), dt=0.01, dt_next=dtv)
    with pytest.raises(P.PPMError):                       # two doubles for the next dt
        lev.hydro_step(U, V, wl.dx, p, dt=0.01, dt_next=dtv[:1])
    lev.ensure_workspace(0)
    rc = P.lib().ppm_hydro_step_dt(lev.ctx, P._ptr(U), P._ptr(V), None, 0.01, None, P._dp3(*wl.dx),
                                   ctypes.byref(p), P.BATCHED, None, None)
    assert rc != 0                                        # null dt_next_dev
    bad = I.Layout(np.array([[0, 0, 0], [2, 0, 0]]), np.array([[3, 3, 3], [5, 3, 3]]), (0, 0, 0), (5, 3, 3))
    with pytest.raises(P.PPMError):
        P.Level(bad)


def test_nonphysical_input_raises_flag():
    wl = I.cfg1(8)
    U0 = wl.arena.copy()
    lay = wl.layout
    v = lay.view(U0, 0)
    v[0, 6, 6, 6] = -1.0
    wl2 = I.Workload("bad", lay, U0, wl.dx, wl.gamma, 1)
    _, _, _, flags, _ = gpu_run(wl2, 1, dt=1e-3)
    assert flags & P.FLAG_NONPHYS


# --------------------------------------------------- full-size sampling ----
def _sample_windows(n, rng, k, w=2):
    out = []
    for _ in range(k):
        lo = tuple(int(rng.integers(0, n[d] - w + 1)) for d in range(3))
        out.append((lo, tuple(v + w - 1 for v in lo)))
    # corners and the jump planes of the Sod set-up
    out.append(((0, 0, 0), (1, 1, 1)))
    out.append(((n[0] - 2, n[1] - 2, n[2] - 2), (n[0] - 1, n[1] - 1, n[2] - 1)))
    out.append(((n[0] // 2 - 1, 5, 9), (n[0] // 2, 6, 10)))
    return out


def test_cfg2_full_size_sampled_windows():
    """256^3 FP64, one step as bench.py runs it (its update also leaving the
    next dt); the oracle recomputes sampled windows of the output one by
    one and the next dt over the whole output; the whole output is checked
    for conservation."""
    wl = I.cfg2()
    lev, arena, dts, flags, _ = gpu_run(wl, 1)
    assert flags == 0
    lev.close()
    # the same step with the next dt from the update: the same state, and
    # the oracle's CFL dt of it, bit for bit
    lev = P.Level(wl.layout)
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    pg = P.params(gamma=wl.gamma)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    lev.fill_boundary(U)
    lev.compute_dt(U, wl.dx, pg, out=dtv)
    lev.hydro_step(U, V, wl.dx, pg, dt_dev=dtv, dt_next=dtv)
    nxt = float(dtv[0].item())
    assert lev.check_status() == 0
    fused = V.cpu().numpy()
    assert np.array_equal(interior(wl.layout.view(fused, 0)), interior(wl.layout.view(arena, 0)))
    del U, V, fused
    lev.close()
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    p = O.params(gamma=wl.gamma)
    s, _ = O.max_wavespeed(st[0], wl.dx, p)
    assert dts[0] == p.cfl / s
    got = lay.view(arena, 0)
    s1, _ = O.max_wavespeed(np.ascontiguousarray(got), wl.dx, p)
    assert nxt == p.cfl / s1
    rng = np.random.default_rng(1)
    n = lay.n(0)
    wins = _sample_windows(n, rng, 12)
    # full x-pencils (across the Sod jump at x = 1/2 and the periodic seam
    # at x = 0) and a whole 256 x 256 x 2 slab
    for _ in range(6):
        y, z = (int(v) for v in rng.integers(0, n[1], 2))
        wins.append(((0, y, z), (n[0] - 1, y, z)))
    z0 = int(rng.integers(0, n[2] - 1))
    wins.append(((0, 0, z0), (n[0] - 1, n[1] - 1, z0 + 1)))
    pairs = []
    for lo, hi in wins:
        ref, _, _ = O.step(st[0], dts[0], wl.dx, p, window=(lo, hi))
        sl = (slice(None),) + tuple(slice(lo[d] + 4, hi[d] + 5) for d in (2, 1, 0))
        pairs.append((got[sl], ref[sl]))
    parity_report(f"256^3 one step, {len(wins)} windows ({sum(g.shape[1] * g.shape[2] * g.shape[3] for g, _ in pairs)}"
                  " zones)", pairs, TOL)
    for c in range(5):
        s0 = math.fsum(interior(lay.view(wl.arena, 0))[c].ravel())
        s1 = math.fsum(interior(got)[c].ravel())
        sc = math.fsum(np.abs(interior(lay.view(wl.arena, 0))[c]).ravel())
        assert abs(s1 - s0) <= 1e-13 * sc


def test_cfg2_recipe_at_64_cubed_twenty_steps_whole_grid():
    """The 256^3 workload's recipe (seeded modes, Sod jump, constant velocity,
    gamma 5/3, periodic) on 64^3 for its 20 steps at CFL 0.5, each step's dt
    from the CFL rule on each side: the whole grid against the oracle."""
    wl = I.cfg2(64)
    _, arena, dts, flags, _ = gpu_run(wl, 20)
    ost, odts, ofl, _ = oracle_run(wl, 20)
    assert flags == ofl == 0
    assert dts_close(dts, odts), (dts, odts)
    compare_level(wl, arena, ost, tag="cfg2 recipe on 64^3, 20 steps")


def test_tiling_does_not_change_results_and_autotuner_caches(tmp_path):
    """Every tile size / strip order gives the same bits; the autotuner
    picks one of them (and one of the three final-stage forms, which give
    the same bits, whichever times fastest) and a second call takes it from
    its cache file."""
    wl = _uneven_level(seed=13)
    ref = gpu_run(wl, 2)[1]
    for tiling in [(128, 8), (512, 0), (64, 16), (256, 64)]:
        got = gpu_run(wl, 2, tiling=tiling)[1]
        assert np.array_equal(np.nan_to_num(got), np.nan_to_num(ref)), tiling
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma)
    U = torch.from_numpy(wl.arena).cuda()
    lev.fill_boundary(U)
    cache = tmp_path / "tune.jsonl"
    t, s, hit = lev.autotune(U, wl.dx, p, reps=1, cache_path=cache)
    assert not hit and t in (128, 256, 512) and s in (0, 8, 16, 32, 64)
    form, shape = lev.get_step_form(), lev.get_stream_tiling()
    assert form in (0, 1, 2)
    lev2 = P.Level(wl.layout)
    t2, s2, hit2 = lev2.autotune(U, wl.dx, p, reps=1, cache_path=cache)
    assert hit2 and (t2, s2) == (t, s) and lev2.get_tiling() == (t, s)
    assert lev2.get_step_form() == form and lev2.get_stream_tiling() == shape


def _smooth_on(lay, seed, gamma=1.4):
    rng = np.random.default_rng(seed)
    L = tuple((np.array(lay.domain_hi) + 1) / 16.0)
    S = [I.ModeSum(rng, 4, 2, L) for _ in range(5)]

    def prim(x, y, z):
        return (1.0 + 0.3 * S[0](x, y, z), 0.5 * S[1](x, y, z), 0.5 * S[2](x, y, z), 0.5 * S[3](x, y, z),
                1.0 + 0.3 * S[4](x, y, z))
    h = (1.0 / 16,) * 3
    return I.Workload("tiny", lay, I._fill_state(lay, h, gamma, prim), h, gamma, 1)


@pytest.mark.parametrize("bc", [(0, 0, 0, 0, 0, 0), (1, 1, 0, 0, 2, 2)])
def test_boxes_thinner_than_the_ghost_width_match_oracle(bc):
    """Boxes of 1, 2 and 3 zones along an axis: a ghost shell then spans
    several boxes (and periodic images) per face, edge and corner."""
    lay = I.tensor_tiling((1, 3, 4), (2, 2), (1, 5), bc=bc)
    wl = _smooth_on(lay, 41)
    _, arena, dts, flags, _ = gpu_run(wl, 2)
    ost, odts, ofl, _ = oracle_run(wl, 2)
    assert dts_close(dts, odts) and flags == ofl == 0
    compare_level(wl, arena, ost, tag=f"thin boxes, bc {bc}, 2 steps")


def test_state_at_rest_preserved_bitwise():
    """u = 0 everywhere: every Riemann solve lands on u* = 0 exactly (the
    two-sided average) and the state must not change at all."""
    wl = I.uniform(10, rho=0.8, vel=(0.0, 0.0, 0.0), p=1.9)
    _, arena, _, flags, _ = gpu_run(wl, 2)
    assert flags == 0
    assert np.array_equal(interior(wl.layout.view(arena, 0)), interior(wl.layout.view(wl.arena, 0)))


@pytest.mark.parametrize("axis", [0, 2])
def test_strong_shock_tube_matches_oracle(axis):
    """Pressure ratio 1e5 and density ratio 10 (a strong blast): flattening,
    the limiter and the two-shock iteration far from the acoustic guess."""
    wl = I.shock_tube(48, axis=axis, left=(10.0, 0.0, 1000.0), right=(1.0, 0.0, 0.01))
    _, arena, dts, flags, _ = gpu_run(wl, 6)
    ost, odts, ofl, _ = oracle_run(wl, 6)
    assert dts_close(dts, odts) and flags == ofl
    compare_level(wl, arena, ost, tag=f"1e5 pressure-ratio shock tube along axis {axis}, 6 steps")


FINAL_FORMS = [(0, None), (1, None), (2, (16, 8, 32)), (2, (16, 4, 5)), (2, (8, 8, 3)), (2, (32, 8, 64)),
               (2, (4, 8, 7))]


@pytest.mark.parametrize("precision", [0, 1])
def test_final_stage_forms_agree_bitwise(precision):
    """The staged pair (final fluxes in the workspace, then the update), the
    brick kernel and the streamed kernel with several tile shapes (tiles
    larger and smaller than the boxes, runs that split the boxes' z extent
    unevenly) give the same state, the same flux output and the same next
    dt bit for bit: uneven boxes, walls, gravity, both launch forms."""
    wl = _uneven_level(seed=9, bc=(0, 0, 1, 1, 2, 2), sizes=(6, 8, 12, 20))
    wl.grav = (0.0, 0.0, -1.0)
    wl.precision = precision
    outs = []
    for form, shape in FINAL_FORMS:
        for mode in (P.BATCHED, P.PER_BOX):
            print(f"final-stage form {form}, tile {shape}, mode {mode}, precision {precision}", flush=True)
            lev = P.Level(wl.layout)
            if shape:
                lev.set_stream_tiling(*shape)
            lev.set_step_form(form)
            assert lev.get_step_form() == form
            U = torch.from_numpy(wl.arena).cuda()
            V = lev.new_state()
            p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
            dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
            lev.compute_dt(U, wl.dx, p, out=dtv)
            F, dts = None, []
            for _ in range(2):
                lev.fill_boundary(U, mode)
                F = lev.new_fluxes()
                lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, fluxes=F, mode=mode, dt_next=dtv)
                dts.append(dtv.cpu().numpy().copy())
                U, V = V, U
            assert lev.check_status() == 0
            outs.append((U.cpu().numpy(), [f.cpu().numpy() for f in F], dts))
            lev.close()
    ref_u, ref_f, ref_dt = outs[0]
    lay = wl.layout
    for k, (u, f, dts) in enumerate(outs[1:]):
        for b in range(lay.nbox):
            assert np.array_equal(interior(lay.view(u, b)), interior(lay.view(ref_u, b))), (k, b)
        for d in range(3):
            assert np.array_equal(f[d], ref_f[d]), (k, d)
        for a, r in zip(dts, ref_dt):
            assert np.array_equal(a, r), k


FRONT_FORMS = [(16, 8, 32), (4, 4, 3), (11, 11, 5), (64, 2, 64), (7, 3, 7), (1, 1, 1), (1, 127, 2)]


@pytest.mark.parametrize("precision", [0, 1])
def test_front_forms_agree_bitwise(precision):
    """The fused front ends (trace and stage-1 solves in one kernel: x-y
    tiles walked along z, with tiles larger and smaller than the boxes,
    single-zone tiles and runs that split the boxes' z extent unevenly; the
    x axis alone; every axis with wavefront patches), in both launch forms
    and with the fused final stages too, give the staged front end's state,
    flux output and next dt bit for bit: uneven boxes, walls, gravity."""
    wl = _uneven_level(seed=9, bc=(0, 0, 1, 1, 2, 2), sizes=(6, 8, 12, 20))
    wl.grav = (0.0, 0.0, -1.0)
    wl.precision = precision
    cases = [(None, 0, P.BATCHED)] + [(sh, 0, P.BATCHED) for sh in FRONT_FORMS] + \
        [(FRONT_FORMS[1], 0, P.PER_BOX), (FRONT_FORMS[0], 2, P.BATCHED), (FRONT_FORMS[3], 1, P.PER_BOX)] + \
        [("x", 0, P.BATCHED), ("x", 0, P.PER_BOX), ("x", 1, P.BATCHED), ("x", 2, P.PER_BOX)] + \
        [("xyz", 0, P.BATCHED), ("xyz", 0, P.PER_BOX), ("xyz", 1, P.BATCHED), ("xyz", 2, P.PER_BOX)]
    outs = []
    for shape, final, mode in cases:
        print(f"front tile {shape}, final-stage form {final}, mode {mode}, precision {precision}", flush=True)
        lev = P.Level(wl.layout)
        if shape is None:
            lev.set_front_form(0)
        elif shape in ("x", "xyz"):
            lev.set_front_form(2 if shape == "x" else 3)
            assert lev.get_front_form() == (2 if shape == "x" else 3)
        else:
            lev.set_front_tiling(*shape)
            lev.set_front_form(1)
            assert lev.get_front_form() == 1 and lev.get_front_tiling() == shape
        lev.set_step_form(final)
        U = torch.from_numpy(wl.arena).cuda()
        V = lev.new_state()
        p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
        dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
        lev.compute_dt(U, wl.dx, p, out=dtv)
        F, dts = None, []
        for _ in range(2):
            lev.fill_boundary(U, mode)
            F = lev.new_fluxes()
            lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, fluxes=F, mode=mode, dt_next=dtv)
            dts.append(dtv.cpu().numpy().copy())
            U, V = V, U
        assert lev.check_status() == 0
        outs.append((U.cpu().numpy(), [f.cpu().numpy() for f in F], dts))
        lev.close()
    ref_u, ref_f, ref_dt = outs[0]
    lay = wl.layout
    for k, (u, f, dts) in enumerate(outs[1:]):
        for b in range(lay.nbox):
            assert np.array_equal(interior(lay.view(u, b)), interior(lay.view(ref_u, b))), (k, b)
        for d in range(3):
            assert np.array_equal(f[d], ref_f[d]), (k, d)
        for a, r in zip(dts, ref_dt):
            assert np.array_equal(a, r), k


def test_front_tiling_rejects_oversized_tiles():
    wl = _uneven_level(seed=9)
    lev = P.Level(wl.layout)
    with pytest.raises(P.PPMError, match="front_tiling"):
        lev.set_front_tiling(16, 16, 8)  # 256 zones per tile
    with pytest.raises(P.PPMError, match="front_form"):
        lev.set_front_form(4)
    lev.close()


def test_power_of_two_change_of_units_on_gpu():
    """Density x 2^20 and pressure x 2^72 (velocity x 2^26), gravity on: the
    GPU run in the new units is the scaled GPU run in the old ones bit for
    bit, dt included (every operation of the FP64 step scales exactly), and
    matches the oracle at these magnitudes."""
    wl = I.cfg2(16)
    wl.grav = (0.3, -0.2, 0.1)
    ws, sc, V = rescaled(wl)
    _, a, dts, fl, _ = gpu_run(wl, 3)
    _, b, dtss, fls, _ = gpu_run(ws, 3)
    assert fl == fls == 0
    assert dtss == [d / V for d in dts]
    lay = wl.layout
    for bx in range(lay.nbox):
        assert np.array_equal(lay.view(b, bx)[:, 4:-4, 4:-4, 4:-4], lay.view(a, bx)[:, 4:-4, 4:-4, 4:-4] * sc)
    ost, odts, ofl, _ = oracle_run(ws, 3)
    assert ofl == 0
    assert dts_close(dtss, odts)
    compare_level(ws, b, ost, tag="rescaled units, 3 steps")


@pytest.mark.parametrize("form", [0, 1])
def test_kernel_roots_are_the_ieee_root(form):
    """The Riemann solver takes its FP64 square roots with the core of the
    compiler's correctly rounded root, without the rescaling of arguments
    below 2^-767 (the wave-speed root, form 0, also without the fix-up of 0
    and inf, which its argument 1 + beta (p/p_s - 1) never reaches).  Both
    must return the IEEE root, bit for bit, for every finite argument from
    2^-767 up: 2^20 random arguments with exponents uniform over that range,
    the wave-speed factor's own range near 1 - beta, the end points, and
    for the sound-speed root (form 1) also 0, -0, +inf, negative and NaN
    arguments."""
    rng = np.random.default_rng(12)
    n = 1 << 20
    mant = rng.integers(0, 1 << 52, size=n, dtype=np.uint64)
    expo = rng.integers(-767, 1024, size=n).astype(np.int64)
    bits = ((expo + 1023).astype(np.uint64) << np.uint64(52)) | mant
    x = bits.view(np.float64)
    beta = (1.4 + 1.0) / 2.8
    near = 1.0 - beta + rng.uniform(0.0, 4.0, size=4096) ** 3
    ends = np.array([2.0 ** -767, np.nextafter(2.0 ** -767, 1.0), 1.0 - beta, 1.0, 2.0, 4.0,
                     np.finfo(np.float64).max, np.nextafter(np.finfo(np.float64).max, 0.0)])
    special = np.array([0.0, -0.0, np.inf, -1.0, -np.inf, np.nan]) if form == 1 else np.array([])
    x = np.concatenate([x, near, ends, special])
    got = P.sqrt_values(torch.from_numpy(x).cuda(), form).cpu().numpy()
    with np.errstate(invalid="ignore"):
        ref = np.sqrt(x)
    same = (got.view(np.uint64) == ref.view(np.uint64)) | (np.isnan(got) & np.isnan(ref))
    bad = np.flatnonzero(~same)
    assert bad.size == 0, (bad.size, x[bad[:5]], got[bad[:5]], ref[bad[:5]])


def test_fp32_wave_root_is_the_ieee_root():
    """The FP32 mode takes the root of the wave-speed factor with hipcc's
    correctly rounded FP32 root minus its rescaling of arguments below
    2^-96 and its fix-up of 0 and inf (the factor is at least 1 - beta).  It
    must return the IEEE FP32 root, bit for bit, for every finite FP32
    argument from 2^-96 up: 2^20 random ones with exponents uniform over
    that range, the factor's own range and the end points."""
    rng = np.random.default_rng(14)
    n = 1 << 20
    mant = rng.integers(0, 1 << 23, size=n, dtype=np.uint32)
    expo = rng.integers(-96, 128, size=n).astype(np.int64)
    bits = ((expo + 127).astype(np.uint32) << np.uint32(23)) | mant
    x = bits.view(np.float32)
    beta = np.float32((1.4 + 1.0) / 2.8)
    near = (np.float32(1.0) - beta + rng.uniform(0.0, 4.0, size=4096).astype(np.float32) ** 3).astype(np.float32)
    ends = np.array([2.0 ** -96, np.nextafter(np.float32(2.0 ** -96), np.float32(1.0)), 1.0 - beta, 1.0, 2.0,
                     np.finfo(np.float32).max], dtype=np.float32)
    x = np.concatenate([x, near, ends]).astype(np.float32)
    got = P.sqrt_values(torch.from_numpy(x.astype(np.float64)).cuda(), 2).cpu().numpy().astype(np.float32)
    ref = np.sqrt(x)
    bad = np.flatnonzero(got.view(np.uint32) != ref.view(np.uint32))
    assert bad.size == 0, (bad.size, x[bad[:5]], got[bad[:5]], ref[bad[:5]])


def test_kernel_quotient_is_the_ieee_quotient():
    """The kernels divide with the compiler's correctly rounded FP64 division
    without its operand scaling.  It must return the IEEE quotient, bit for
    bit, whenever both exponents lie in [-900, 900] and differ by at most
    700, and for zero, infinite and NaN operands: 2^20 random pairs of
    either sign over that range (half of them with nearby exponents, as the
    method's quotients have), signed zeros and infinities over either sign,
    divisions by zero, and the range's corners."""
    rng = np.random.default_rng(13)
    n = 1 << 20

    def make(expo):
        mant = rng.integers(0, 1 << 52, size=expo.size, dtype=np.uint64)
        bits = ((expo + 1023).astype(np.uint64) << np.uint64(52)) | mant
        x = bits.view(np.float64)
        return np.where(rng.integers(0, 2, size=expo.size) == 1, -x, x)
    eb = rng.integers(-900, 901, size=n).astype(np.int64)
    near = eb + rng.integers(-30, 31, size=n)
    far = eb + rng.integers(-700, 701, size=n)
    ea = np.clip(np.where(np.arange(n) % 2 == 0, near, far), -900, 900)
    a, b = make(ea), make(eb)
    inf = np.inf
    zeros = np.array([0.0, -0.0] * 4 + [1.5, -1.5, 0.0, -0.0, inf, -inf, inf, 2.0, np.nan, 1.0])
    zb = np.array([1.0, 1.0, -1.0, -1.0, 2.0 ** 900, 2.0 ** -900, -3.5, 7.25]
                  + [0.0, 0.0, -0.0, 0.0, 3.0, 3.0, -inf, inf, 1.0, np.nan])
    ca = np.array([2.0 ** 900, 2.0 ** -900, 2.0 ** 200, 2.0 ** -200, 1.0, 1.0 - 2.0 ** -52])
    cb = np.array([2.0 ** 200, 2.0 ** -200, 2.0 ** 900, 2.0 ** -900, 3.0, 1.0 + 2.0 ** -52])
    a = np.concatenate([a, zeros, ca])
    b = np.concatenate([b, zb, cb])
    got = P.quotient_values(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    with np.errstate(divide="ignore", invalid="ignore"):
        ref = a / b
    same = (got.view(np.uint64) == ref.view(np.uint64)) | (np.isnan(got) & np.isnan(ref))
    bad = np.flatnonzero(~same)
    assert bad.size == 0, (bad.size, a[bad[:5]], b[bad[:5]], got[bad[:5]], ref[bad[:5]])


def test_zone_index_division_on_the_device():
    """The kernels' zone-index division (high multiply and shift) on the
    device equals numpy's floor division for dividends across [0, 2^31),
    for the row lengths of boxes and bricks and for arbitrary divisors."""
    rng = np.random.default_rng(32)
    top = 2 ** 31 - 1
    divisors = [3, 5, 10, 18, 33, 66, 72, 130, 136, 258, 264, 1026, 1032] + [int(v) for v in rng.integers(2, 2 ** 31,
                                                                                                     size=12)]
    for d in divisors:
        base = rng.integers(0, 2 ** 31, size=200000, dtype=np.int64)
        edges = np.array([k * d + e for k in (1, 2, 5, 999, top // d) for e in (-1, 0, 1)] + [0, 1, top, top - 1],
                         dtype=np.int64)
        n = np.concatenate([base, edges[(edges >= 0) & (edges <= top)]]).astype(np.int32)
        got = P.div31_values(torch.from_numpy(n).cuda(), d).cpu().numpy()
        ref = (n.astype(np.int64) // d).astype(np.int32)
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, (d, bad.size, n[bad[:5]], got[bad[:5]], ref[bad[:5]])


@pytest.mark.parametrize("mode,precision,fused", [(P.BATCHED, 0, 0), (P.PER_BOX, 0, 0), (P.BATCHED, 1, 0),
                                                  (P.BATCHED, 0, 1), (P.BATCHED, 0, 2), (P.PER_BOX, 1, 2)])
def test_fused_next_dt_is_compute_dt_of_the_new_state(mode, precision, fused):
    """ppm_hydro_step_dt leaves the CFL dt of the state it writes: bit for
    bit what a separate ppm_compute_dt pass over Unew gives (dt and the
    maximum signal speed), on uneven boxes with walls and gravity, in the
    per-box launch form, in FP32-reconstruction mode, in the brick form
    (which runs that separate pass itself) and in the streamed form."""
    wl = _uneven_level(seed=17, bc=(0, 0, 1, 1, 2, 2), sizes=(6, 8, 12, 20))
    wl.grav = (0.0, 0.0, -1.0)
    wl.precision = precision
    lev = P.Level(wl.layout)
    lev.set_step_form(fused)
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    nxt = torch.zeros(2, dtype=torch.float64, device="cuda")
    ref = torch.zeros(2, dtype=torch.float64, device="cuda")
    lev.fill_boundary(U, mode)
    lev.compute_dt(U, wl.dx, p, out=dtv)
    for _ in range(3):
        lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, mode=mode, dt_next=nxt)
        lev.compute_dt(V, wl.dx, p, out=ref)
        assert torch.equal(nxt.view(torch.int64), ref.view(torch.int64)), (nxt.tolist(), ref.tolist())
        dtv.copy_(nxt)
        U, V = V, U
        lev.fill_boundary(U, mode)
    assert lev.check_status() == 0
    lev.close()


def test_run_with_fused_dt_equals_the_plain_run():
    """Steps that read their dt from the previous step's update (one dt
    buffer, passed as both dt_dev and dt_next) reproduce the plain loop of
    fill, compute_dt and step bit for bit: every dt and the final state."""
    wl = _uneven_level(seed=18, bc=(0, 0, 0, 0, 1, 1), sizes=(8, 12, 16))
    _, plain, dts, flags, _ = gpu_run(wl, 4)
    assert flags == 0
    lev = P.Level(wl.layout)
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    p = P.params(gamma=wl.gamma, grav=wl.grav)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    lev.fill_boundary(U)
    lev.compute_dt(U, wl.dx, p, out=dtv)
    got = []
    for _ in range(4):
        got.append(float(dtv[0].item()))
        lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, dt_next=dtv)
        U, V = V, U
        lev.fill_boundary(U)
    assert got == dts
    fused = U.cpu().numpy()
    for b in range(wl.layout.nbox):
        assert np.array_equal(interior(wl.layout.view(fused, b)), interior(wl.layout.view(plain, b)))
    assert lev.check_status() == 0
    lev.close()


def test_graph_launch_refused_after_the_context_changes():
    """A captured graph replays the workspace, tile lists and step form it
    was captured with: after set_tiling, a new workspace, a changed step
    form or the context's destruction, its launch is refused (PPM_EINVAL)
    and replays nothing; a graph captured afterwards runs."""
    wl = I.cfg2(16)
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma)
    A = torch.from_numpy(wl.arena).cuda()
    B = lev.new_state()
    g = lev.graph(A, B, wl.dx, p, 2)
    g.launch()
    torch.cuda.synchronize()
    before = A.clone()
    lev.set_tiling(128, 8)
    with pytest.raises(P.PPMError, match="changed since the graph was captured"):
        g.launch()
    torch.cuda.synchronize()
    assert torch.equal(A, before)                 # nothing was replayed
    g.close()
    g = lev.graph(A, B, wl.dx, p, 2)              # captured again: runs
    g.launch()
    torch.cuda.synchronize()
    lev.set_step_form(True)
    with pytest.raises(P.PPMError):
        g.launch()
    lev.set_step_form(False)
    g.close()
    g = lev.graph(A, B, wl.dx, p, 2)
    lev._work = None
    lev.ensure_workspace(0)                       # a new workspace buffer
    with pytest.raises(P.PPMError):
        g.launch()
    g.close()
    g = lev.graph(A, B, wl.dx, p, 2)
    lev.close()                                   # the context is gone
    rc = P.lib().ppm_graph_launch(g.g, None)
    assert rc == P.PPM_EINVAL
    g.close()


def test_state_outside_the_exact_range_raises_the_range_flag():
    """The shortened FP64 divisions and roots are the IEEE results for
    states whose densities, pressures and sound speeds lie in
    [2^-120, 2^120] (velocities up to 2^120): a zone outside raises
    FLAG_RANGE (the step still runs); floors outside that range are
    refused."""
    wl = I.cfg1(8)
    lay = wl.layout
    U0 = wl.arena.copy()
    v = lay.view(U0, 0)
    v[:, 6, 6, 6] *= 2.0 ** -130          # density, momenta, energy: rho ~ 1e-39, p ~ 1e-39
    wl2 = I.Workload("tiny", lay, U0, wl.dx, wl.gamma, 1)
    _, out, _, flags, _ = gpu_run(wl2, 1, dt=1e-3)
    assert flags & P.FLAG_RANGE and not flags & P.FLAG_NONPHYS
    _, _, _, flags, _ = gpu_run(wl, 1, dt=1e-3)
    assert flags == 0
    lev = P.Level(lay)
    U = torch.from_numpy(wl.arena).cuda()
    with pytest.raises(P.PPMError, match="floors"):
        lev.hydro_step(U, lev.new_state(), wl.dx, P.params(gamma=1.4, small_pres=1e-40), dt=1e-3)

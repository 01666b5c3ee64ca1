"""Full-size GPU checks of the batched multi-box workloads against the
oracle on sampled windows and pencils (the oracle recomputes each window
from the same input), conservation over the whole level, the
FP32-reconstruction error per field against FP64, and the Rayleigh-Taylor
set-up (reflecting walls, gravity) on a reduced instance against the oracle
in both precisions.  Bars: 1e-12 per field (FP64), 1e-5 per field against
the oracle's own FP32 mode."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1008_2801_amd import inputs as I  # noqa: E402
from paper_1008_2801_amd import ppm as P  # noqa: E402
from tests.helpers import interior, parity_report  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12
# against the oracle's FP32 mode; see test_gpu_parity.FP32_TOL
FP32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _one_step(wl, precision=0, mode=P.BATCHED):
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    U = torch.from_numpy(wl.arena).cuda()
    lev.fill_boundary(U, mode)
    dtv = lev.compute_dt(U, wl.dx, p)
    V = lev.new_state()
    lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, mode=mode)
    out = V.cpu().numpy()
    flags = lev.check_status()
    dt = float(dtv[0].item())
    lev.close()
    return out, dt, flags


@pytest.fixture(scope="module")
def cfg3_state():
    return I.cfg3()


def _window_pairs(wl, st, out, dt, p, wins):
    """(gpu, oracle) pairs of the windows [(box, lo, hi)] of a one-step output."""
    lay = wl.layout
    pairs = []
    for b, lo, hi in wins:
        ref, _, _ = O.step(st[b], dt, wl.dx, p, window=(lo, hi),
                           walls=O.box_walls(lay.boxes(), lay.domain(), lay.bc, b))
        sl = (slice(None),) + tuple(slice(lo[d] + 4, hi[d] + 5) for d in (2, 1, 0))
        pairs.append((lay.view(out, b)[sl], ref[sl]))
    return pairs


def _cfg3_windows(lay, rng):
    """2^3 windows in 24 boxes, plus a full x-pencil and a full z-pencil in
    6 more boxes (each crossing the box's low and high faces, where the
    ghost zones come from neighbouring boxes and periodic images)."""
    wins = []
    for b in rng.choice(lay.nbox, 24, replace=False):
        n = lay.n(b)
        for _ in range(2):
            lo = tuple(int(rng.integers(0, n[d] - 1)) for d in range(3))
            wins.append((int(b), lo, tuple(v + 1 for v in lo)))
    for b in rng.choice(lay.nbox, 6, replace=False):
        n = lay.n(b)
        y, z = int(rng.integers(0, n[1])), int(rng.integers(0, n[2]))
        wins.append((int(b), (0, y, z), (n[0] - 1, y, z)))
        x, y = int(rng.integers(0, n[0])), int(rng.integers(0, n[1]))
        wins.append((int(b), (x, y, 0), (x, y, n[2] - 1)))
    return wins


def test_cfg3_full_level_sampled_windows_and_conservation(cfg3_state):
    wl = cfg3_state
    lay = wl.layout
    out, dt, flags = _one_step(wl)
    assert flags == 0
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    p = O.params(gamma=wl.gamma)
    s = max(O.max_wavespeed(u, wl.dx, p)[0] for u in st)
    assert dt == p.cfl / s
    wins = _cfg3_windows(lay, np.random.default_rng(2))
    parity_report(f"512-box level, one step, {len(wins)} windows and pencils",
                  _window_pairs(wl, st, out, dt, p, wins), TOL)
    for c in range(5):
        s0 = math.fsum(np.concatenate([interior(lay.view(wl.arena, b))[c].ravel() for b in range(lay.nbox)]))
        s1 = math.fsum(np.concatenate([interior(lay.view(out, b))[c].ravel() for b in range(lay.nbox)]))
        sc = math.fsum(np.abs(np.concatenate([interior(lay.view(wl.arena, b))[c].ravel()
                                              for b in range(lay.nbox)])))
        assert abs(s1 - s0) <= 1e-13 * sc


def test_cfg3_fp32_mode_sampled_windows_against_the_oracle_fp32_mode(cfg3_state):
    """The same level in FP32-reconstruction mode against the oracle's FP32
    mode (reconstruction, tracing and Riemann solves in float, the update
    in double) on the same windows and pencils."""
    wl = cfg3_state
    lay = wl.layout
    out, dt, flags = _one_step(wl, precision=1)
    assert flags == 0
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    p = O.params(gamma=wl.gamma, precision=1)
    wins = _cfg3_windows(lay, np.random.default_rng(3))
    parity_report(f"512-box level, FP32 mode, one step, {len(wins)} windows and pencils",
                  _window_pairs(wl, st, out, dt, p, wins), FP32_TOL)


def test_cfg3_fp32_reconstruction_error_per_field(cfg3_state):
    """One step in FP32-reconstruction mode against the FP64 step: per field,
    the max error normalised by the field's max and the L1 error normalised
    by its L1 norm; conservation still holds to FP64 round-off."""
    wl = cfg3_state
    lay = wl.layout
    o64, dt64, _ = _one_step(wl, 0)
    o32, dt32, flags = _one_step(wl, 1)
    assert flags == 0 and dt32 == dt64
    a = np.concatenate([interior(lay.view(o32, b)).reshape(5, -1) for b in range(lay.nbox)], axis=1)
    r = np.concatenate([interior(lay.view(o64, b)).reshape(5, -1) for b in range(lay.nbox)], axis=1)
    u0 = np.concatenate([interior(lay.view(wl.arena, b)).reshape(5, -1) for b in range(lay.nbox)], axis=1)
    linf = np.abs(a - r).max(axis=1) / np.abs(r).max(axis=1)
    l1 = np.abs(a - r).sum(axis=1) / np.abs(r).sum(axis=1)
    print("fp32-reconstruction vs fp64, one step, per field (rho, mx, my, mz, E): Linf",
          np.array2string(linf, precision=3), "L1", np.array2string(l1, precision=3))
    assert linf.max() < 2e-5 and l1.max() < 2e-6
    for c in range(5):
        assert abs(math.fsum(a[c]) - math.fsum(u0[c])) <= 1e-13 * math.fsum(np.abs(u0[c]))


@pytest.mark.parametrize("precision", [1, 0])
def test_rayleigh_taylor_reduced_instance_matches_oracle(precision):
    """2x2x2 boxes of 16^3 of the Rayleigh-Taylor set-up (walls in z,
    g = -1 in z), 3 steps, against the oracle in the same precision mode."""
    wl = I.cfg5(2, 16)
    lay = wl.layout
    lev = P.Level(lay)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    for _ in range(3):
        lev.fill_boundary(U)
        lev.compute_dt(U, wl.dx, p, out=dtv)
        lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv)
        U, V = V, U
    got = U.cpu().numpy()
    assert lev.check_status() == 0
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    op = O.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    ost, _, ofl, _ = O.advance(lay.boxes(), lay.domain(), lay.bc, st, 3, wl.dx, op)
    assert ofl == 0
    parity_report(f"Rayleigh-Taylor 2x2x2 boxes of 16^3, precision {precision}, 3 steps",
                  [(interior(lay.view(got, b)), interior(ost[b])) for b in range(lay.nbox)],
                  TOL if precision == 0 else FP32_TOL)


@pytest.fixture(scope="module")
def cfg5_state():
    wl = I.cfg5()
    lay = wl.layout
    st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
    O.fill(lay.boxes(), lay.domain(), lay.bc, st)
    return wl, st


@pytest.mark.parametrize("precision", [1, 0])
def test_rayleigh_taylor_full_level_sampled_windows(cfg5_state, precision):
    """The 512^3 Rayleigh-Taylor level as timed (512 boxes of 64^3, walls in
    z, g = (0, 0, -1)), one step in FP32-reconstruction and FP64 mode: the dt,
    sampled 2^3 windows against the oracle in the same mode (boxes at both
    walls and inside; windows at box corners and inside), conservation of
    mass and of the x and y momenta (gravity and the walls act along z)."""
    wl, st = cfg5_state
    lay = wl.layout
    out, dt, flags = _one_step(wl, precision)
    assert flags == 0
    p = O.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    s = max(O.max_wavespeed(u, wl.dx, p)[0] for u in st)
    assert dt == p.cfl / s
    rng = np.random.default_rng(50 + precision)
    zlo = [b for b in range(lay.nbox) if lay.lo[b, 2] == 0]
    zhi = [b for b in range(lay.nbox) if lay.hi[b, 2] == lay.domain_hi[2]]
    mid = [b for b in range(lay.nbox) if b not in zlo and b not in zhi]
    boxes = list(rng.choice(zlo, 3, replace=False)) + list(rng.choice(zhi, 3, replace=False)) + \
        list(rng.choice(mid, 4, replace=False))
    wins = []
    for b in boxes:
        n = lay.n(b)
        corners = [(0, 0, 0), tuple(n[d] - 2 for d in range(3))]
        inner = [tuple(int(rng.integers(1, n[d] - 2)) for d in range(3))]
        for lo in corners + inner:
            wins.append((int(b), lo, tuple(v + 1 for v in lo)))
    # z-pencils along the box edges of wall boxes: from the wall through the
    # box's other z face
    for b in list(rng.choice(zlo, 2, replace=False)) + list(rng.choice(zhi, 2, replace=False)):
        n = lay.n(b)
        for x, y in ((0, 0), (n[0] - 1, n[1] - 1)):
            wins.append((int(b), (x, y, 0), (x, y, n[2] - 1)))
    parity_report(f"512^3 Rayleigh-Taylor, precision {precision}, one step, {len(wins)} windows and pencils",
                  _window_pairs(wl, st, out, dt, p, wins), TOL if precision == 0 else FP32_TOL)
    # pairwise sums per box, exact sum over boxes (rounding ~1e-15 of the
    # scale: the total mass times the sound speed, about 1)
    mass = math.fsum(float(np.sum(interior(lay.view(wl.arena, b))[0])) for b in range(lay.nbox))
    for c in range(3):
        s0 = math.fsum(float(np.sum(interior(lay.view(wl.arena, b))[c])) for b in range(lay.nbox))
        s1 = math.fsum(float(np.sum(interior(lay.view(out, b))[c])) for b in range(lay.nbox))
        assert abs(s1 - s0) <= 1e-13 * mass, (c, s1 - s0, mass)

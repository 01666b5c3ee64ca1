"""GPU parity of the two-level advance (ppm_amr_* through the C ABI) against
the oracle's two-level advance on the same seeded inputs.  FP64 bar: per
field max |gpu - oracle| / max |oracle| <= 1e-12 (the kernels evaluate the
same definitions in the same order, so the values are expected to agree bit
for bit)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import amr as A  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1008_2801_amd import inputs as I  # noqa: E402
from paper_1008_2801_amd import ppm as P  # noqa: E402
from tests.helpers import dts_close, interior, parity_report  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def hier(t):
    c, f = t.coarse.layout, t.fine.layout
    return A.Hierarchy(c.boxes(), c.domain(), c.bc, f.boxes(), t.region)


def ostates(t):
    c, f = t.coarse.layout, t.fine.layout
    return ([c.view(t.coarse.arena, b).copy() for b in range(c.nbox)],
            [f.view(t.fine.arena, b).copy() for b in range(f.nbox)])


def gpu_run(t, nsteps, dt=0.0, **pk):
    H = P.TwoLevel(t.coarse.layout, t.fine.layout)
    Uc = torch.from_numpy(t.coarse.arena).cuda()
    Vc = H.coarse.new_state()
    Uf = torch.from_numpy(t.fine.arena).cuda()
    Tf = H.fine.new_state()
    p = P.params(gamma=t.coarse.gamma, grav=t.coarse.grav, **pk)
    dto = torch.zeros(2, dtype=torch.float64, device="cuda")
    dts = []
    for _ in range(nsteps):
        H.step(Uc, Vc, Uf, Tf, t.coarse.dx, p, dt=dt, dt_out=dto)
        dts.append(float(dto[0].item()))
        Uc, Vc = Vc, Uc
    flags = H.coarse.check_status() | H.fine.check_status()
    out = (Uc.cpu().numpy(), Uf.cpu().numpy(), dts, flags)
    H.close()
    return out


def compare(t, gc, gf, oc, of, tol=TOL, tag="two-level"):
    """Per-field parity over both levels' valid zones."""
    pairs = []
    for lay, arena, ref in ((t.coarse.layout, gc, oc), (t.fine.layout, gf, of)):
        for b in range(lay.nbox):
            pairs.append((interior(lay.view(arena, b)), interior(ref[b])))
    err, nbits = parity_report(tag, pairs, tol)
    return float(err.max()), nbits


def _ragged_prim(x, y, z):
    return (1.0 + 0.2 * np.sin(6.0 * x) * np.cos(4.0 * y), 0.3, -0.2 + 0.1 * np.cos(5.0 * z), 0.1,
            1.0 + 0.1 * np.sin(3.0 * (x + z)))


CASES = {
    "aligned": lambda: (I.amr_random(16, 8, 8), 3),
    "misaligned": lambda: (I.amr_random(16, 8, 6, seed=22), 2),
    "gravity": lambda: (I.amr_random(16, 16, 4, seed=23, grav=(0.3, -0.2, 0.1)), 2),
    "wave": lambda: (I.amr_wave(16, 8, 8), 2),
    "ragged": lambda: (I.two_level((20, 16, 24), 12, 10, _ragged_prim, 1.4, "ragged"), 2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_two_level_step_matches_oracle(name):
    t, nsteps = CASES[name]()
    print(f"amr parity case {name}: coarse boxes {t.coarse.layout.nbox}, fine boxes {t.fine.layout.nbox}, "
          f"{nsteps} coarse steps", flush=True)
    gc, gf, dts, flags = gpu_run(t, nsteps)
    oc, of = ostates(t)
    p = O.params(gamma=t.coarse.gamma, grav=t.coarse.grav)
    oc, of, odts, ofl = A.advance(hier(t), oc, of, nsteps, t.coarse.dx, p)
    assert flags == 0 and ofl == 0
    assert dts_close(dts, odts)
    compare(t, gc, gf, oc, of, tag=f"two-level {name}, {nsteps} coarse steps")


def test_fill_fine_matches_oracle_bitwise():
    """Intra-level copies and the interpolation at both time fractions,
    from two different coarse states."""
    t = I.amr_random(16, 8, 6, seed=24)
    t2 = I.amr_random(16, 8, 6, seed=25)
    h = hier(t)
    H = P.TwoLevel(t.coarse.layout, t.fine.layout)
    Uo = torch.from_numpy(t.coarse.arena).cuda()
    Un = torch.from_numpy(t2.coarse.arena).cuda()
    H.coarse.fill_boundary(Uo)
    H.coarse.fill_boundary(Un)
    oc, of = ostates(t)
    oc2, _ = ostates(t2)
    Go, Gn = A.coarse_global(h, oc), A.coarse_global(h, oc2)
    for half in (0, 1):
        Uf = torch.from_numpy(t.fine.arena).cuda()
        H.fill_fine(Uo, Un, half, Uf)
        got = Uf.cpu().numpy()
        ref = [u.copy() for u in of]
        A.fill_fine(h, Go, Gn, 0.5 * half, ref)
        for b in range(t.fine.layout.nbox):
            assert np.array_equal(t.fine.layout.view(got, b), ref[b]), (half, b)
    sz = H.sizes()
    assert sz["register_faces"] == 6 * 8 * 8 and sz["covered_zones"] == 8 ** 3 and sz["interp_zones"] > 0
    H.close()


def test_uniform_state_preserved_bitwise_on_gpu():
    def prim(x, y, z):
        return (1.3, 0.3, -0.2, 0.1, 0.7)
    t = I.two_level(16, 8, 6, prim, 1.4, "uniform")
    gc, gf, _, flags = gpu_run(t, 2)
    assert flags == 0
    for lay, arena, ref in ((t.coarse.layout, gc, t.coarse.arena), (t.fine.layout, gf, t.fine.arena)):
        for b in range(lay.nbox):
            assert np.array_equal(interior(lay.view(arena, b)), interior(lay.view(ref, b)))


def _composite(t, gc, gf):
    h = hier(t)
    cs = [t.coarse.layout.view(gc, b) for b in range(t.coarse.layout.nbox)]
    fs = [t.fine.layout.view(gf, b) for b in range(t.fine.layout.nbox)]
    return A.composite_sums(h, cs, fs, t.coarse.dx)


def test_composite_conservation_on_gpu_multibox():
    """64^3 coarse (8 boxes) with the inner 12.5% refined (8 fine boxes of
    32^3), 3 coarse steps: mass, momentum and energy of the composite
    solution conserved to round-off."""
    t = I.amr_cfg2(64, cbox=32, fbox=32)
    s0 = _composite(t, t.coarse.arena, t.fine.arena)
    gc, gf, dts, flags = gpu_run(t, 3)
    assert flags == 0
    s1 = _composite(t, gc, gf)
    h = hier(t)
    scale = A.composite_sums(h, [np.abs(t.coarse.layout.view(t.coarse.arena, b)) for b in range(t.coarse.layout.nbox)],
                             [np.abs(t.fine.layout.view(t.fine.arena, b)) for b in range(t.fine.layout.nbox)],
                             t.coarse.dx)
    for c in range(5):
        assert abs(s1[c] - s0[c]) <= 1e-14 * scale[c], (c, s1[c] - s0[c])


def test_full_size_hierarchy_conservation_and_interpolation():
    """The timed hierarchy: 256^3 coarse with the inner 12.5% refined
    (256^3 fine zones), one box per level.  One coarse step conserves the
    composite mass and momentum to round-off; the fine ghost fill of the
    first sub-step matches the oracle's interpolation bit for bit."""
    t = I.amr_cfg2(256)
    h = hier(t)
    H = P.TwoLevel(t.coarse.layout, t.fine.layout)
    Uc = torch.from_numpy(t.coarse.arena).cuda()
    H.coarse.fill_boundary(Uc)
    Uf = torch.from_numpy(t.fine.arena).cuda()
    H.fill_fine(Uc, Uc, 0, Uf)
    got = Uf.cpu().numpy()
    oc, of = ostates(t)
    O.fill(h.cboxes, h.cdomain, h.cbc, oc)
    G = A.coarse_global(h, oc)
    A.interpolate_fine_ghosts(h, G, G, 0.0, of)
    ref = of[0]
    g = t.fine.layout.view(got, 0)
    assert np.array_equal(g, ref)
    del ref, of, g, got
    s0 = _composite(t, t.coarse.arena, t.fine.arena)
    Vc = H.coarse.new_state()
    Tf = H.fine.new_state()
    Uf = torch.from_numpy(t.fine.arena).cuda()
    Uc = torch.from_numpy(t.coarse.arena).cuda()
    p = P.params(gamma=t.coarse.gamma)
    H.step(Uc, Vc, Uf, Tf, t.coarse.dx, p)
    flags = H.coarse.check_status() | H.fine.check_status()
    assert flags == 0
    s1 = _composite(t, Vc.cpu().numpy(), Uf.cpu().numpy())
    H.close()
    mass = abs(s0[0])
    for c in range(4):
        assert abs(s1[c] - s0[c]) <= 1e-13 * mass, (c, s1[c] - s0[c])


def test_hierarchy_requirements_are_rejected():
    t = I.amr_random(16, 8, 8)
    # fine boxes not aligned to the coarse zones
    lay = I.tensor_tiling([7, 9], [8, 8], [8, 8], bc=(I.BC_COARSE_FINE,) * 6, origin=(8, 8, 8))
    with pytest.raises(P.PPMError, match="coarse-zone boundaries"):
        P.TwoLevel(t.coarse.layout, lay)
    # fine faces that are not coarse-fine
    lay = I.tensor_tiling([8, 8], [8, 8], [8, 8], bc=(0,) * 6, origin=(8, 8, 8))
    with pytest.raises(P.PPMError, match="COARSE_FINE"):
        P.TwoLevel(t.coarse.layout, lay)
    # refined region too close to the domain face
    lay = I.tensor_tiling([8, 8], [8, 8], [8, 8], bc=(I.BC_COARSE_FINE,) * 6, origin=(2, 8, 8))
    with pytest.raises(P.PPMError, match="3 coarse zones"):
        P.TwoLevel(t.coarse.layout, lay)

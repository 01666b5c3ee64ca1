"""The allocation-free step (ppm_hydro_step_noalloc, step scratch in the
library's static device array) against ppm_hydro_step with a caller-owned
workspace, through the C ABI: bit for bit, on two calls in a row, the
second on a smaller level (so the scratch holds the first call's larger
contents), and the refusal of a level whose scratch does not fit."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1008_2801_amd import inputs as I  # noqa: E402
from paper_1008_2801_amd import ppm as P  # noqa: E402
from tests.helpers import interior  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _uneven(seed):
    rng = np.random.default_rng(seed)
    lay = I.tensor_tiling(rng.choice((6, 8, 10), 2), rng.choice((6, 9), 2), rng.choice((5, 8), 2),
                          bc=(0, 0, 0, 0, 2, 2))
    L = tuple((np.array(lay.domain_hi) + 1) / 32.0)
    S = [I.ModeSum(rng, 5, 3, L) for _ in range(5)]

    def prim(x, y, z):
        return (1.2 + 0.4 * S[0](x, y, z), 0.4 * S[1](x, y, z), 0.4 * S[2](x, y, z), 0.4 * S[3](x, y, z),
                1.2 + 0.4 * S[4](x, y, z))
    h = (1.0 / 32,) * 3
    wl = I.Workload("uneven", lay, I._fill_state(lay, h, 1.4, prim), h, 1.4, 1)
    wl.grav = (0.0, 0.0, -1.0)
    return wl


def _both(wl, precision, mode):
    """(noalloc output, workspace output) of one step from the same filled
    state, each with its flux output, dt on the device."""
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma, grav=wl.grav, precision=precision)
    U = torch.from_numpy(wl.arena).cuda()
    lev.fill_boundary(U, mode)
    dtv = lev.compute_dt(U, wl.dx, p)
    outs = []
    for fn in ("ppm_hydro_step_noalloc", "ppm_hydro_step"):
        if fn == "ppm_hydro_step":
            lev.ensure_workspace(precision)  # torch-allocated, set with ppm_set_workspace
            assert lev.workspace_bytes(precision) <= P.NOALLOC_SCRATCH_BYTES
        V = torch.full_like(U, float("nan"))
        F = lev.new_fluxes()
        fl = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in F])
        rc = getattr(P.lib(), fn)(lev.ctx, P._ptr(U), P._ptr(V), fl, 0.0, P._ptr(dtv), P._dp3(*wl.dx),
                                  ctypes.byref(p), int(mode), None)
        assert rc == P.PPM_OK, (fn, rc, P.lib().ppm_last_error(lev.ctx))
        torch.cuda.synchronize()
        outs.append((V.cpu().numpy(), [f.cpu().numpy() for f in F]))
    assert lev.check_status() == 0
    lev.close()
    return outs


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_step_equals_the_workspace_step_on_two_calls(precision):
    big = I.cfg2(40)
    small = _uneven(seed=81)
    assert small.layout.arena_len() < big.layout.arena_len()
    for k, (wl, mode) in enumerate(((big, P.BATCHED), (small, P.PER_BOX))):
        print(f"noalloc call {k}: {wl.name}, {wl.layout.nbox} box(es), precision {precision}, mode {mode}",
              flush=True)
        (a, fa), (b, fb) = _both(wl, precision, mode)
        lay = wl.layout
        for bx in range(lay.nbox):
            assert np.array_equal(interior(lay.view(a, bx)), interior(lay.view(b, bx))), (k, bx)
        for d in range(3):
            assert np.array_equal(fa[d], fb[d]), (k, d)


def test_noalloc_refuses_a_level_whose_scratch_does_not_fit():
    wl = I.cfg2(64)  # 8 (6 72^3 + 91 66^3) bytes: 227 MB in FP64
    lev = P.Level(wl.layout)
    p = P.params(gamma=wl.gamma)
    assert lev.workspace_bytes(0) > P.NOALLOC_SCRATCH_BYTES
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    rc = P.lib().ppm_hydro_step_noalloc(lev.ctx, P._ptr(U), P._ptr(V), None, 1e-3, None, P._dp3(*wl.dx),
                                        ctypes.byref(p), P.BATCHED, None)
    assert rc == P.PPM_EINVAL
    assert b"step scratch" in P.lib().ppm_last_error(lev.ctx)
    # the FP32-reconstruction mode's scratch of the same level fits
    p32 = P.params(gamma=wl.gamma, precision=1)
    assert lev.workspace_bytes(1) <= P.NOALLOC_SCRATCH_BYTES
    lev.fill_boundary(U)
    rc = P.lib().ppm_hydro_step_noalloc(lev.ctx, P._ptr(U), P._ptr(V), None, 1e-3, None, P._dp3(*wl.dx),
                                        ctypes.byref(p32), P.BATCHED, None)
    assert rc == P.PPM_OK
    assert lev.check_status() == 0
    lev.close()

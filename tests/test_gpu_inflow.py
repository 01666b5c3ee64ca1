"""GPU parity of inflow faces (ppm_set_inflow + the fill) and of the
inflowing-jet workload against the oracle.  FP64 bar: per-field max
|gpu - oracle| / max |oracle| <= 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def gpu_jet(wl, nsteps, graph=False):
    lev = P.Level(wl.layout)
    for f, a in wl.meta["inflow"].items():
        lev.set_inflow(f, torch.from_numpy(np.ascontiguousarray(a)).cuda())
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    p = P.params(gamma=wl.gamma)
    dts = []
    if graph:
        g = lev.graph(U, V, wl.dx, p, nsteps)
        g.launch()
        torch.cuda.synchronize()
        out = (U if nsteps % 2 == 0 else V).cpu().numpy()
        g.close()
    else:
        dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
        for _ in range(nsteps):
            lev.fill_boundary(U)
            lev.compute_dt(U, wl.dx, p, out=dtv)
            lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv)
            dts.append(float(dtv[0].item()))
            U, V = V, U
        out = U.cpu().numpy()
    flags = lev.check_status()
    lev.close()
    return out, dts, flags


@pytest.mark.parametrize("graph", [False, True])
def test_jet_matches_oracle(graph):
    wl = I.jet(48, nz=4)
    got, dts, flags = gpu_jet(wl, 30, graph=graph)
    lay = wl.layout
    st = [lay.view(wl.arena, 0).copy()]
    ost, odts, ofl, _ = O.advance(lay.boxes(), lay.domain(), lay.bc, st, 30, wl.dx, O.params(gamma=wl.gamma),
                                  inflow=wl.meta["inflow"])
    assert flags == 0 and ofl == 0
    if not graph:
        assert dts_close(dts, odts)
    parity_report(f"jet 48^2 x 4, 30 steps ({'graph' if graph else 'eager'})",
                  [(interior(lay.view(got, 0)), interior(ost[0]))], TOL)


def test_inflow_on_a_multibox_level_with_walls_matches_oracle():
    lay = I.tensor_tiling([10, 14], [12, 8, 12], [6, 6],
                          bc=(I.BC_REFLECT, I.BC_OUTFLOW, I.BC_INFLOW, I.BC_OUTFLOW, I.BC_PERIODIC, I.BC_PERIODIC))
    h = (1.0 / 32,) * 3
    rng = np.random.default_rng(11)
    S = I.ModeSum(rng, 4, 2, (1.0, 1.0, 1.0))

    # every velocity component away from zero: where a component is zero up
    # to rounding, the tracing switches the entropy-wave term on or off with
    # the sign of that rounding (a discontinuity of the scheme at u_n = 0),
    # and the kernels and the oracle round differently
    def prim(x, y, z):
        return (1.0 + 0.2 * S(x, y, z), 0.05, 0.1, 0.05, 1.0)
    wl = I.Workload("inflow_boxes", lay, I._fill_state(lay, h, 1.4, prim), h, 1.4, 1)
    face = np.zeros((5, 12, 24))
    x = (np.arange(24) + 0.5) * h[0]
    v = 0.3 + 0.2 * np.sin(2 * np.pi * x)
    face[0] = 0.8
    face[1] = 0.8 * 0.05
    face[2] = 0.8 * v[None, :]
    face[4] = 1.1 / 0.4 + 0.5 * 0.8 * (0.05 ** 2 + v * v)[None, :]
    wl.meta["inflow"] = {2: face}
    lev = P.Level(lay)
    lev.set_inflow(2, torch.from_numpy(face).cuda())
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    p = P.params(gamma=1.4)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    for mode in (P.BATCHED, P.PER_BOX):
        U = torch.from_numpy(wl.arena).cuda()
        for _ in range(4):
            lev.fill_boundary(U, mode)
            lev.compute_dt(U, wl.dx, p, out=dtv)
            lev.hydro_step(U, V, wl.dx, p, dt_dev=dtv, mode=mode)
            U, V = V, U
        got = U.cpu().numpy()
        st = [lay.view(wl.arena, b).copy() for b in range(lay.nbox)]
        ost, _, ofl, _ = O.advance(lay.boxes(), lay.domain(), lay.bc, st, 4, wl.dx, O.params(gamma=1.4),
                                   inflow=wl.meta["inflow"])
        assert ofl == 0 and lev.check_status() == 0
        parity_report(f"inflow level with a wall, mode {mode}, 4 steps",
                      [(interior(lay.view(got, b)), interior(ost[b])) for b in range(lay.nbox)], TOL)
    lev.close()


def test_inflow_errors():
    wl = I.jet(16, nz=4)
    lev = P.Level(wl.layout)
    U = torch.from_numpy(wl.arena).cuda()
    with pytest.raises(P.PPMError, match="inflow"):
        lev.fill_boundary(U)
    with pytest.raises(P.PPMError, match="not an inflow face"):
        lev.set_inflow(0, torch.zeros(5 * 4 * 16, dtype=torch.float64, device="cuda"))
    lev.set_inflow(2, torch.from_numpy(wl.meta["inflow"][2]).cuda())
    lev.fill_boundary(U)
    R = lev.new_species(1)
    with pytest.raises(P.PPMError, match="inflow"):
        lev.fill_species(R, 1)
    torch.cuda.synchronize()
    lev.close()


def test_jet_to_300_microseconds_stays_symmetric():
    """The paper's run length on a 256^2 x 4 grid (about 5,000 steps): the
    flow stays mirror symmetric about the jet axis (to the rounding of the
    sampled profile), positive, and the acoustic wave launched at the inflow
    face has reached the far side."""
    wl = I.jet(256, nz=4)
    lev = P.Level(wl.layout)
    lev.set_inflow(2, torch.from_numpy(wl.meta["inflow"][2]).cuda())
    U = torch.from_numpy(wl.arena).cuda()
    V = lev.new_state()
    p = P.params(gamma=wl.gamma)
    dtv = torch.zeros(2, dtype=torch.float64, device="cuda")
    t, t_end, nsteps = 0.0, wl.meta["t_end"], 0
    while t < t_end * (1 - 1e-12):
        lev.fill_boundary(U)
        lev.compute_dt(U, wl.dx, p, out=dtv)
        dt = min(float(dtv[0].item()), t_end - t)
        lev.hydro_step(U, V, wl.dx, p, dt=dt)
        U, V = V, U
        t += dt
        nsteps += 1
        if nsteps % 1000 == 0:
            print(f"jet: {nsteps} steps, t = {t:.3e} s", flush=True)
    assert lev.check_status() == 0
    A = interior(wl.layout.view(U.cpu().numpy(), 0))
    M = np.flip(A, axis=3).copy()
    M[1] = -M[1]
    scale = np.abs(A).max(axis=(1, 2, 3))
    scale[1] = scale[3] = scale[2]
    err = (np.abs(A - M).max(axis=(1, 2, 3)) / scale).max()
    assert err <= 1e-8, err
    assert (A[0] > 0).all()
    rho0 = wl.meta["rho0"]
    top = A[0, :, -8:, :]
    assert np.abs(top - rho0).max() > 1e-4 * rho0  # the acoustic signal reached the far side
    print(f"jet 256^2 x 4 to t = 300 us: {nsteps} steps, symmetry error {err:.2e}")
    lev.close()

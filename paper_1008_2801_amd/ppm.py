"""Python binding of the C ABI in include/ppm.h (argument marshalling only).

Every step of the path runs in the HIP kernels of libppm.so; this module
converts Python/torch arguments into pointers and sizes.  PyTorch provides
device memory and the current stream.  There is no CPU fallback: if the
library is missing, or no GPU is present, the calls raise.
"""
import ctypes
import os

import numpy as np

from . import inputs as _inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppm.so")

PPM_OK, PPM_EINVAL, PPM_EHIP, PPM_ENONPHYS = 0, 1, 2, 3
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
FLAG_NONPHYS, FLAG_FLOOR, FLAG_RANGE = 1, 2, 4
BATCHED, PER_BOX = 0, 1

# Every exported symbol of include/ppm.h.
SYMBOLS = ("ppm_ctx_create", "ppm_ctx_destroy", "ppm_last_error", "ppm_layout_offsets",
           "ppm_flux_offsets", "ppm_workspace_bytes", "ppm_set_workspace", "ppm_fill_boundary",
           "ppm_compute_dt", "ppm_hydro_step", "ppm_graph_create", "ppm_graph_launch",
           "ppm_graph_destroy", "ppm_check_status", "ppm_plan_build", "ppm_fill_boundary_host",
           "ppm_plan_cache_stats", "ppm_profile_enable", "ppm_profile_read",
           "ppm_adjoint_workspace_bytes", "ppm_set_adjoint_workspace", "ppm_hydro_step_adjoint",
           "ppm_set_tiling", "ppm_get_tiling", "ppm_autotune", "ppm_species_offsets",
           "ppm_species_workspace_bytes", "ppm_set_species_workspace", "ppm_fill_species",
           "ppm_hydro_step_species", "ppm_amr_create", "ppm_amr_destroy", "ppm_amr_last_error",
           "ppm_amr_sizes", "ppm_amr_fill_fine", "ppm_amr_step", "ppm_set_inflow",
           "ppm_hydro_step_adjoint_saved", "ppm_set_step_form", "ppm_get_step_form",
           "ppm_hydro_step_dt", "ppm_hydro_step_noalloc",
           "ppm_set_stream_tiling", "ppm_get_stream_tiling", "ppm_set_front_form", "ppm_get_front_form",
           "ppm_set_front_tiling", "ppm_get_front_tiling")
# Every exported symbol of include/ppm_diag.h (libppm_diag.so).
DIAG_SYMBOLS = ("ppm_diag_sqrt_values", "ppm_diag_quotient_values", "ppm_diag_div31_params",
                "ppm_diag_div31_values")
DIAG_LIB_PATH = os.path.join(HERE, "libppm_diag.so")
NOALLOC_SCRATCH_BYTES = 128 << 20
MAX_SPECIES = 64
PROF_TAGS = ("fill", "dt", "prim", "flatten", "trace", "riemann1", "riemann2", "riemann3", "update")


class PPMError(RuntimeError):
    pass


class Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3)]


class LayoutC(ctypes.Structure):
    _fields_ = [("nbox", ctypes.c_int32), ("boxes", ctypes.POINTER(Box)), ("domain", Box),
                ("bc", ctypes.c_int32 * 6), ("ngrow", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("small_dens", ctypes.c_double), ("small_pres", ctypes.c_double),
                ("grav", ctypes.c_double * 3), ("limiter", ctypes.c_int32),
                ("flattening", ctypes.c_int32), ("riemann_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


def params(gamma=1.4, cfl=0.5, small_dens=1e-12, small_pres=1e-12, grav=(0.0, 0.0, 0.0), limiter=1,
           flattening=1, riemann_iters=3, precision=0):
    p = Params()
    p.gamma, p.cfl, p.small_dens, p.small_pres = gamma, cfl, small_dens, small_pres
    for d in range(3):
        p.grav[d] = float(grav[d])
    p.limiter, p.flattening, p.riemann_iters, p.precision = limiter, flattening, riemann_iters, precision
    return p


_lib = None
_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp3 = ctypes.c_double * 3


def lib():
    """Load libppm.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PPMError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.ppm_ctx_create.argtypes = [ctypes.POINTER(LayoutC), ctypes.POINTER(_vp)]
        L.ppm_ctx_destroy.argtypes = [_vp]
        L.ppm_last_error.argtypes = [_vp]
        L.ppm_last_error.restype = ctypes.c_char_p
        L.ppm_layout_offsets.argtypes = [_vp, _i64p]
        L.ppm_flux_offsets.argtypes = [_vp, ctypes.c_int32, _i64p]
        L.ppm_workspace_bytes.argtypes = [_vp, ctypes.c_int32]
        L.ppm_workspace_bytes.restype = ctypes.c_size_t
        L.ppm_set_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.ppm_fill_boundary.argtypes = [_vp, _vp, ctypes.c_int32, _vp]
        L.ppm_compute_dt.argtypes = [_vp, _vp, _dp3, ctypes.POINTER(Params), _vp, _vp]
        L.ppm_hydro_step.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_vp), ctypes.c_double, _vp, _dp3,
                                     ctypes.POINTER(Params), ctypes.c_int32, _vp]
        L.ppm_hydro_step_dt.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_vp), ctypes.c_double, _vp, _dp3,
                                        ctypes.POINTER(Params), ctypes.c_int32, _vp, _vp]
        L.ppm_hydro_step_noalloc.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_vp), ctypes.c_double, _vp, _dp3,
                                             ctypes.POINTER(Params), ctypes.c_int32, _vp]
        L.ppm_graph_create.argtypes = [_vp, _vp, _vp, _dp3, ctypes.POINTER(Params), ctypes.c_int32, _vp,
                                       ctypes.POINTER(_vp)]
        L.ppm_graph_launch.argtypes = [_vp, _vp]
        L.ppm_graph_destroy.argtypes = [_vp]
        L.ppm_check_status.argtypes = [_vp, _vp, _i32p]
        L.ppm_plan_build.argtypes = [ctypes.POINTER(LayoutC), ctypes.c_int32, ctypes.c_int32, _i32p, _i32p]
        L.ppm_fill_boundary_host.argtypes = [ctypes.POINTER(LayoutC), ctypes.POINTER(ctypes.c_double)]
        L.ppm_plan_cache_stats.argtypes = [_i64p, _i64p, _i32p]
        L.ppm_profile_enable.argtypes = [_vp, ctypes.c_int32]
        L.ppm_set_tiling.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
        L.ppm_get_tiling.argtypes = [_vp, _i32p, _i32p]
        L.ppm_autotune.argtypes = [_vp, _vp, _vp, _dp3, ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_char_p,
                                   _vp, _i32p, _i32p, _i32p]
        L.ppm_adjoint_workspace_bytes.argtypes = [_vp, ctypes.c_int32]
        L.ppm_adjoint_workspace_bytes.restype = ctypes.c_size_t
        L.ppm_set_adjoint_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.ppm_hydro_step_adjoint.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_vp), _vp, ctypes.c_double, _vp, _dp3,
                                             ctypes.POINTER(Params), _vp]
        L.ppm_profile_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _i64p]
        L.ppm_hydro_step_adjoint_saved.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_vp), _vp, ctypes.c_double, _vp,
                                                   _dp3, ctypes.POINTER(Params), _vp]
        L.ppm_set_inflow.argtypes = [_vp, ctypes.c_int32, _vp]
        L.ppm_set_step_form.argtypes = [_vp, ctypes.c_int32]
        L.ppm_get_step_form.argtypes = [_vp, _i32p]
        L.ppm_set_stream_tiling.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ppm_get_stream_tiling.argtypes = [_vp, _i32p, _i32p, _i32p]
        L.ppm_set_front_form.argtypes = [_vp, ctypes.c_int32]
        L.ppm_get_front_form.argtypes = [_vp, _i32p]
        L.ppm_set_front_tiling.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ppm_get_front_tiling.argtypes = [_vp, _i32p, _i32p, _i32p]
        L.ppm_amr_create.argtypes = [_vp, _vp, ctypes.POINTER(_vp)]
        L.ppm_amr_destroy.argtypes = [_vp]
        L.ppm_amr_last_error.argtypes = [_vp]
        L.ppm_amr_last_error.restype = ctypes.c_char_p
        L.ppm_amr_sizes.argtypes = [_vp, _i64p, _i64p, _i64p]
        L.ppm_amr_fill_fine.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp]
        L.ppm_amr_step.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _dp3,
                                   ctypes.POINTER(Params), ctypes.c_double, _vp, _vp]
        L.ppm_species_offsets.argtypes = [_vp, ctypes.c_int32, _i64p]
        L.ppm_species_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
        L.ppm_species_workspace_bytes.restype = ctypes.c_size_t
        L.ppm_set_species_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.ppm_fill_species.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp]
        L.ppm_hydro_step_species.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(_vp),
                                             ctypes.c_double, _vp, _dp3, ctypes.POINTER(Params), _vp]
        for name in SYMBOLS:
            f = getattr(L, name)
            if name not in ("ppm_last_error", "ppm_workspace_bytes", "ppm_adjoint_workspace_bytes",
                            "ppm_species_workspace_bytes", "ppm_amr_last_error"):
                f.restype = ctypes.c_int
        _lib = L
    return _lib


def layout_struct(layout):
    """ppm_layout for an inputs.Layout (the struct keeps its box array alive)."""
    nb = layout.nbox
    arr = (Box * nb)()
    for b in range(nb):
        for d in range(3):
            arr[b].lo[d] = int(layout.lo[b, d])
            arr[b].hi[d] = int(layout.hi[b, d])
    L = LayoutC()
    L.nbox = nb
    L.boxes = ctypes.cast(arr, ctypes.POINTER(Box))
    for d in range(3):
        L.domain.lo[d] = int(layout.domain_lo[d])
        L.domain.hi[d] = int(layout.domain_hi[d])
    for f in range(6):
        L.bc[f] = int(layout.bc[f])
    L.ngrow = int(layout.ngrow)
    L._keep = arr
    return L


def plan_build(layout, brute=False):
    """Fill-plan descriptors as an (ndesc, 20) int32 array (host only)."""
    L = layout_struct(layout)
    cnt = ctypes.c_int32(0)
    rc = lib().ppm_plan_build(ctypes.byref(L), int(brute), 0, None, ctypes.byref(cnt))
    if rc != PPM_OK:
        raise PPMError(f"ppm_plan_build failed ({rc})")
    out = np.zeros((cnt.value, 20), dtype=np.int32)
    rc = lib().ppm_plan_build(ctypes.byref(L), int(brute), cnt.value,
                              out.ctypes.data_as(_i32p), ctypes.byref(cnt))
    if rc != PPM_OK:
        raise PPMError(f"ppm_plan_build failed ({rc})")
    return out


def fill_boundary_host(layout, arena):
    """Executes the cached fill plan on a host float64 arena (in place)."""
    assert arena.dtype == np.float64 and arena.flags.c_contiguous
    L = layout_struct(layout)
    rc = lib().ppm_fill_boundary_host(ctypes.byref(L), arena.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != PPM_OK:
        raise PPMError(f"ppm_fill_boundary_host failed ({rc})")
    return arena


def plan_cache_stats():
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    lib().ppm_plan_cache_stats(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


_diag_handle = None


def diag_lib():
    """The arithmetic diagnostics library (include/ppm_diag.h)."""
    global _diag_handle
    if _diag_handle is None:
        if not os.path.exists(DIAG_LIB_PATH):
            raise PPMError(f"HIP library not built: {DIAG_LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(DIAG_LIB_PATH)
        _vp = ctypes.c_void_p
        L.ppm_diag_sqrt_values.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp]
        L.ppm_diag_quotient_values.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp]
        L.ppm_diag_div31_params.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                            ctypes.POINTER(ctypes.c_int32)]
        L.ppm_diag_div31_values.argtypes = [_vp, ctypes.c_uint32, _vp, ctypes.c_int64, _vp]
        _diag_handle = L
    return _diag_handle


def sqrt_values(x, form=0, stream=None):
    """Device values of one of the Riemann solver's square roots (form 0:
    the FP64 wave-speed factor's, 1: the FP64 sound speeds', 2: the FP32
    wave-speed factor's, of x rounded to float) for the float64 CUDA tensor
    x (diagnostic; ppm_diag_sqrt_values)."""
    import torch
    if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
        raise PPMError("sqrt_values: x must be a contiguous float64 CUDA tensor")
    out = torch.empty_like(x)
    rc = diag_lib().ppm_diag_sqrt_values(_ptr(x), _ptr(out), x.numel(), int(form), _stream(stream))
    if rc != 0:
        raise PPMError(f"ppm_diag_sqrt_values failed ({rc})")
    return out


def quotient_values(a, b, stream=None):
    """Device values of the kernels' FP64 quotient a / b for float64 CUDA
    tensors a, b of one shape (diagnostic; ppm_diag_quotient_values)."""
    import torch
    for t in (a, b):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise PPMError("quotient_values: operands must be contiguous float64 CUDA tensors")
    if a.shape != b.shape:
        raise PPMError("quotient_values: operands differ in shape")
    out = torch.empty_like(a)
    rc = diag_lib().ppm_diag_quotient_values(_ptr(a), _ptr(b), _ptr(out), a.numel(), _stream(stream))
    if rc != 0:
        raise PPMError(f"ppm_diag_quotient_values failed ({rc})")
    return out


def _torch():
    import torch
    return torch


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Level:
    """A level (MultiFAB) on the GPU: the library context for a layout plus
    a torch-owned workspace.  States are torch float64 CUDA tensors of
    length arena_len laid out as in include/ppm.h."""

    def __init__(self, layout):
        import torch
        self.layout = layout
        self._L = layout_struct(layout)
        h = ctypes.c_void_p()
        rc = lib().ppm_ctx_create(ctypes.byref(self._L), ctypes.byref(h))
        if rc != PPM_OK:
            raise PPMError(f"ppm_ctx_create failed ({rc})")
        self.ctx = h
        nb = layout.nbox
        off = np.zeros(nb + 1, dtype=np.int64)
        lib().ppm_layout_offsets(self.ctx, off.ctypes.data_as(_i64p))
        self.offsets = off
        self.flux_offsets = []
        for d in range(3):
            fo = np.zeros(nb + 1, dtype=np.int64)
            lib().ppm_flux_offsets(self.ctx, d, fo.ctypes.data_as(_i64p))
            self.flux_offsets.append(fo)
        assert np.array_equal(off, layout.offsets()), "arena offsets differ from the layout's"
        self._work = None
        self._work_prec = None
        self._slot = None
        self._slots = {}
        self.device = torch.device("cuda")

    def close(self):
        if getattr(self, "ctx", None):
            lib().ppm_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def arena_len(self):
        return int(self.offsets[-1])

    def _check(self, rc, what):
        if rc != PPM_OK:
            msg = lib().ppm_last_error(self.ctx)
            raise PPMError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def workspace_bytes(self, precision=0):
        return int(lib().ppm_workspace_bytes(self.ctx, int(precision)))

    def ensure_workspace(self, precision=0):
        import torch
        need = self.workspace_bytes(precision)
        if self._work is None or self._work.numel() < need + 256:  # room for the 256-byte alignment
            self._work = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self._work.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(lib().ppm_set_workspace(self.ctx, ctypes.c_void_p(aligned), need), "ppm_set_workspace")
        self._work_prec = precision
        self._slot = None

    def new_state(self):
        import torch
        return torch.full((self.arena_len,), float("nan"), dtype=torch.float64, device=self.device)

    def new_fluxes(self):
        import torch
        return [torch.zeros(int(self.flux_offsets[d][-1]), dtype=torch.float64, device=self.device)
                for d in range(3)]

    def set_inflow(self, face, state):
        """Prescribed conserved state of an inflow face: a float64 CUDA
        tensor (5, E_t2, E_t1) over the domain's transverse extents (kept
        alive by the level)."""
        if not hasattr(self, "_inflow"):
            self._inflow = {}
        self._inflow[int(face)] = state
        self._check(lib().ppm_set_inflow(self.ctx, int(face), _ptr(state)), "ppm_set_inflow")

    def fill_boundary(self, U, mode=BATCHED, stream=None):
        self._check(lib().ppm_fill_boundary(self.ctx, _ptr(U), int(mode), _stream(stream)), "ppm_fill_boundary")

    def compute_dt(self, U, dx, p, out=None, stream=None):
        import torch
        out = torch.zeros(2, dtype=torch.float64, device=self.device) if out is None else out
        self._check(lib().ppm_compute_dt(self.ctx, _ptr(U), _dp3(*dx), ctypes.byref(p), _ptr(out),
                                         _stream(stream)), "ppm_compute_dt")
        return out

    def hydro_step(self, U, Unew, dx, p, dt=0.0, dt_dev=None, fluxes=None, mode=BATCHED, stream=None,
                   dt_next=None):
        """One step U -> Unew.  dt_next: a device float64 tensor of 2 that
        receives the next step's dt from the valid zones of Unew, computed
        by the update (ppm_hydro_step_dt); it may be dt_dev itself."""
        if self._slot is None and (self._work is None or self._work_prec != p.precision or
                                   self._work.numel() < self.workspace_bytes(p.precision)):
            self.ensure_workspace(p.precision)
        fl = None
        if fluxes is not None:
            fl = (_vp * 3)(*[f.data_ptr() if f is not None else None for f in fluxes])
        if dt_next is None:
            self._check(lib().ppm_hydro_step(self.ctx, _ptr(U), _ptr(Unew), fl, float(dt), _ptr(dt_dev),
                                             _dp3(*dx), ctypes.byref(p), int(mode), _stream(stream)),
                        "ppm_hydro_step")
            return
        if dt_next.dtype != _torch().float64 or not dt_next.is_cuda or dt_next.numel() < 2:
            raise PPMError("hydro_step: dt_next must be a float64 CUDA tensor of 2 elements")
        self._check(lib().ppm_hydro_step_dt(self.ctx, _ptr(U), _ptr(Unew), fl, float(dt), _ptr(dt_dev),
                                            _dp3(*dx), ctypes.byref(p), int(mode), _ptr(dt_next),
                                            _stream(stream)),
                    "ppm_hydro_step_dt")

    def profile_enable(self, on=True):
        self._check(lib().ppm_profile_enable(self.ctx, int(bool(on))), "ppm_profile_enable")

    def profile_read(self):
        """{stage: (total ms, launches)} of the launches timed since the last read."""
        n = len(PROF_TAGS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._check(lib().ppm_profile_read(self.ctx, ms, cnt), "ppm_profile_read")
        return {PROF_TAGS[k]: (ms[k], cnt[k]) for k in range(n)}

    def set_tiling(self, tile, strip_rows):
        self._check(lib().ppm_set_tiling(self.ctx, int(tile), int(strip_rows)), "ppm_set_tiling")

    def set_step_form(self, fused):
        """0/False: the staged final-flux and update kernels; 1/True: one
        brick kernel (fluxes in LDS); 2: the streamed kernel (x-y tiles
        walked along z).  Same results."""
        self._check(lib().ppm_set_step_form(self.ctx, int(fused)), "ppm_set_step_form")

    def get_step_form(self):
        f = ctypes.c_int32()
        self._check(lib().ppm_get_step_form(self.ctx, ctypes.byref(f)), "ppm_get_step_form")
        return f.value

    def set_stream_tiling(self, sx, sy, sz):
        self._check(lib().ppm_set_stream_tiling(self.ctx, int(sx), int(sy), int(sz)), "ppm_set_stream_tiling")

    def set_front_form(self, form):
        """0: trace and stage-1 solves as two staged kernels; 1: one kernel
        streamed along z; 2: the x axis fused, y and z staged; 3: every
        axis fused (ppm_set_front_form)."""
        self._check(lib().ppm_set_front_form(self.ctx, int(form)), "ppm_set_front_form")

    def get_front_form(self):
        v = ctypes.c_int32()
        self._check(lib().ppm_get_front_form(self.ctx, ctypes.byref(v)), "ppm_get_front_form")
        return v.value

    def set_front_tiling(self, sx, sy, sz):
        self._check(lib().ppm_set_front_tiling(self.ctx, int(sx), int(sy), int(sz)), "ppm_set_front_tiling")

    def get_front_tiling(self):
        v = [ctypes.c_int32() for _ in range(3)]
        self._check(lib().ppm_get_front_tiling(self.ctx, *[ctypes.byref(x) for x in v]), "ppm_get_front_tiling")
        return tuple(x.value for x in v)

    def get_stream_tiling(self):
        v = [ctypes.c_int32() for _ in range(3)]
        self._check(lib().ppm_get_stream_tiling(self.ctx, *[ctypes.byref(x) for x in v]), "ppm_get_stream_tiling")
        return tuple(x.value for x in v)

    def get_tiling(self):
        t, s = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().ppm_get_tiling(self.ctx, ctypes.byref(t), ctypes.byref(s)), "ppm_get_tiling")
        return t.value, s.value

    def autotune(self, U, dx, p, reps=3, cache_path=None, stream=None):
        """Pick the tiling by timing the batched step from U (ghosts filled);
        returns (tile, strip_rows, from_cache)."""
        if self._work is None or self._work_prec != p.precision or self._work.numel() < self.workspace_bytes(p.precision):
            self.ensure_workspace(p.precision)
        scratch = self.new_state()
        t, s, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        path = None if cache_path is None else str(cache_path).encode()
        self._check(lib().ppm_autotune(self.ctx, _ptr(U), _ptr(scratch), _dp3(*dx), ctypes.byref(p), int(reps),
                                       path, _stream(stream), ctypes.byref(t), ctypes.byref(s), ctypes.byref(c)),
                    "ppm_autotune")
        return t.value, s.value, bool(c.value)

    def ensure_adjoint_workspace(self, precision=0):
        import torch
        need = int(lib().ppm_adjoint_workspace_bytes(self.ctx, int(precision)))
        if getattr(self, "_awork", None) is None or self._awork.numel() < need + 256:
            self._awork = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self._awork.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(lib().ppm_set_adjoint_workspace(self.ctx, ctypes.c_void_p(aligned), need),
                    "ppm_set_adjoint_workspace")

    def hydro_step_adjoint(self, U, Unew_bar, U_bar, dx, p, dt=0.0, dt_dev=None, stream=None, saved=False,
                           flux_bar=None):
        """U_bar = J^T (Unew_bar, flux_bar) for the step from U (ghosts
        filled), dt frozen; flux_bar: None or three flux-arena tensors (any
        None) holding the adjoints of the step's flux outputs.  The reverse
        runs in the step's precision (p.precision).  saved=True: the
        selected workspace still holds this step's forward intermediates
        (no recompute)."""
        prec = int(p.precision)
        if self._slot is None and (self._work is None or self._work_prec != prec or
                                   self._work.numel() < self.workspace_bytes(prec) + 256):
            self.ensure_workspace(prec)
        if getattr(self, "_awork", None) is None or getattr(self, "_awork_prec", None) != prec:
            self.ensure_adjoint_workspace(prec)
            self._awork_prec = prec
        fn = lib().ppm_hydro_step_adjoint_saved if saved else lib().ppm_hydro_step_adjoint
        fb = None
        if flux_bar is not None:
            fb = (_vp * 3)(*[f.data_ptr() if f is not None else None for f in flux_bar])
        self._check(fn(self.ctx, _ptr(U), _ptr(Unew_bar), fb, _ptr(U_bar), float(dt), _ptr(dt_dev), _dp3(*dx),
                       ctypes.byref(p), _stream(stream)), "ppm_hydro_step_adjoint")

    def select_workspace(self, slot, precision=0):
        """Make workspace slot `slot` (allocated on first use) the step
        workspace, or the default one for slot None.  A checkpoint segment
        keeps one slot per step so that its adjoints need no recompute."""
        import torch
        if slot is None:
            self._slot = None
            self.ensure_workspace(precision)
            return
        need = self.workspace_bytes(precision)
        t = self._slots.get(slot)
        if t is None or t.numel() < need + 256:
            t = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            self._slots[slot] = t
        aligned = (t.data_ptr() + 255) // 256 * 256
        self._check(lib().ppm_set_workspace(self.ctx, ctypes.c_void_p(aligned), need), "ppm_set_workspace")
        self._slot = slot

    def release_workspace_slots(self):
        self._slots = {}
        if self._slot is not None:
            self._slot = None
            self.ensure_workspace(self._work_prec or 0)

    # ------------------------------------------------ passive species ----
    def species_offsets(self, ns):
        """Element offsets (nbox + 1) of each box in a species arena of ns
        components."""
        off = np.zeros(self.layout.nbox + 1, dtype=np.int64)
        self._check(lib().ppm_species_offsets(self.ctx, int(ns), off.ctypes.data_as(_i64p)), "ppm_species_offsets")
        return off

    def new_species(self, ns):
        import torch
        return torch.full((int(self.species_offsets(ns)[-1]),), float("nan"), dtype=torch.float64,
                          device=self.device)

    def species_view(self, RX, ns, b):
        """Box b of a species arena as (ns, Nz, Ny, Nx)."""
        o = self.species_offsets(ns)
        return RX[int(o[b]):int(o[b + 1])].view((int(ns),) + tuple(self.layout.stored_shape(b)[1:]))

    def ensure_species_workspace(self, ns, precision=0):
        import torch
        need = int(lib().ppm_species_workspace_bytes(self.ctx, int(ns), int(precision)))
        if need == 0:
            raise PPMError(f"species workspace: invalid ns={ns} or precision={precision}")
        if getattr(self, "_swork", None) is None or self._swork.numel() < need + 256:
            self._swork = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self._swork.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(lib().ppm_set_species_workspace(self.ctx, ctypes.c_void_p(aligned), need),
                    "ppm_set_species_workspace")
        self._swork_key = (int(ns), int(precision))

    def fill_species(self, RX, ns, mode=BATCHED, stream=None):
        self._check(lib().ppm_fill_species(self.ctx, _ptr(RX), int(ns), int(mode), _stream(stream)),
                    "ppm_fill_species")

    def hydro_step_species(self, U, Unew, RX, RXnew, ns, dx, p, dt=0.0, dt_dev=None, fluxes=None, stream=None):
        """The batched step from U to Unew and the species update from RX to
        RXnew (ghosts of U and RX filled)."""
        prec = int(p.precision)
        if self._work is None or self._work_prec != prec or self._work.numel() < self.workspace_bytes(prec) + 256:
            self.ensure_workspace(prec)
        if getattr(self, "_swork_key", None) != (int(ns), prec):
            self.ensure_species_workspace(ns, prec)
        fl = None
        if fluxes is not None:
            fl = (_vp * 3)(*[f.data_ptr() if f is not None else None for f in fluxes])
        self._check(lib().ppm_hydro_step_species(self.ctx, _ptr(U), _ptr(Unew), _ptr(RX), _ptr(RXnew), int(ns), fl,
                                                 float(dt), _ptr(dt_dev), _dp3(*dx), ctypes.byref(p),
                                                 _stream(stream)),
                    "ppm_hydro_step_species")

    def check_status(self, stream=None):
        f = ctypes.c_int32(0)
        rc = lib().ppm_check_status(self.ctx, _stream(stream), ctypes.byref(f))
        if rc not in (PPM_OK, PPM_ENONPHYS):
            self._check(rc, "ppm_check_status")
        return f.value

    def graph(self, Ua, Ub, dx, p, nsteps, stream=None):
        return Graph(self, Ua, Ub, dx, p, nsteps, stream)

    def box_view(self, U, b):
        """Box b of a state tensor as (5, Nz, Ny, Nx)."""
        o = self.offsets
        return U[int(o[b]):int(o[b + 1])].view(self.layout.stored_shape(b))

    def flux_view(self, F, d, b):
        nx, ny, nz = self.layout.n(b)
        e = [nx, ny, nz]
        e[d] += 1
        o = self.flux_offsets[d]
        return F[int(o[b]):int(o[b + 1])].view(5, e[2], e[1], e[0])


class TwoLevel:
    """Two-level hierarchy (ratio 2, subcycling) on the GPU: a coarse Level,
    a fine Level whose layout is the refinement of a rectangle of coarse
    zones with coarse-fine faces, the library's hierarchy object and the
    six flux arenas the coarse step needs."""

    def __init__(self, coarse_layout, fine_layout):
        self.coarse = Level(coarse_layout)
        self.fine = Level(fine_layout)
        h = ctypes.c_void_p()
        rc = lib().ppm_amr_create(self.coarse.ctx, self.fine.ctx, ctypes.byref(h))
        if rc != PPM_OK:
            msg = lib().ppm_last_error(self.coarse.ctx)
            raise PPMError(f"ppm_amr_create failed ({rc}): {msg.decode() if msg else ''}")
        self.amr = h
        self.Fc = self.coarse.new_fluxes()
        self.Ff = self.fine.new_fluxes()

    def close(self):
        if getattr(self, "amr", None):
            lib().ppm_amr_destroy(self.amr)
            self.amr = None
        for lev in (getattr(self, "fine", None), getattr(self, "coarse", None)):
            if lev is not None:
                lev.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != PPM_OK:
            msg = lib().ppm_amr_last_error(self.amr)
            raise PPMError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def sizes(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().ppm_amr_sizes(self.amr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                    "ppm_amr_sizes")
        return {"interp_zones": a.value, "register_faces": b.value, "covered_zones": c.value}

    def fill_fine(self, Uc_old, Uc_new, half, Uf, stream=None):
        self._check(lib().ppm_amr_fill_fine(self.amr, _ptr(Uc_old), _ptr(Uc_new), int(half), _ptr(Uf),
                                            _stream(stream)), "ppm_amr_fill_fine")

    def step(self, Uc, Uc_new, Uf, Uf_tmp, dxc, p, dt=0.0, dt_out=None, stream=None):
        """One coarse step: Uc -> Uc_new (synchronised), Uf -> Uf (two fine
        steps through Uf_tmp).  dt = 0: the CFL rule of both levels."""
        for lev in (self.coarse, self.fine):
            if lev._work is None or lev._work_prec != p.precision or \
                    lev._work.numel() < lev.workspace_bytes(p.precision) + 256:
                lev.ensure_workspace(p.precision)
        fc = (_vp * 3)(*[f.data_ptr() for f in self.Fc])
        ff = (_vp * 3)(*[f.data_ptr() for f in self.Ff])
        self._check(lib().ppm_amr_step(self.amr, _ptr(Uc), _ptr(Uc_new), _ptr(Uf), _ptr(Uf_tmp), fc, ff,
                                       _dp3(*dxc), ctypes.byref(p), float(dt), _ptr(dt_out), _stream(stream)),
                    "ppm_amr_step")


class Graph:
    """nsteps batched steps [fill, dt, step] captured in a HIP graph, A -> B -> A ..."""

    def __init__(self, level, Ua, Ub, dx, p, nsteps, stream=None):
        import torch
        level.ensure_workspace(p.precision)
        self.level = level
        # the buffers the graph replays from: the states and the workspace
        # it was captured with stay alive while the graph does
        self._keep = (Ua, Ub, level._work)
        g = ctypes.c_void_p()
        # capture needs a stream other than the legacy null stream
        cap = torch.cuda.Stream() if stream is None else stream
        cap.wait_stream(torch.cuda.current_stream())
        level._check(lib().ppm_graph_create(level.ctx, _ptr(Ua), _ptr(Ub), _dp3(*dx), ctypes.byref(p),
                                            int(nsteps), _stream(cap), ctypes.byref(g)),
                     "ppm_graph_create")
        torch.cuda.current_stream().wait_stream(cap)
        self.g = g
        self.nsteps = nsteps

    def launch(self, stream=None):
        self.level._check(lib().ppm_graph_launch(self.g, _stream(stream)), "ppm_graph_launch")

    def close(self):
        if getattr(self, "g", None):
            lib().ppm_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_levels = {}


def hydro_step(boxes, U, dt, dx, gamma, bc=(0, 0, 0, 0, 0, 0), domain=None, fluxes=True, **kw):
    """One step of a level: (U', fluxes) = hydro_step(boxes, U, dt, dx, gamma, bc).

    boxes: list of (lo, hi) inclusive index triples tiling the domain (the
    bounding box of the boxes unless `domain` is given); U: float64 CUDA
    tensor state arena (ghosts need not be filled: the fill runs first);
    returns the new state (ghosts unfilled) and, if fluxes, the three flux
    arenas.  Extra keyword arguments go to params()."""
    import torch
    lo = np.array([b[0] for b in boxes], dtype=np.int64)
    hi = np.array([b[1] for b in boxes], dtype=np.int64)
    if domain is None:
        domain = (tuple(lo.min(axis=0)), tuple(hi.max(axis=0)))
    lay = _inputs.Layout(lo, hi, tuple(domain[0]), tuple(domain[1]), tuple(bc))
    key = (lo.tobytes(), hi.tobytes(), tuple(domain[0]), tuple(domain[1]), tuple(bc))
    lev = _levels.get(key)
    if lev is None:
        lev = _levels[key] = Level(lay)
    p = params(gamma=gamma, **kw)
    Uf = U.clone()
    lev.fill_boundary(Uf)
    Un = lev.new_state()
    F = lev.new_fluxes() if fluxes else None
    lev.hydro_step(Uf, Un, dx, p, dt=dt, fluxes=F)
    return Un, F


def _autograd():
    import torch

    class HydroStep(torch.autograd.Function):
        """One step U -> U' of a level as an autograd function (FP64).

        Input: a state arena (valid zones used; ghosts ignored).  Output: the
        new state arena with zero ghosts.  dt: a float or a device tensor
        whose element 0 is dt; it is not differentiated (frozen).  The
        backward applies the hand-written adjoint kernels."""

        @staticmethod
        def forward(ctx, U, level, dt, dx, p):
            Uf = U.detach().clone()
            level.fill_boundary(Uf)
            Un = torch.zeros_like(Uf)
            if torch.is_tensor(dt):
                level.hydro_step(Uf, Un, dx, p, dt_dev=dt)
            else:
                level.hydro_step(Uf, Un, dx, p, dt=dt)
            ctx.level, ctx.dt, ctx.dx, ctx.p = level, dt, dx, p
            ctx.save_for_backward(Uf)
            return Un

        @staticmethod
        def backward(ctx, g):
            (Uf,) = ctx.saved_tensors
            Ub = torch.empty_like(Uf)
            lev = ctx.level
            if torch.is_tensor(ctx.dt):
                lev.hydro_step_adjoint(Uf, g.contiguous(), Ub, ctx.dx, ctx.p, dt_dev=ctx.dt)
            else:
                lev.hydro_step_adjoint(Uf, g.contiguous(), Ub, ctx.dx, ctx.p, dt=ctx.dt)
            return Ub, None, None, None, None

    class Rollout(torch.autograd.Function):
        """nsteps steps with the CFL dt of each step computed in the forward
        pass and frozen; the backward recomputes each segment of
        `every` steps from its checkpoint and runs the step adjoints in
        reverse (memory: the checkpoints plus one segment of states)."""

        @staticmethod
        def forward(ctx, U0, level, nsteps, dx, p, every, dts_in, saved):
            U = U0.detach().clone()
            dts = torch.zeros(nsteps, 2, dtype=torch.float64, device=U.device) if dts_in is None else dts_in
            ckpts = {}
            V = torch.zeros_like(U)
            for k in range(nsteps):
                if k % every == 0:
                    ckpts[k] = U.clone()
                level.fill_boundary(U)
                if dts_in is None:
                    level.compute_dt(U, dx, p, out=dts[k])
                level.hydro_step(U, V, dx, p, dt_dev=dts[k])
                U, V = V, U
            ctx.level, ctx.nsteps, ctx.dx, ctx.p, ctx.every = level, nsteps, dx, p, every
            ctx.ckpts, ctx.dts, ctx.saved = ckpts, dts, saved
            out = U.clone()
            return out

        @staticmethod
        def backward(ctx, g):
            lev, n, every = ctx.level, ctx.nsteps, ctx.every
            g = g.contiguous().clone()
            Ub = torch.empty_like(g)
            m = min(every, n)
            prec = int(ctx.p.precision)
            saved = ctx.saved
            if saved is None:  # keep one workspace per segment step if it fits in half the free memory
                free, _ = torch.cuda.mem_get_info(g.device)
                saved = m * (lev.workspace_bytes(prec) + 256) <= free // 2
            # the filled input states of one segment; without saved
            # workspaces the segment's last step is not replayed (its output
            # is not needed), with them every step runs on its own workspace
            slots = [torch.empty_like(g) for _ in range(m)]
            scratch = torch.empty_like(g) if saved else None
            try:
                for s0 in reversed(range(0, n, every)):
                    s1 = min(n, s0 + every)
                    slots[0].copy_(ctx.ckpts[s0])
                    for k in range(s0, s1):
                        lev.fill_boundary(slots[k - s0])
                        if saved:
                            lev.select_workspace(k - s0, prec)
                            out = slots[k + 1 - s0] if k + 1 < s1 else scratch
                            lev.hydro_step(slots[k - s0], out, ctx.dx, ctx.p, dt_dev=ctx.dts[k])
                        elif k + 1 < s1:
                            lev.hydro_step(slots[k - s0], slots[k + 1 - s0], ctx.dx, ctx.p, dt_dev=ctx.dts[k])
                    for k in reversed(range(s0, s1)):
                        if saved:
                            lev.select_workspace(k - s0, prec)
                        lev.hydro_step_adjoint(slots[k - s0], g, Ub, ctx.dx, ctx.p, dt_dev=ctx.dts[k], saved=saved)
                        g, Ub = Ub, g
            finally:
                if saved:
                    lev.select_workspace(None, prec)
            return g, None, None, None, None, None, None, None

    return HydroStep, Rollout


def hydro_step_autograd(U, level, dt, dx, p):
    HydroStep, _ = _autograd()
    return HydroStep.apply(U, level, dt, dx, p)


def rollout(U0, level, nsteps, dx, p, checkpoint_every=5, dts=None, saved=None):
    """Differentiable roll-out of nsteps (dt per step from the CFL rule,
    frozen; or the given (nsteps, 2) device tensor of [dt, s]).  saved: the
    backward replays each segment with one workspace per step and runs the
    adjoints on the kept intermediates (True), recomputes them in every
    adjoint (False), or chooses by free memory (None)."""
    _, Rollout = _autograd()
    return Rollout.apply(U0, level, nsteps, dx, p, checkpoint_every, dts, saved)


def div31_params(d):
    """The multiplier m and shift s with which the kernels divide zone
    indices below 2^31 by d: floor(n / d) = ((n m) >> 32) >> s (diagnostic,
    host only; ppm_diag_div31_params)."""
    m, sh = ctypes.c_uint32(), ctypes.c_int32()
    rc = diag_lib().ppm_diag_div31_params(int(d), ctypes.byref(m), ctypes.byref(sh))
    if rc != 0:
        raise PPMError(f"ppm_diag_div31_params failed ({rc})")
    return m.value, sh.value


def div31_values(n, d, stream=None):
    """Device values of the kernels' zone-index division floor(n / d) for a
    contiguous int32 CUDA tensor n of dividends in [0, 2^31) (diagnostic;
    ppm_diag_div31_values)."""
    import torch
    if n.dtype != torch.int32 or not n.is_cuda or not n.is_contiguous():
        raise PPMError("div31_values: n must be a contiguous int32 CUDA tensor")
    out = torch.empty_like(n)
    rc = diag_lib().ppm_diag_div31_values(_ptr(n), int(d), _ptr(out), n.numel(), _stream(stream))
    if rc != 0:
        raise PPMError(f"ppm_diag_div31_values failed ({rc})")
    return out

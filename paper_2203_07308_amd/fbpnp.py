"""Thin ctypes binding of libfbpnp (include/fbpnp.h) for torch tensors.

Argument marshalling only: every array must be a contiguous float32 (or int32 for
view lists) tensor on the GPU; the call is enqueued on torch's current stream. All
arithmetic runs in the library's HIP kernels. There is no CPU fallback: a missing
library or a failing call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfbpnp.so")

FB_OK = 0
_STATUS = {-1: "FB_EINVAL", -2: "FB_EGEOM", -3: "FB_EDIV", -4: "FB_ESUBSET", -5: "FB_EHIP", -6: "FB_ENOMEM"}

# every exported entry point, in the order of include/fbpnp.h
EXPORTS = [
    "fb_last_error", "fb_plan_create", "fb_plan_destroy", "fb_plan_stage_info", "fanbeam_fp", "fb_check_views",
    "fanbeam_bp",
    "sketch_down", "sketch_up", "fb_tv_workspace_bytes", "tv_prox", "pnp_step", "fb_graph_create",
    "fb_graph_launch", "fb_graph_destroy", "fb_tv_vjp_workspace_bytes", "tv_prox_vjp",
    "fb_pnp_vjp_workspace_bytes", "pnp_step_vjp", "fb_power_lipschitz", "fb_plan_view_samples",
    "fb_workspace_bytes", "fb_plan_set_config", "fb_plan_get_config", "fb_batch_create", "fb_batch_destroy",
    "fb_batch_layout", "fb_batch_slice_plan", "fb_batch_set_config", "fb_batch_get_config", "fb_batch_prepare",
    "pnp_step_batched",
    "fb_batch_graph_create", "fb_autotune", "fb_batch_autotune", "fb_plan_set_sketch", "fb_plan_sketch_down",
    "fb_plan_sketch_up", "tv_prox_noalloc", "fb_clock_khz", "fb_clock_stamp",
]


class FbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Geom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
        ("n_views", ctypes.c_int32), ("n_bins", ctypes.c_int32),
        ("sod_mm", ctypes.c_double), ("sdd_mm", ctypes.c_double),
        ("det_pitch_mm", ctypes.c_double), ("det_offset_mm", ctypes.c_double),
        ("angle0_rad", ctypes.c_double), ("angle_step_rad", ctypes.c_double),
    ]


class StageInfo(ctypes.Structure):
    _fields_ = [("factor", ctypes.c_int32), ("nxs", ctypes.c_int32), ("nys", ctypes.c_int32),
                ("samples_all_views", ctypes.c_int64)]


class PnpArgs(ctypes.Structure):
    _fields_ = [
        ("stage", ctypes.c_int32), ("views", ctypes.c_void_p), ("n_sel", ctypes.c_int32),
        ("sigma", ctypes.c_float), ("eta", ctypes.c_float), ("alpha", ctypes.c_float), ("a_t", ctypes.c_float),
        ("lambda_", ctypes.c_float), ("tau", ctypes.c_float), ("tv_iters", ctypes.c_int32),
        ("b", ctypes.c_void_p), ("y_prev", ctypes.c_void_p), ("x_prev", ctypes.c_void_p),
        ("x_out", ctypes.c_void_p), ("y_out", ctypes.c_void_p), ("history", ctypes.c_void_p),
        ("next_stage", ctypes.c_int32), ("prepared", ctypes.c_int32),
        ("events", ctypes.POINTER(ctypes.c_void_p)),
        ("vr_mode", ctypes.c_int32), ("snap_proj", ctypes.c_void_p), ("snap_grad", ctypes.c_void_p),
        ("n_sub", ctypes.c_int32), ("subset", ctypes.c_int32), ("grad", ctypes.c_void_p),
        ("stamp", ctypes.c_void_p),
    ]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("fp_seg", ctypes.c_int32), ("bp_px", ctypes.c_int32), ("bp_vg", ctypes.c_int32),
                ("tv_tile", ctypes.c_int32), ("fp_lds", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchArgs(ctypes.Structure):
    _fields_ = [
        ("stage", ctypes.c_int32), ("n_sub", ctypes.c_int32), ("subset", ctypes.c_int32),
        ("sigma", ctypes.c_float), ("alpha", ctypes.c_float), ("a_t", ctypes.c_float),
        ("lambda_", ctypes.c_float), ("tau", ctypes.c_float), ("tv_iters", ctypes.c_int32),
        ("eta", ctypes.c_void_p), ("b", ctypes.c_void_p), ("y_prev", ctypes.c_void_p), ("x_prev", ctypes.c_void_p),
        ("x_out", ctypes.c_void_p), ("y_out", ctypes.c_void_p), ("history", ctypes.c_void_p),
        ("next_stage", ctypes.c_int32), ("prepared", ctypes.c_int32),
        ("events", ctypes.POINTER(ctypes.c_void_p)),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Loads libfbpnp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_07308_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_float, vp = ctypes.c_int, ctypes.c_float, ctypes.c_void_p
    P = ctypes.POINTER
    lib.fb_last_error.restype = ctypes.c_char_p
    lib.fb_last_error.argtypes = []
    lib.fb_plan_create.argtypes = [P(Geom), c_int, P(ctypes.c_int32), P(vp)]
    lib.fb_plan_destroy.argtypes = [vp]
    lib.fb_plan_stage_info.argtypes = [vp, c_int, P(StageInfo)]
    lib.fanbeam_fp.argtypes = [vp, c_int, vp, vp, vp, c_int, vp]
    lib.fanbeam_bp.argtypes = [vp, c_int, vp, vp, vp, c_int, c_float, vp]
    lib.sketch_down.argtypes = [vp, c_int, c_int, c_int, vp, vp]
    lib.sketch_up.argtypes = [vp, c_int, c_int, c_int, vp, vp]
    lib.fb_tv_workspace_bytes.argtypes = [c_int, c_int, c_int]
    lib.fb_tv_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_prox.argtypes = [vp, vp, c_int, c_int, c_float, c_int, c_float, vp, ctypes.c_size_t, vp]
    lib.tv_prox_noalloc.argtypes = [vp, vp, c_int, c_int, c_float, c_int, c_float, vp]
    lib.pnp_step.argtypes = [vp, P(PnpArgs), vp]
    lib.fb_graph_create.argtypes = [vp, P(PnpArgs), c_int, P(vp)]
    lib.fb_graph_launch.argtypes = [vp, vp]
    lib.fb_graph_destroy.argtypes = [vp]
    lib.fb_plan_view_samples.argtypes = [vp, c_int, P(ctypes.c_int64)]
    lib.fb_plan_set_config.argtypes = [vp, c_int, P(LaunchConfig)]
    lib.fb_plan_set_sketch.argtypes = [vp, c_int]
    lib.fb_plan_sketch_down.argtypes = [vp, c_int, vp, vp, vp]
    lib.fb_plan_sketch_up.argtypes = [vp, c_int, vp, vp, vp]
    lib.fb_plan_get_config.argtypes = [vp, c_int, c_int, P(LaunchConfig)]
    lib.fb_batch_create.argtypes = [P(Geom), c_int, c_int, P(ctypes.c_int32), P(vp)]
    lib.fb_batch_destroy.argtypes = [vp]
    lib.fb_batch_layout.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64)]
    lib.fb_batch_slice_plan.argtypes = [vp, c_int, P(vp)]
    lib.fb_batch_set_config.argtypes = [vp, c_int, P(LaunchConfig)]
    lib.fb_batch_get_config.argtypes = [vp, c_int, c_int, P(LaunchConfig)]
    lib.fb_batch_prepare.argtypes = [vp, c_int]
    lib.fb_workspace_bytes.argtypes = [vp, c_int, P(ctypes.c_size_t)]
    lib.pnp_step_batched.argtypes = [vp, P(BatchArgs), vp]
    lib.fb_batch_graph_create.argtypes = [vp, P(BatchArgs), c_int, P(vp)]
    lib.fb_autotune.argtypes = [vp, c_int, ctypes.c_char_p, vp]
    lib.fb_batch_autotune.argtypes = [vp, c_int, ctypes.c_char_p, vp]
    lib.fb_power_lipschitz.argtypes = [vp, c_int, c_int, P(ctypes.c_double), vp]
    lib.fb_tv_vjp_workspace_bytes.argtypes = [c_int, c_int, c_int]
    lib.fb_tv_vjp_workspace_bytes.restype = ctypes.c_size_t
    lib.tv_prox_vjp.argtypes = [vp, vp, vp, c_int, c_int, c_float, c_int, c_float, c_float, vp, ctypes.c_size_t, vp]
    lib.fb_pnp_vjp_workspace_bytes.argtypes = [vp, c_int]
    lib.fb_pnp_vjp_workspace_bytes.restype = ctypes.c_size_t
    lib.pnp_step_vjp.argtypes = [vp, P(PnpArgs), vp, vp, vp, vp, vp, c_int, vp, ctypes.c_size_t, vp]
    lib.fb_check_views.argtypes = [vp, vp, c_int, vp]
    lib.fb_clock_khz.argtypes = []
    lib.fb_clock_stamp.argtypes = [vp, vp]
    for name in EXPORTS:
        if name not in ("fb_last_error", "fb_tv_workspace_bytes", "fb_tv_vjp_workspace_bytes",
                        "fb_pnp_vjp_workspace_bytes"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != FB_OK:
        raise FbError(status, load().fb_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None, dtype=torch.float32, numel: int | None = None, name: str = "tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    pixel_mm: float
    n_views: int
    n_bins: int
    sod_mm: float
    sdd_mm: float
    det_pitch_mm: float
    det_offset_mm: float = 0.0
    angle0_rad: float = 0.0
    angle_step_rad: float | None = None

    def c(self) -> Geom:
        import math

        step = self.angle_step_rad if self.angle_step_rad is not None else 2 * math.pi / max(self.n_views, 1)
        return Geom(self.nx, self.ny, self.pixel_mm, self.n_views, self.n_bins, self.sod_mm, self.sdd_mm,
                    self.det_pitch_mm, self.det_offset_mm, self.angle0_rad, step)


class Plan:
    """Projector plan (fb_plan_create): one geometry, one stage per pooling factor."""

    def __init__(self, geom: Geometry, factors=(1,), _borrowed=None):
        lib = load()
        self.geom = geom
        self.factors = [int(f) for f in factors]
        self._owner = _borrowed  # a plan held by a batch is not destroyed here
        if _borrowed is not None:
            return
        arr = (ctypes.c_int32 * len(self.factors))(*self.factors)
        h = ctypes.c_void_p()
        _check(lib.fb_plan_create(ctypes.byref(geom.c()), len(self.factors), arr, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            if self._owner is None:
                load().fb_plan_destroy(self._h)
            self._h = None

    def set_config(self, stage: int, cfg: dict | None = None) -> None:
        """Launch configuration of a stage (fb_launch_config fields; None or 0: defaults)."""
        c = None if cfg is None else ctypes.byref(LaunchConfig(**cfg))
        _check(load().fb_plan_set_config(self._h, stage, c))

    SKETCHES = {"pool": 0, "bicubic": 1}

    def set_sketch(self, kind: str = "pool") -> None:
        """Sketch of the stages with f > 1: "pool" (f x f average, U = D^T) or "bicubic"
        (Keys' kernel stretched by f, U = S^T); see fb_plan_set_sketch."""
        _check(load().fb_plan_set_sketch(self._h, self.SKETCHES[kind]))

    def sketch_down(self, stage: int, x: torch.Tensor, v: torch.Tensor, stream=None) -> torch.Tensor:
        nys, nxs = self.coarse_shape(stage)
        _check(load().fb_plan_sketch_down(self._h, stage, _ptr(x, numel=self.geom.nx * self.geom.ny, name="x"),
                                          _ptr(v, numel=nxs * nys, name="v"), _stream(stream)))
        return v

    def sketch_up(self, stage: int, v: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
        nys, nxs = self.coarse_shape(stage)
        _check(load().fb_plan_sketch_up(self._h, stage, _ptr(v, numel=nxs * nys, name="v"),
                                        _ptr(x, numel=self.geom.nx * self.geom.ny, name="x"), _stream(stream)))
        return x

    def get_config(self, stage: int, n_sel: int | None = None) -> dict:
        out = LaunchConfig()
        _check(load().fb_plan_get_config(self._h, stage, n_sel or self.geom.n_views, ctypes.byref(out)))
        return out.as_dict()

    def autotune(self, n_sel: int | None = None, cache_path: str | None = None, stream=None) -> None:
        cp = None if cache_path is None else os.fsencode(cache_path)
        _check(load().fb_autotune(self._h, n_sel or self.geom.n_views, cp, _stream(stream)))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stage_info(self, stage: int) -> StageInfo:
        out = StageInfo()
        _check(load().fb_plan_stage_info(self._h, stage, ctypes.byref(out)))
        return out

    def workspace_bytes(self, stage: int) -> int:
        """Bytes of the plan's own device workspace that calls at this stage use."""
        out = ctypes.c_size_t()
        _check(load().fb_workspace_bytes(self._h, stage, ctypes.byref(out)))
        return out.value

    def view_samples(self, stage: int):
        """In-grid Joseph samples of each view at this stage (host list of n_views ints)."""
        out = (ctypes.c_int64 * self.geom.n_views)()
        _check(load().fb_plan_view_samples(self._h, stage, out))
        return list(out)

    def coarse_shape(self, stage: int):
        f = self.factors[stage]
        return (self.geom.ny // f, self.geom.nx // f)


def _views(plan: Plan, views: torch.Tensor | None):
    if views is None:
        return None, plan.geom.n_views
    return _ptr(views, torch.int32, name="views"), views.numel()


def fanbeam_fp(plan: Plan, stage: int, x: torch.Tensor, y: torch.Tensor, views: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    ny, nx = plan.coarse_shape(stage)
    vp, n_sel = _views(plan, views)
    _check(load().fanbeam_fp(plan.handle, stage, _ptr(x, numel=nx * ny, name="x"),
                             _ptr(y, numel=n_sel * plan.geom.n_bins, name="y"), vp, n_sel, _stream(stream)))
    return y


def check_views(plan: Plan, views: torch.Tensor, stream=None) -> None:
    """fb_check_views: raises FbError (FB_ESUBSET) if the device view list holds an index
    outside [0, n_views) or more entries than views; synchronises the stream."""
    vp, n_sel = _views(plan, views)
    _check(load().fb_check_views(plan.handle, vp, n_sel, _stream(stream)))


def fanbeam_bp(plan: Plan, stage: int, y: torch.Tensor, x: torch.Tensor, views: torch.Tensor | None = None,
               scale: float = 1.0, stream=None) -> torch.Tensor:
    ny, nx = plan.coarse_shape(stage)
    vp, n_sel = _views(plan, views)
    _check(load().fanbeam_bp(plan.handle, stage, _ptr(y, numel=n_sel * plan.geom.n_bins, name="y"),
                             _ptr(x, numel=nx * ny, name="x"), vp, n_sel, float(scale), _stream(stream)))
    return x


def sketch_down(x: torch.Tensor, f: int, v: torch.Tensor, stream=None) -> torch.Tensor:
    ny, nx = x.shape
    _check(load().sketch_down(_ptr(x, name="x"), nx, ny, f, _ptr(v, numel=(nx // f) * (ny // f), name="v"),
                              _stream(stream)))
    return v


def sketch_up(v: torch.Tensor, f: int, x: torch.Tensor, stream=None) -> torch.Tensor:
    nys, nxs = v.shape
    _check(load().sketch_up(_ptr(v, name="v"), nxs, nys, f, _ptr(x, numel=nxs * nys * f * f, name="x"),
                            _stream(stream)))
    return x


def tv_workspace_bytes(nx: int, ny: int, n_iter: int) -> int:
    return int(load().fb_tv_workspace_bytes(nx, ny, n_iter))


def tv_prox(z: torch.Tensor, x: torch.Tensor, lam: float, n_iter: int = 5, tau: float = 0.125,
            ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    ny, nx = z.shape
    need = tv_workspace_bytes(nx, ny, n_iter)
    if need and ws is None:
        ws = torch.empty(need // 4, dtype=torch.float32, device=z.device)
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(load().tv_prox(_ptr(z, name="z"), _ptr(x, numel=nx * ny, name="x"), nx, ny, float(lam), int(n_iter),
                          float(tau), None if ws is None else ctypes.c_void_p(ws.data_ptr()), wsb, _stream(stream)))
    return x


def tv_prox_noalloc(z: torch.Tensor, x: torch.Tensor, lam: float, n_iter: int = 5, tau: float = 0.125,
                    stream=None) -> torch.Tensor:
    """tv_prox with the library's static scratch instead of a workspace (at most 2^20 pixels)."""
    ny, nx = z.shape
    _check(load().tv_prox_noalloc(_ptr(z, name="z"), _ptr(x, numel=nx * ny, name="x"), nx, ny, float(lam),
                                  int(n_iter), float(tau), _stream(stream)))
    return x


def pnp_args(plan: Plan, stage: int, b, y_prev, x_prev, x_out, y_out, eta: float, a_t: float,
             views: torch.Tensor | None = None, sigma: float = 1.0, alpha: float = 1.0, lam: float = 0.01,
             tau: float = 0.125, tv_iters: int = 5, history: torch.Tensor | None = None,
             events=None, vr_mode: int = 0, snap_proj: torch.Tensor | None = None,
             snap_grad: torch.Tensor | None = None, subset: tuple[int, int] | None = None,
             grad: torch.Tensor | None = None, stamp: torch.Tensor | None = None) -> PnpArgs:
    """Arguments of one pnp_step. events: optional sequence of six torch.cuda.Event
    (enable_timing=True) or None, recorded around the step's fp, bp and TV kernels.
    vr_mode 1 / 2 with snap_proj [n_views * n_bins] and snap_grad (the stage's coarse
    image size): variance-reduced snapshot / step (see include/fbpnp.h).
    subset = (k, n_sub), with views None: the interleaved subset k, k + n_sub, ...
    of the views, whose indices the kernels compute instead of reading a list.
    grad (the stage's coarse image size): pnp_step stores the coarse gradient there,
    and pnp_step_vjp reads it back instead of recomputing it.
    stamp: one int64 element (a view into a zeroed buffer) that receives the device
    clock at which the step's denoiser kernel finished (see clock_khz)."""
    npix = plan.geom.nx * plan.geom.ny
    if subset is not None and views is not None:
        raise ValueError("pnp_args: give views or subset, not both")
    vp, n_sel = _views(plan, views)
    k_sub, n_sub = (0, 0) if subset is None else (int(subset[0]), int(subset[1]))
    if subset is not None:
        n_sel = len(range(k_sub, plan.geom.n_views, max(n_sub, 1)))
    a = PnpArgs(stage, vp, n_sel, sigma, eta, alpha, a_t, lam, tau, tv_iters,
                _ptr(b, numel=plan.geom.n_views * plan.geom.n_bins, name="b"),
                _ptr(y_prev, numel=npix, name="y_prev"), _ptr(x_prev, numel=npix, name="x_prev"),
                _ptr(x_out, numel=npix, name="x_out"), _ptr(y_out, numel=npix, name="y_out"),
                _ptr(history, numel=npix, name="history"), -1, 0)
    a.n_sub, a.subset = n_sub, k_sub
    if vr_mode:
        nys, nxs = plan.coarse_shape(stage)
        a.vr_mode = vr_mode
        a.snap_proj = _ptr(snap_proj, numel=plan.geom.n_views * plan.geom.n_bins, name="snap_proj")
        a.snap_grad = _ptr(snap_grad, numel=nxs * nys, name="snap_grad")
    if grad is not None:
        nys, nxs = plan.coarse_shape(stage)
        a.grad = _ptr(grad, numel=nxs * nys, name="grad")
    if stamp is not None:
        if stamp.dtype != torch.int64 or not stamp.is_cuda or stamp.numel() < 1:
            raise ValueError("stamp: need a CUDA int64 tensor with at least one element")
        a.stamp = stamp.data_ptr()
    if events is not None:
        if len(events) != 6:
            raise ValueError("events: need six entries (fp, bp, TV; begin and end)")
        a.events = _events(events)  # the struct keeps the array alive
    return a


def chain_steps(steps) -> None:
    """Sets next_stage / prepared on consecutive step arguments the way fb_graph_create
    does (step i pools y_t for step i + 1 when that step reads it), for a schedule run
    by direct pnp_step calls in this order."""
    for a in steps:
        a.next_stage, a.prepared = -1, 0
    for a, b in zip(steps[:-1], steps[1:]):
        if b.y_prev == a.y_out:
            a.next_stage, b.prepared = b.stage, 1


def clock_khz() -> int:
    """Ticks per millisecond of the device clock behind step stamps (0 if unknown)."""
    return int(load().fb_clock_khz())


def clock_stamp(dst: torch.Tensor, stream=None) -> None:
    """Writes the device clock to dst (one CUDA int64 element) when the stream gets there."""
    if dst.dtype != torch.int64 or not dst.is_cuda or dst.numel() < 1:
        raise ValueError("clock_stamp: need a CUDA int64 tensor with at least one element")
    _check(load().fb_clock_stamp(ctypes.c_void_p(dst.data_ptr()), _stream(stream)))


def pnp_step(plan: Plan, args: PnpArgs, stream=None) -> None:
    _check(load().pnp_step(plan.handle, ctypes.byref(args), _stream(stream)))


class Graph:
    """A schedule of pnp_step calls captured into one HIP graph (fb_graph_create)."""

    def __init__(self, plan: Plan, steps):
        arr = (PnpArgs * len(steps))(*steps)
        h = ctypes.c_void_p()
        _check(load().fb_graph_create(plan.handle, arr, len(steps), ctypes.byref(h)))
        self._h = h
        self._plan = plan  # keep the plan alive

    def launch(self, stream=None):
        _check(load().fb_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().fb_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many slices advanced together (fb_batch_create): geometries may differ, the
    stage factors are shared. Images and sinograms live in packed arenas whose
    offsets (floats) are image_offsets / sino_offsets."""

    def __init__(self, geoms, factors=(1,)):
        lib = load()
        self.geoms = list(geoms)
        self.factors = [int(f) for f in factors]
        n = len(self.geoms)
        garr = (Geom * n)(*[g.c() for g in self.geoms])
        farr = (ctypes.c_int32 * len(self.factors))(*self.factors)
        h = ctypes.c_void_p()
        _check(lib.fb_batch_create(garr, n, len(self.factors), farr, ctypes.byref(h)))
        self._h = h
        io, so = (ctypes.c_int64 * (n + 1))(), (ctypes.c_int64 * (n + 1))()
        _check(lib.fb_batch_layout(h, io, so))
        self.image_offsets, self.sino_offsets = list(io), list(so)
        self.image_size, self.sino_size = self.image_offsets[-1], self.sino_offsets[-1]

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return len(self.geoms)

    def slice_plan(self, i: int) -> Plan:
        """The batch's own plan of slice i (shares its workspace; not for concurrent use)."""
        h = ctypes.c_void_p()
        _check(load().fb_batch_slice_plan(self._h, i, ctypes.byref(h)))
        p = Plan(self.geoms[i], self.factors, _borrowed=self)
        p._h = h
        return p

    def image(self, arena: torch.Tensor, i: int) -> torch.Tensor:
        g = self.geoms[i]
        o = self.image_offsets[i]
        return arena[o:o + g.nx * g.ny].view(g.ny, g.nx)

    def sinogram(self, arena: torch.Tensor, i: int) -> torch.Tensor:
        g = self.geoms[i]
        o = self.sino_offsets[i]
        return arena[o:o + g.n_views * g.n_bins].view(g.n_views, g.n_bins)

    def set_config(self, stage: int, cfg: dict | None = None) -> None:
        c = None if cfg is None else ctypes.byref(LaunchConfig(**cfg))
        _check(load().fb_batch_set_config(self._h, stage, c))

    def get_config(self, stage: int, n_sub: int = 1) -> dict:
        out = LaunchConfig()
        _check(load().fb_batch_get_config(self._h, stage, n_sub, ctypes.byref(out)))
        return out.as_dict()

    def autotune(self, n_sub: int = 1, cache_path: str | None = None, stream=None) -> None:
        cp = None if cache_path is None else os.fsencode(cache_path)
        _check(load().fb_batch_autotune(self._h, n_sub, cp, _stream(stream)))

    def prepare(self, n_sub: int) -> None:
        """Builds the work lists of steps with n_sub subsets (a set-up call; steps over all
        views are prepared at creation)."""
        _check(load().fb_batch_prepare(self._h, int(n_sub)))

    def close(self):
        if getattr(self, "_h", None):
            load().fb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _events(events):
    handles = []
    for ev in events:
        if ev is None:
            handles.append(None)
            continue
        if not ev.cuda_event:  # torch creates the event on its first record
            ev.record()
        handles.append(ev.cuda_event)
    return (ctypes.c_void_p * 6)(*handles)


def batch_args(batch: Batch, stage: int, b, y_prev, x_prev, x_out, y_out, eta: torch.Tensor, a_t: float,
               n_sub: int = 1, subset: int = 0, sigma: float = 1.0, alpha: float = 1.0, lam: float = 0.01,
               tau: float = 0.125, tv_iters: int = 5, history: torch.Tensor | None = None, events=None) -> BatchArgs:
    """Arguments of one pnp_step_batched on arenas (b: sino_size floats, images:
    image_size floats, eta: one step size per slice)."""
    ni, ns = batch.image_size, batch.sino_size
    a = BatchArgs(stage, n_sub, subset, sigma, alpha, a_t, lam, tau, tv_iters,
                  _ptr(eta, numel=len(batch), name="eta"), _ptr(b, numel=ns, name="b"),
                  _ptr(y_prev, numel=ni, name="y_prev"), _ptr(x_prev, numel=ni, name="x_prev"),
                  _ptr(x_out, numel=ni, name="x_out"), _ptr(y_out, numel=ni, name="y_out"),
                  _ptr(history, numel=ni, name="history"), -1, 0)
    if events is not None:
        if len(events) != 6:
            raise ValueError("events: need six entries (fp, bp, TV; begin and end)")
        a.events = _events(events)
    return a


def pnp_step_batched(batch: Batch, args: BatchArgs, stream=None) -> None:
    _check(load().pnp_step_batched(batch.handle, ctypes.byref(args), _stream(stream)))


class BatchGraph(Graph):
    """A schedule of batched steps captured into one HIP graph (fb_batch_graph_create)."""

    def __init__(self, batch: Batch, steps):
        arr = (BatchArgs * len(steps))(*steps)
        h = ctypes.c_void_p()
        _check(load().fb_batch_graph_create(batch.handle, arr, len(steps), ctypes.byref(h)))
        self._h = h
        self._plan = batch


def tv_prox_vjp(z: torch.Tensor, xbar: torch.Tensor, zbar: torch.Tensor, lam: float, n_iter: int = 5,
                tau: float = 0.125, alpha: float = 1.0, ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """zbar = J^T xbar of z -> (1 - alpha) z + alpha tv_prox(z)."""
    ny, nx = z.shape
    need = int(load().fb_tv_vjp_workspace_bytes(nx, ny, n_iter))
    if ws is None and need > 0:
        ws = torch.empty((need + 3) // 4, dtype=torch.float32, device=z.device)
    ws_ptr, ws_bytes = (ws.data_ptr(), ws.numel() * 4) if ws is not None else (None, 0)
    _check(load().tv_prox_vjp(_ptr(z, name="z"), _ptr(xbar, numel=nx * ny, name="xbar"),
                              _ptr(zbar, numel=nx * ny, name="zbar"), nx, ny, float(lam), int(n_iter), float(tau),
                              float(alpha), ctypes.c_void_p(ws_ptr), ws_bytes, _stream(stream)))
    return zbar


def pnp_vjp_workspace(plan: Plan, tv_iters: int = 5, device="cuda") -> torch.Tensor:
    need = int(load().fb_pnp_vjp_workspace_bytes(plan.handle, tv_iters))
    return torch.empty((need + 3) // 4, dtype=torch.float32, device=device)


def pnp_step_vjp(plan: Plan, args: PnpArgs, xbar: torch.Tensor, ybar: torch.Tensor | None,
                 xbar_prev: torch.Tensor | None, ybar_prev: torch.Tensor, eta_bar: torch.Tensor,
                 ws: torch.Tensor, combine: bool = False, stream=None) -> None:
    """Reverse mode of one pnp_step (see include/fbpnp.h)."""
    npix = plan.geom.nx * plan.geom.ny
    _check(load().pnp_step_vjp(plan.handle, ctypes.byref(args), _ptr(xbar, numel=npix, name="xbar"),
                               _ptr(ybar, numel=npix, name="ybar"), _ptr(xbar_prev, numel=npix, name="xbar_prev"),
                               _ptr(ybar_prev, numel=npix, name="ybar_prev"), _ptr(eta_bar, name="eta_bar"),
                               int(combine), ctypes.c_void_p(ws.data_ptr()), ws.numel() * 4, _stream(stream)))


def power_lipschitz(plan: Plan, stage: int, n_iter: int = 100, stream=None) -> float:
    out = ctypes.c_double()
    _check(load().fb_power_lipschitz(plan.handle, stage, n_iter, ctypes.byref(out), _stream(stream)))
    return out.value

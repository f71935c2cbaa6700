"""FP64 CPU oracle for sketched plug-and-play fan-beam CT (arXiv:2203.07308).

TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package. It wraps ``oracle.c`` through ctypes on NumPy
float64 arrays and shares no code with the GPU library.

Each function cites the passage of the paper it implements; the geometric and
algorithmic readings where the paper is silent are stated in ``oracle.c``.
Parity status: every function here is pinned by a ``-m "not gpu"`` test against an
independent fact (closed forms, brute force, symmetry, LAPACK), listed in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
             _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
        ("n_views", ctypes.c_int32), ("n_bins", ctypes.c_int32),
        ("sod_mm", ctypes.c_double), ("sdd_mm", ctypes.c_double),
        ("det_pitch_mm", ctypes.c_double), ("det_offset_mm", ctypes.c_double),
        ("angle0_rad", ctypes.c_double), ("angle_step_rad", ctypes.c_double),
    ]


@dataclass(frozen=True)
class Geometry:
    """Fan-beam geometry on an nx x ny grid of pixel_mm pixels (flat detector)."""
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

    def c(self) -> _Geom:
        step = self.angle_step_rad if self.angle_step_rad is not None else 2 * np.pi / self.n_views
        return _Geom(self.nx, self.ny, self.pixel_mm, self.n_views, self.n_bins, self.sod_mm,
                     self.sdd_mm, self.det_pitch_mm, self.det_offset_mm, self.angle0_rad, step)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, gp = ctypes.c_double, ctypes.c_int, P(_Geom)
        dp, ip = P(ctypes.c_double), P(ctypes.c_int32)
        lib.orc_ray_geometry.argtypes = [gp, i32, i32, dp]
        lib.orc_fp.argtypes = [gp, i32, dp, dp, ip, i32]
        lib.orc_bp.argtypes = [gp, i32, dp, dp, ip, i32, d]
        lib.orc_count_samples.argtypes = [gp, i32, ip, i32]
        lib.orc_count_samples.restype = ctypes.c_long
        lib.orc_dense_matrix.argtypes = [gp, i32, ip, i32, dp]
        lib.orc_down.argtypes = [dp, i32, i32, i32, dp]
        lib.orc_up.argtypes = [dp, i32, i32, i32, dp]
        lib.orc_grad.argtypes = [gp, i32, dp, dp, ip, i32, d, dp]
        lib.orc_tv_prox.argtypes = [dp, i32, i32, d, i32, d, dp]
        lib.orc_pnp_run.argtypes = [gp, i32, ip, ip, ip, ip, dp, dp, dp, d, d, i32, d, dp, dp, dp, dp]
        lib.orc_grad_vr.argtypes = [gp, i32, dp, dp, ip, i32, d, dp, dp]
        lib.orc_bicubic_matrix.argtypes = [i32, i32, dp]
        lib.orc_sketch_down.argtypes = [i32, dp, i32, i32, i32, dp]
        lib.orc_sketch_up.argtypes = [i32, dp, i32, i32, i32, dp]
        lib.orc_grad_k.argtypes = [gp, i32, i32, dp, dp, ip, i32, d, dp]
        lib.orc_pnp_run_k.argtypes = [gp, i32, i32, ip, ip, ip, ip, dp, dp, dp, d, d, i32, d, dp, dp, dp, dp]
        lib.orc_power_lipschitz_k.argtypes = [gp, i32, i32, i32]
        lib.orc_power_lipschitz_k.restype = d
        lib.orc_pnp_run_vr.argtypes = [gp, i32, ip, ip, ip, ip, dp, ip, dp, dp, d, d, i32, d, dp, dp, dp, dp]
        lib.orc_power_lipschitz.argtypes = [gp, i32, i32]
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_power_lipschitz.restype = d
        lib.orc_psnr.argtypes = [dp, dp, ctypes.c_size_t]
        lib.orc_psnr.restype = d
        lib.orc_tv_relax_vjp.argtypes = [dp, dp, i32, i32, d, i32, d, d, dp]
        lib.orc_pnp_vjp.argtypes = [gp, i32, ip, ip, ip, ip, dp, dp, dp, d, d, i32, d, dp, dp, dp, dp, dp]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _views(views):
    if views is None:
        return None, None
    v = np.ascontiguousarray(views, dtype=np.int32)
    return v, v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def ray_geometry(g: Geometry, view: int, bin_: int) -> np.ndarray:
    """(S_x, S_y, d_x, d_y) of one ray: source and direction towards the bin centre."""
    out = np.zeros(4)
    _load().orc_ray_geometry(ctypes.byref(g.c()), view, bin_, _dp(out))
    return out


def fp(g: Geometry, x, f: int = 1, views=None) -> np.ndarray:
    """Forward projection M A_s x on the grid coarsened by f (Sec. 1 Eq. (1); Sec. 2.1 Eq. (4)).

    x: (ny/f, nx/f). Returns (n_sel, n_bins)."""
    x = _f64(x)
    assert x.shape == (g.ny // f, g.nx // f)
    v, vp = _views(views)
    n_sel = g.n_views if v is None else len(v)
    y = np.zeros((n_sel, g.n_bins))
    _load().orc_fp(ctypes.byref(g.c()), f, _dp(x), _dp(y), vp, n_sel)
    return y


def bp(g: Geometry, y, f: int = 1, views=None, scale: float = 1.0) -> np.ndarray:
    """Backprojection scale * (M A_s)^T y, the exact transpose of ``fp``."""
    y = _f64(y)
    v, vp = _views(views)
    n_sel = g.n_views if v is None else len(v)
    assert y.shape == (n_sel, g.n_bins)
    x = np.zeros((g.ny // f, g.nx // f))
    _load().orc_bp(ctypes.byref(g.c()), f, _dp(y), _dp(x), vp, n_sel, scale)
    return x


def count_samples(g: Geometry, f: int = 1, views=None) -> int:
    """In-grid Joseph interpolation samples of one projection (projector work)."""
    v, vp = _views(views)
    n_sel = g.n_views if v is None else len(v)
    return int(_load().orc_count_samples(ctypes.byref(g.c()), f, vp, n_sel))


def dense_matrix(g: Geometry, f: int = 1, views=None) -> np.ndarray:
    """Dense M A_s for tiny grids, column m = projection of the m-th unit image."""
    v, vp = _views(views)
    n_sel = g.n_views if v is None else len(v)
    d = (g.nx // f) * (g.ny // f)
    A = np.zeros((n_sel * g.n_bins, d))
    _load().orc_dense_matrix(ctypes.byref(g.c()), f, vp, n_sel, _dp(A))
    return A


def down(x, f: int) -> np.ndarray:
    """Sketch S = D_f, f x f average pooling (Sec. 2.1, Eq. (4))."""
    x = _f64(x)
    ny, nx = x.shape
    v = np.zeros((ny // f, nx // f))
    _load().orc_down(_dp(x), nx, ny, f, _dp(v))
    return v


def up(v, f: int) -> np.ndarray:
    """Upsampler U = D_f^T (Sec. 2.1, Eq. (6))."""
    v = _f64(v)
    nys, nxs = v.shape
    x = np.zeros((nys * f, nxs * f))
    _load().orc_up(_dp(v), nxs, nys, f, _dp(x))
    return x


SKETCHES = {"pool": 0, "bicubic": 1}


def bicubic_matrix(n: int, f: int) -> np.ndarray:
    """The 1-D bicubic sketch (n / f x n): Keys' cubic kernel (a = -1/2) stretched by f,
    half-sample reflection at the ends, rows normalised to 1 (Sec. 3, bicubic resizing)."""
    S = np.zeros((n // f, n))
    _load().orc_bicubic_matrix(n, f, _dp(S))
    return S


def sketch_down(x, f: int, sketch: str = "pool") -> np.ndarray:
    x = _f64(x)
    ny, nx = x.shape
    v = np.zeros((ny // f, nx // f))
    _load().orc_sketch_down(SKETCHES[sketch], _dp(x), nx, ny, f, _dp(v))
    return v


def sketch_up(v, f: int, sketch: str = "pool") -> np.ndarray:
    """U = S^T (for pooling D^T: replicate and divide by f^2)."""
    v = _f64(v)
    nys, nxs = v.shape
    x = np.zeros((nys * f, nxs * f))
    _load().orc_sketch_up(SKETCHES[sketch], _dp(v), nxs, nys, f, _dp(x))
    return x


def grad(g: Geometry, y, b, f: int = 1, views=None, sigma: float = 1.0, sketch: str = "pool") -> np.ndarray:
    """Sketched minibatch gradient sigma * U (M A_s)^T (M A_s S y - M b) (Sec. 2.1, Eqs. (6)-(7))."""
    y, b = _f64(y), _f64(b)
    assert y.shape == (g.ny, g.nx) and b.shape == (g.n_views, g.n_bins)
    v, vp = _views(views)
    n_sel = g.n_views if v is None else len(v)
    out = np.zeros((g.ny, g.nx))
    _load().orc_grad_k(ctypes.byref(g.c()), SKETCHES[sketch], f, _dp(y), _dp(b), vp, n_sel, sigma, _dp(out))
    return out


def grad_vr(g: Geometry, y, b, y_snap, f: int = 1, views=None, sigma: float = 1.0) -> np.ndarray:
    """Variance-reduced (SVRG) estimator over view subsets: grad(y; M) - grad(y_snap; M)
    + grad(y_snap; all views), the minibatch terms scaled by sigma."""
    y, b, ys = _f64(y), _f64(b), _f64(y_snap)
    assert y.shape == (g.ny, g.nx) and ys.shape == y.shape and b.shape == (g.n_views, g.n_bins)
    v, vp = _views(views)
    n_sel = g.n_views if v is None else len(v)
    out = np.zeros((g.ny, g.nx))
    _load().orc_grad_vr(ctypes.byref(g.c()), f, _dp(y), _dp(b), vp, n_sel, sigma, _dp(ys), _dp(out))
    return out


def tv_prox(z, lam: float, n_iter: int = 5, tau: float = 0.125) -> np.ndarray:
    """Denoiser D: n_iter Chambolle dual-projection steps for isotropic TV (Sec. 2.1, after Eq. (5))."""
    z = _f64(z)
    ny, nx = z.shape
    x = np.zeros_like(z)
    _load().orc_tv_prox(_dp(z), nx, ny, lam, n_iter, tau, _dp(x))
    return x


def pnp_run(g: Geometry, b, schedule, eta, a, alpha: float = 1.0, lam: float = 0.01,
            tv_iters: int = 5, tau: float = 0.125, x0=None, history: bool = False, vr=None, sketch: str = "pool"):
    """PnP-MS2G (Sec. 2.1, Algorithm 1) for T iterations.

    schedule: list of (f, views or None, sigma) per iteration; eta, a: length-T arrays.
    vr (optional): gradient mode per iteration, 0 minibatch, 1 snapshot (full-view
    gradient, remembered), 2 variance-reduced against the last snapshot of the same f.
    Returns x_T, or (x_T, history[T, ny, nx]) when history is True."""
    T = len(schedule)
    b = _f64(b)
    factor = np.array([s[0] for s in schedule], dtype=np.int32)
    sigma = _f64([s[2] for s in schedule])
    eta, a = _f64(eta), _f64(a)
    assert eta.shape == (T,) and a.shape == (T,)
    lists = [np.arange(g.n_views, dtype=np.int32) if s[1] is None else np.asarray(s[1], np.int32)
             for s in schedule]
    n_sel = np.array([len(l) for l in lists], dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(n_sel)[:-1]]).astype(np.int32)
    views = np.ascontiguousarray(np.concatenate(lists), dtype=np.int32)
    x0 = np.zeros((g.ny, g.nx)) if x0 is None else _f64(x0)
    xo = np.zeros((g.ny, g.nx))
    hist = np.zeros((T, g.ny, g.nx)) if history else None
    ip = lambda arr: arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    if vr is None:
        _load().orc_pnp_run_k(ctypes.byref(g.c()), SKETCHES[sketch], T, ip(factor), ip(views), ip(off), ip(n_sel),
                              _dp(sigma), _dp(eta), _dp(a), alpha, lam, tv_iters, tau, _dp(b), _dp(x0), _dp(xo),
                              _dp(hist) if history else None)
    else:
        assert sketch == "pool", "variance reduction is defined with the pooling sketch"
        mode = np.ascontiguousarray(vr, dtype=np.int32)
        assert mode.shape == (T,) and set(mode.tolist()) <= {0, 1, 2}
        snap_f = None
        for t in range(T):  # a variance-reduced step needs a snapshot of its own stage
            if mode[t] == 1:
                snap_f = factor[t]
            elif mode[t] == 2 and snap_f != factor[t]:
                raise ValueError(f"iteration {t}: variance-reduced step without a snapshot at f = {factor[t]}")
        _load().orc_pnp_run_vr(ctypes.byref(g.c()), T, ip(factor), ip(views), ip(off), ip(n_sel), _dp(sigma),
                               ip(mode), _dp(eta), _dp(a), alpha, lam, tv_iters, tau, _dp(b), _dp(x0), _dp(xo),
                               _dp(hist) if history else None)
    return (xo, hist) if history else xo


def tv_relax_vjp(z, xbar, lam: float, n_iter: int = 5, tau: float = 0.125, alpha: float = 1.0) -> np.ndarray:
    """Vector-Jacobian product of z -> (1 - alpha) z + alpha TV_prox(z) (reverse mode of
    the relaxed denoiser step of Algorithm 1)."""
    z, xbar = _f64(z), _f64(xbar)
    ny, nx = z.shape
    out = np.zeros_like(z)
    _load().orc_tv_relax_vjp(_dp(z), _dp(xbar), nx, ny, lam, n_iter, tau, alpha, _dp(out))
    return out


def _schedule_arrays(g: Geometry, schedule):
    factor = np.array([s[0] for s in schedule], dtype=np.int32)
    sigma = _f64([s[2] for s in schedule])
    lists = [np.arange(g.n_views, dtype=np.int32) if s[1] is None else np.asarray(s[1], np.int32)
             for s in schedule]
    n_sel = np.array([len(l) for l in lists], dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(n_sel)[:-1]]).astype(np.int32)
    views = np.ascontiguousarray(np.concatenate(lists), dtype=np.int32)
    return factor, sigma, views, off, n_sel


def pnp_vjp(g: Geometry, b, schedule, eta, a, xT_bar, alpha: float = 1.0, lam: float = 0.01,
            tv_iters: int = 5, tau: float = 0.125, x0=None):
    """Reverse mode of pnp_run: given dL/dx_T, returns (dL/dx_0, dL/deta_t for t = 1..T)."""
    T = len(schedule)
    factor, sigma, views, off, n_sel = _schedule_arrays(g, schedule)
    eta, a, b = _f64(eta), _f64(a), _f64(b)
    x0 = np.zeros((g.ny, g.nx)) if x0 is None else _f64(x0)
    xT_bar = _f64(xT_bar)
    x0_bar = np.zeros((g.ny, g.nx))
    eta_bar = np.zeros(T)
    ip = lambda arr: arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    _load().orc_pnp_vjp(ctypes.byref(g.c()), T, ip(factor), ip(views), ip(off), ip(n_sel), _dp(sigma), _dp(eta),
                        _dp(a), alpha, lam, tv_iters, tau, _dp(b), _dp(x0), _dp(xT_bar), _dp(x0_bar),
                        _dp(eta_bar))
    return x0_bar, eta_bar


def power_lipschitz(g: Geometry, f: int = 1, n_iter: int = 100, sketch: str = "pool") -> float:
    """L = ||A_s S||_2^2 by power iteration, for the step eta = 1/L (Sec. 3)."""
    return float(_load().orc_power_lipschitz_k(ctypes.byref(g.c()), SKETCHES[sketch], f, n_iter))


def set_threads(n: int) -> int:
    """Number of OpenMP threads for later oracle calls (n <= 0 leaves it); returns the
    number in force before (timing support only)."""
    return int(_load().orc_set_threads(int(n)))


def psnr(x, ref) -> float:
    """PSNR with peak max(ref) - min(ref) and MSE over all pixels."""
    x, ref = _f64(x).ravel(), _f64(ref).ravel()
    return float(_load().orc_psnr(_dp(x), _dp(ref), x.size))

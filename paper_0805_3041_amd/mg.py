"""ctypes binding of libmg.so (include/mg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  torch is used for device memory (tensors' data pointers) and streams.
Loading fails loudly if the library has not been built; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch  # loaded first so that the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmg.so")

MG_OK, MG_NOT_CONVERGED, MG_DIVERGED = 0, 1, 2
MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_EUNSUPPORTED = -1, -2, -3, -4
MG_COEF_CONST5, MG_COEF_CELL9 = 0, 1
MG_CYCLE_F, MG_CYCLE_V, MG_CYCLE_W = 0, 1, 2
MG_SMOOTH_JACOBI, MG_SMOOTH_RBGS, MG_SMOOTH_GS4C = 0, 1, 2
MG_SMOOTH_TRI_X, MG_SMOOTH_TRI_Y, MG_SMOOTH_ADI = 3, 4, 5
MG_SMOOTH_GSTRI_X, MG_SMOOTH_GSTRI_Y, MG_SMOOTH_GSADI = 6, 7, 8
MG_PREC_FP64, MG_PREC_MIXED = 0, 1
MG_TILES_FUSED, MG_TILES_PER_OP, MG_TILES_NARROW, MG_TILES_WIDE = 0, 1, 2, 3
MG_COARSE_DEFAULT, MG_COARSE_GALERKIN = 0, 1

SMOOTHERS = {"jacobi": MG_SMOOTH_JACOBI, "rbgs": MG_SMOOTH_RBGS, "gs4c": MG_SMOOTH_GS4C,
             "tri_x": MG_SMOOTH_TRI_X, "tri_y": MG_SMOOTH_TRI_Y, "adi": MG_SMOOTH_ADI,
             "gstri_x": MG_SMOOTH_GSTRI_X, "gstri_y": MG_SMOOTH_GSTRI_Y, "gsadi": MG_SMOOTH_GSADI}
CYCLES = {"F": MG_CYCLE_F, "V": MG_CYCLE_V, "W": MG_CYCLE_W}
PRECISIONS = {"fp64": MG_PREC_FP64, "mixed": MG_PREC_MIXED}

EXPORTED = (
    "mg_setup", "mg_solve", "mg_residual", "mg_coeff_grad", "mg_setup_batched", "mg_solve_batched",
    "mg_destroy", "mg_status_string", "mg_last_error", "mg_level_shape", "mg_num_levels", "mg_profile_pass",
    "mg_pass_info", "mg_start_nested", "mg_update_coeffs", "mg_residual_noalloc", "mg_batch_schedule",
)


class mg_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("periodic_x", ctypes.c_int32),
                ("periodic_y", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("xs", ctypes.POINTER(ctypes.c_double)), ("ys", ctypes.POINTER(ctypes.c_double))]


class mg_coeffs(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("eps_x", ctypes.c_double), ("eps_y", ctypes.c_double),
                ("kx", ctypes.c_void_p), ("ky", ctypes.c_void_p), ("kx_1d_along_x", ctypes.c_int32)]


class mg_options(ctypes.Structure):
    _fields_ = [("cycle", ctypes.c_int32), ("smoother", ctypes.c_int32), ("nu_pre", ctypes.c_int32),
                ("nu_post", ctypes.c_int32), ("omega", ctypes.c_double), ("precision", ctypes.c_int32),
                ("coarse_cta_nodes", ctypes.c_int32), ("tile_mode", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("stream", ctypes.c_void_p), ("sor", ctypes.c_double),
                ("inner_cycles", ctypes.c_int32), ("coarse_op", ctypes.c_int32), ("adaptive_omega", ctypes.c_int32),
                ("tune", ctypes.c_int32)]


class mg_info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("res0", ctypes.c_double), ("res", ctypes.c_double),
                ("rel_res", ctypes.c_double), ("rho_last", ctypes.c_double), ("rho_mean", ctypes.c_double),
                ("seconds", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("status", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmg.so (once).  Raises if it is missing: build it with
    ``python -m paper_0805_3041_amd.build``."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing; build it with `python -m paper_0805_3041_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.mg_setup.argtypes = [P(mg_grid), P(mg_coeffs), ctypes.c_int32, P(mg_options), P(ctypes.c_void_p)]
    lib.mg_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                             P(mg_info)]
    lib.mg_residual.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                P(ctypes.c_double)]
    lib.mg_coeff_grad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.mg_setup_batched.argtypes = [P(mg_grid), P(mg_coeffs), ctypes.c_int32, ctypes.c_int32, P(mg_options),
                                     P(ctypes.c_void_p)]
    lib.mg_solve_batched.argtypes = [ctypes.c_void_p, P(ctypes.c_void_p), P(ctypes.c_void_p), ctypes.c_double,
                                     ctypes.c_int32, P(mg_info)]
    lib.mg_destroy.argtypes = [ctypes.c_void_p]
    lib.mg_status_string.argtypes = [ctypes.c_int]
    lib.mg_status_string.restype = ctypes.c_char_p
    lib.mg_last_error.argtypes = [ctypes.c_void_p]
    lib.mg_last_error.restype = ctypes.c_char_p
    lib.mg_level_shape.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.mg_num_levels.argtypes = [ctypes.c_void_p]
    lib.mg_profile_pass.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, P(ctypes.c_double)]
    lib.mg_pass_info.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32)]
    lib.mg_start_nested.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.mg_update_coeffs.argtypes = [ctypes.c_void_p, P(mg_coeffs)]
    lib.mg_batch_schedule.argtypes = [ctypes.c_void_p, P(ctypes.c_int32)]
    lib.mg_residual_noalloc.argtypes = [P(mg_grid), P(mg_coeffs), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        P(ctypes.c_double), ctypes.c_void_p]
    for name in ("mg_setup", "mg_solve", "mg_residual", "mg_coeff_grad", "mg_setup_batched", "mg_solve_batched",
                 "mg_destroy", "mg_level_shape", "mg_profile_pass", "mg_pass_info", "mg_start_nested",
                 "mg_update_coeffs", "mg_residual_noalloc", "mg_batch_schedule"):
        getattr(lib, name).restype = ctypes.c_int
    lib.mg_num_levels.restype = ctypes.c_int32
    _lib = lib
    return lib


class MGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


def status_string(s: int) -> str:
    return load_library().mg_status_string(int(s)).decode()


def last_error(h=None) -> str:
    return load_library().mg_last_error(h).decode()


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("arrays must be device (cuda) tensors")
    return ctypes.c_void_p(t.data_ptr())


def _check_f64(t: torch.Tensor, shape, name):
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape {tuple(shape)}")


def _stream_ptr(stream):
    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(None)
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class SolveInfo:
    status: int
    cycles: int
    res0: float
    res: float
    rel_res: float
    rho_last: float
    rho_mean: float
    seconds: float
    history: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def converged(self) -> bool:
        return self.status == MG_OK


def mg_setup(grid: mg_grid, coeffs: mg_coeffs, levels: int, opts: mg_options):
    lib = load_library()
    h = ctypes.c_void_p()
    s = lib.mg_setup(ctypes.byref(grid), ctypes.byref(coeffs), int(levels), ctypes.byref(opts), ctypes.byref(h))
    if s != MG_OK:
        raise MGError(s, last_error(None))
    return h


def mg_solve(h, rhs: torch.Tensor, x: torch.Tensor, tol: float, max_cycles: int, history: bool = True) -> SolveInfo:
    lib = load_library()
    info = mg_info()
    hist = None
    if history:
        hist = np.zeros(max_cycles + 1, dtype=np.float64)
        info.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s = lib.mg_solve(h, _ptr(rhs), _ptr(x), float(tol), int(max_cycles), ctypes.byref(info))
    if s < 0:
        raise MGError(s, last_error(h))
    return SolveInfo(info.status, info.cycles, info.res0, info.res, info.rel_res, info.rho_last, info.rho_mean, info.seconds,
                     hist[: info.cycles + 1].copy() if hist is not None else np.zeros(0))


def mg_residual(h, rhs: torch.Tensor, x: torch.Tensor, r: torch.Tensor | None = None) -> float:
    lib = load_library()
    nrm = ctypes.c_double()
    s = lib.mg_residual(h, _ptr(rhs), _ptr(x), _ptr(r), ctypes.byref(nrm))
    if s != MG_OK:
        raise MGError(s, last_error(h))
    return nrm.value


def mg_residual_noalloc(grid: mg_grid, coeffs: mg_coeffs, rhs: torch.Tensor, x: torch.Tensor,
                        r: torch.Tensor | None = None, stream=None) -> float:
    """r = rhs - A x and ||r||_2 without a handle and without device allocation
    (the library's static scratch); arrays as for mg_residual."""
    lib = load_library()
    nrm = ctypes.c_double()
    s = lib.mg_residual_noalloc(ctypes.byref(grid), ctypes.byref(coeffs), _ptr(rhs), _ptr(x), _ptr(r),
                                ctypes.byref(nrm), _stream_ptr(stream))
    if s != MG_OK:
        raise MGError(s, last_error(None))
    return nrm.value


def mg_coeff_grad(h, u: torch.Tensor, lam: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    lib = load_library()
    s = lib.mg_coeff_grad(h, _ptr(u), _ptr(lam), _ptr(out))
    if s != MG_OK:
        raise MGError(s, last_error(h))
    return out


def mg_update_coeffs(h, coeffs: mg_coeffs) -> None:
    lib = load_library()
    s = lib.mg_update_coeffs(h, ctypes.byref(coeffs))
    if s != MG_OK:
        raise MGError(s, last_error(h))


def mg_start_nested(h, rhs: torch.Tensor, x: torch.Tensor) -> None:
    lib = load_library()
    s = lib.mg_start_nested(h, _ptr(rhs), _ptr(x))
    if s != MG_OK:
        raise MGError(s, last_error(h))


def mg_profile_pass(h, rhs: torch.Tensor, x: torch.Tensor, level: int, which: int, reps: int) -> float:
    lib = load_library()
    us = ctypes.c_double()
    s = lib.mg_profile_pass(h, _ptr(rhs), _ptr(x), int(level), int(which), int(reps), ctypes.byref(us))
    if s != MG_OK:
        raise MGError(s, last_error(h))
    return us.value


PASS_INFO_KEYS = ("wide", "tx", "ty", "halo", "workgroups", "colours", "stencil", "bands_1d", "forms_residual",
                  "halo_y")


def mg_pass_info(h, level: int, which: int) -> dict:
    lib = load_library()
    out = (ctypes.c_int32 * 10)()
    s = lib.mg_pass_info(h, int(level), int(which), out)
    if s != MG_OK:
        raise MGError(s, last_error(h))
    return dict(zip(PASS_INFO_KEYS, list(out)))


def mg_setup_batched(grids, coeffs, opts: mg_options, levels: int = 0):
    lib = load_library()
    n = len(grids)
    ga = (mg_grid * n)(*grids)
    ca = (mg_coeffs * n)(*coeffs)
    h = ctypes.c_void_p()
    s = lib.mg_setup_batched(ga, ca, n, int(levels), ctypes.byref(opts), ctypes.byref(h))
    if s != MG_OK:
        raise MGError(s, last_error(None))
    return h


def mg_solve_batched(h, rhs: list, x: list, tol: float, max_cycles: int, history: bool = False):
    lib = load_library()
    n = len(rhs)
    ra = (ctypes.c_void_p * n)(*[t.data_ptr() for t in rhs])
    xa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in x])
    infos = (mg_info * n)()
    hists = []
    if history:
        for k in range(n):
            hh = np.zeros(max_cycles + 1, dtype=np.float64)
            infos[k].history = hh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            hists.append(hh)
    s = lib.mg_solve_batched(h, ra, xa, float(tol), int(max_cycles), infos)
    if s < 0:
        raise MGError(s, last_error(h))
    out = []
    for k in range(n):
        i = infos[k]
        out.append(SolveInfo(i.status, i.cycles, i.res0, i.res, i.rel_res, i.rho_last, i.rho_mean, i.seconds,
                             hists[k][: i.cycles + 1].copy() if history else np.zeros(0)))
    return s, out


def mg_batch_schedule(h) -> dict:
    out = (ctypes.c_int32 * 4)()
    s = load_library().mg_batch_schedule(h, out)
    if s != MG_OK:
        raise MGError(s, last_error(h))
    return {"merged": out[0], "groups_merged": out[1], "standalone": out[2], "launches_per_cycle": out[3]}


def mg_destroy(h) -> None:
    if h is not None and h.value:
        load_library().mg_destroy(h)


def mg_num_levels(h) -> int:
    return int(load_library().mg_num_levels(h))


def mg_level_shape(h, l: int):
    nx, ny = ctypes.c_int32(), ctypes.c_int32()
    s = load_library().mg_level_shape(h, int(l), ctypes.byref(nx), ctypes.byref(ny))
    if s != MG_OK:
        raise MGError(s, last_error(h))
    return nx.value, ny.value


TILE_MODES = {"fused": MG_TILES_FUSED, "per_op": MG_TILES_PER_OP, "narrow": MG_TILES_NARROW,
              "wide": MG_TILES_WIDE}


COARSE_OPS = {"default": MG_COARSE_DEFAULT, "galerkin": MG_COARSE_GALERKIN}
MG_TUNE_AUTO, MG_TUNE_OFF, MG_TUNE_REFRESH = 0, 1, 2
TUNE_MODES = {"auto": MG_TUNE_AUTO, "off": MG_TUNE_OFF, "refresh": MG_TUNE_REFRESH}


def make_options(cycle="F", smoother="rbgs", nu_pre=2, nu_post=2, omega=0.8, precision="fp64",
                 coarse_cta_nodes=0, tile_mode="fused", tile_x=0, tile_y=0, stream=None, sor=1.0,
                 inner_cycles=1, coarse_op="default", adaptive_omega=False, tune="auto") -> mg_options:
    return mg_options(CYCLES[cycle], SMOOTHERS[smoother], int(nu_pre), int(nu_post), float(omega),
                      PRECISIONS[precision], int(coarse_cta_nodes), TILE_MODES[tile_mode], int(tile_x), int(tile_y),
                      _stream_ptr(stream), float(sor), int(inner_cycles), COARSE_OPS[coarse_op],
                      1 if adaptive_omega else 0, TUNE_MODES[tune])


class Solver:
    """Owns one handle.  Grid arrays are float64 device tensors [ny][nx]."""

    def __init__(self, nx: int, ny: int, *, periodic_y: bool = False, lx: float = 1.0, ly: float = 1.0,
                 eps_x: float = 1.0, eps_y: float = 1.0, kx: torch.Tensor | None = None,
                 ky: torch.Tensor | None = None, kx_1d_along_x: bool = False, levels: int = 0,
                 xs=None, ys=None, **opt):
        """xs, ys: node coordinates of a refined (graded) grid (host arrays of
        nx, ny values; None = equidistant)."""
        self.nx, self.ny, self.periodic_y = nx, ny, periodic_y
        self.grid = mg_grid(nx, ny, 0, 1 if periodic_y else 0, lx, ly)
        self._coords = tuple(None if c is None else np.ascontiguousarray(c, dtype=np.float64) for c in (xs, ys))
        for name, c in zip(("xs", "ys"), self._coords):
            if c is not None:
                setattr(self.grid, name, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if kx is None:
            self.coeffs = mg_coeffs(MG_COEF_CONST5, eps_x, eps_y, None, None, 0)
            self._keep = ()
        else:
            self.coeffs = self._cell_coeffs(kx, ky, kx_1d_along_x)
        self.opts = make_options(**opt)
        self.h = mg_setup(self.grid, self.coeffs, levels, self.opts)

    def _cell_coeffs(self, kx: torch.Tensor, ky: torch.Tensor | None, oned: bool) -> mg_coeffs:
        same = ky is None or ky is kx
        kx = kx.contiguous().to(torch.float64)
        ky = kx if same else ky.contiguous().to(torch.float64)
        self._keep = (kx, ky)
        return mg_coeffs(MG_COEF_CELL9, 0.0, 0.0, _ptr(kx), _ptr(ky), 1 if oned else 0)

    def update_coefficients(self, kx: torch.Tensor, ky: torch.Tensor | None = None) -> None:
        """Rebuild every level's operator for new cell coefficients in the
        handle's buffers (mg_update_coeffs); same layout as at construction,
        and ky omitted (or kx itself) if it was omitted there."""
        self.coeffs = self._cell_coeffs(kx, ky, bool(self.coeffs.kx_1d_along_x))
        mg_update_coeffs(self.h, self.coeffs)

    def level_shape(self, level: int):
        """(nx, ny) stored shape of a level."""
        return mg_level_shape(self.h, level)

    @property
    def nlevels(self) -> int:
        return mg_num_levels(self.h)

    def solve(self, rhs: torch.Tensor, x: torch.Tensor, tol: float = 1e-10, max_cycles: int = 100,
              history: bool = True) -> SolveInfo:
        _check_f64(rhs, (self.ny, self.nx), "rhs")
        _check_f64(x, (self.ny, self.nx), "x")
        return mg_solve(self.h, rhs, x, tol, max_cycles, history)

    def residual(self, rhs: torch.Tensor, x: torch.Tensor, r: torch.Tensor | None = None) -> float:
        _check_f64(rhs, (self.ny, self.nx), "rhs")
        _check_f64(x, (self.ny, self.nx), "x")
        if r is not None:
            _check_f64(r, (self.ny, self.nx), "r")
        return mg_residual(self.h, rhs, x, r)

    def coeff_grad(self, u: torch.Tensor, lam: torch.Tensor) -> torch.Tensor:
        ncy = self.ny if self.periodic_y else self.ny - 1
        out = torch.empty((ncy, self.nx - 1), dtype=torch.float64, device=u.device)
        return mg_coeff_grad(self.h, u, lam, out)

    def nested_start(self, rhs: torch.Tensor, x: torch.Tensor) -> None:
        """Overwrite x with the nested-iteration start vector for rhs (mg_start_nested)."""
        _check_f64(rhs, (self.ny, self.nx), "rhs")
        _check_f64(x, (self.ny, self.nx), "x")
        mg_start_nested(self.h, rhs, x)

    def profile_pass(self, rhs: torch.Tensor, x: torch.Tensor, level: int, which: int, reps: int = 50) -> float:
        """Average device time (us) of one fused pre-pass (which=0) or post-pass (1) on `level`, or with
        a line smoother (which=2) of its first line sweep."""
        return mg_profile_pass(self.h, rhs, x, level, which, reps)

    def pass_info(self, level: int, which: int) -> dict:
        """Launch shape of the fused pass (see mg_pass_info in include/mg.h)."""
        return mg_pass_info(self.h, level, which)

    def pass_kernel_name(self, level: int, which: int) -> str:
        """Symbol (as profilers print it) of the kernel that runs the fused pass."""
        i = self.pass_info(level, which)
        t = "float" if self.opts.precision == MG_PREC_MIXED else "double"
        base = ("k_pre" if which == 0 else "k_post") + ("_w" if i["wide"] else "")
        flag = "true" if level == 0 else "false"
        b1 = "true" if i["bands_1d"] else "false"
        return f"mg::{base}<{t}, {i['stencil']}, {flag}, {i['colours']}, {b1}>"

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedSolver:
    """Many independent 5-point problems solved by one sequence of launches
    (mg_setup_batched).  grids: list of (nx, ny) or (nx, ny, periodic_y);
    eps: list of eps_x (eps_y = 1) or (eps_x, eps_y)."""

    def __init__(self, grids, eps, levels: int = 0, **opt):
        gs, cs = [], []
        for g, e in zip(grids, eps):
            nx, ny = g[0], g[1]
            py = g[2] if len(g) > 2 else False
            gs.append(mg_grid(nx, ny, 0, 1 if py else 0, 1.0, 1.0))
            ex, ey = (e, 1.0) if not isinstance(e, (tuple, list)) else e
            cs.append(mg_coeffs(MG_COEF_CONST5, float(ex), float(ey), None, None, 0))
        self.shapes = [(g.ny, g.nx) for g in gs]
        self.opts = make_options(**opt)
        self.h = mg_setup_batched(gs, cs, self.opts, levels)

    def schedule(self) -> dict:
        """How the batch runs (mg_batch_schedule)."""
        return mg_batch_schedule(self.h)

    def solve(self, rhs: list, x: list, tol: float = 1e-10, max_cycles: int = 100, history: bool = False):
        """Returns (worst status, [SolveInfo per problem]); each info.status is
        MG_OK if that problem met the tolerance."""
        for r, xx, shp in zip(rhs, x, self.shapes):
            _check_f64(r, shp, "rhs")
            _check_f64(xx, shp, "x")
        return mg_solve_batched(self.h, rhs, x, tol, max_cycles, history)

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

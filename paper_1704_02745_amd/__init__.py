"""pbgpu: linear finite-difference Poisson-Boltzmann solver for MI355X.

Thin Python binding over the C ABI in include/pbgpu.h (libpbgpu.so, built
in-tree for gfx950). This module only marshals arguments: every step of the
computation runs in the HIP library. PyTorch provides device memory and the
current stream. If the library is missing, importing this package raises.

    sysm = pbgpu.setup(grid, xyz, radius, charge)        # section 2.7 setup
    x, info = pbgpu.solve(sysm, tol=1e-6, precision="f32")  # Jacobi PCG
    e = pbgpu.energy(grid, xyz, charge, x)                # kcal/mol
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbgpu.so")

PB_OK, PB_NOT_CONVERGED = 0, 1
PB_ERR_ARG, PB_ERR_BREAKDOWN, PB_ERR_NONFINITE = -1, -2, -3
PB_ERR_NOMEM, PB_ERR_HIP, PB_ERR_TIMEOUT = -4, -5, -6
STATUS_NAMES = {0: "PB_OK", 1: "PB_NOT_CONVERGED", -1: "PB_ERR_ARG", -2: "PB_ERR_BREAKDOWN",
                -3: "PB_ERR_NONFINITE", -4: "PB_ERR_NOMEM", -5: "PB_ERR_HIP", -6: "PB_ERR_TIMEOUT"}
PRECISIONS = {"f64": 0, "f32": 1, "f32_refine64": 2}
OPERATORS = {"stencil": 0, "dia": 1, "mg": 2}

# Every entry point declared in include/pbgpu.h.
EXPORTS = ("pb_version", "pb_last_error", "pb_setup_workspace_bytes", "pb_setup",
           "pb_solve_workspace_bytes", "pb_solve", "pb_autotune", "pb_set_tuning", "pb_tiling_candidates",
           "pb_get_tuning", "pb_set_coded_coefficients", "pb_get_coded_coefficients",
           "pb_batch_workspace_bytes", "pb_solve_batch", "pb_batch_set_zchunk", "pb_batch_get_zchunk",
           "pb_batch_autotune_workspace_bytes", "pb_batch_autotune", "pb_batch_graph_create", "pb_batch_graph_launch",
           "pb_batch_graph_results", "pb_batch_graph_is_cooperative", "pb_batch_graph_destroy",
           "pb_server_request_bytes", "pb_server_create", "pb_server_submit", "pb_server_step",
           "pb_server_stats", "pb_server_destroy", "pb_server_submit_atoms", "pb_server_request_bytes_atoms",
           "pb_energy_workspace_bytes", "pb_energy",
           "pb_solvation_workspace_bytes", "pb_solvation_energy",
           "pb_setup_ex_workspace_bytes", "pb_setup_ex", "pb_solve_noalloc", "pb_solve_noalloc_max_bytes",
           "pb_stream_copy", "pb_set_periodic_pass", "pb_get_periodic_pass")


class PBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("boundary", ctypes.c_int32), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3)]


class SetupOpts(ctypes.Structure):
    _fields_ = [("edge_model", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7)]


EDGE_MODELS = {"node": 0, "fraction": 1}


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("op", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("boundary", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("kernel_launches", ctypes.c_int32),
                ("relres_recur", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("seconds", ctypes.c_double), ("kernel_seconds", ctypes.c_double),
                ("coded_launches", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d.pop("reserved")
        return d


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("groups", ctypes.c_int32), ("zchunk", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("us_per_iter", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("scheme", ctypes.c_int32), ("streaming", ctypes.c_int32),
                ("segments", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("maxiter", ctypes.c_int32), ("h", ctypes.c_double), ("tol", ctypes.c_double),
                ("eps_x", ctypes.c_void_p), ("eps_y", ctypes.c_void_p), ("eps_z", ctypes.c_void_p),
                ("kappa2", ctypes.c_void_p), ("rhs", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("warm_start", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int32), ("active", ctypes.c_int32), ("arena_used", ctypes.c_size_t),
                ("arena_bytes", ctypes.c_size_t), ("launches", ctypes.c_int64),
                ("device_seconds", ctypes.c_double), ("coded_launches", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"pbgpu: {LIB_PATH} is not built; run python paper_1704_02745_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    G = ctypes.POINTER(Grid)
    lib.pb_version.restype = ctypes.c_char_p
    lib.pb_version.argtypes = []
    lib.pb_last_error.restype = ctypes.c_char_p
    lib.pb_last_error.argtypes = []
    lib.pb_setup_workspace_bytes.restype = sz
    lib.pb_setup_workspace_bytes.argtypes = [G, i64]
    lib.pb_setup.restype = ctypes.c_int
    lib.pb_setup.argtypes = [G, i64, vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pb_solve_workspace_bytes.restype = sz
    lib.pb_solve_workspace_bytes.argtypes = [i32, i32, i32, ctypes.POINTER(SolveOpts)]
    lib.pb_solve.restype = ctypes.c_int
    lib.pb_solve.argtypes = [i32, i32, i32, dbl, vp, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                             vp, sz, vp, ctypes.POINTER(Info)]
    lib.pb_autotune.restype = ctypes.c_int
    lib.pb_solve_noalloc.restype = ctypes.c_int
    lib.pb_solve_noalloc.argtypes = [i32, i32, i32, dbl, vp, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts), vp,
                                     ctypes.POINTER(Info)]
    lib.pb_stream_copy.restype = ctypes.c_int
    lib.pb_stream_copy.argtypes = [vp, vp, sz, i32, vp]
    lib.pb_solve_noalloc_max_bytes.restype = sz
    lib.pb_solve_noalloc_max_bytes.argtypes = []
    lib.pb_autotune.argtypes = [i32, i32, i32, dbl, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts), i32,
                                vp, sz, vp, ctypes.POINTER(Tuning)]
    lib.pb_set_tuning.restype = ctypes.c_int
    lib.pb_set_tuning.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Tuning)]
    lib.pb_get_tuning.restype = ctypes.c_int
    lib.pb_get_tuning.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Tuning)]
    lib.pb_set_coded_coefficients.restype = None
    lib.pb_set_coded_coefficients.argtypes = [i32]
    lib.pb_get_coded_coefficients.restype = i32
    lib.pb_get_coded_coefficients.argtypes = []
    lib.pb_set_periodic_pass.restype = None
    lib.pb_set_periodic_pass.argtypes = [i32]
    lib.pb_get_periodic_pass.restype = i32
    lib.pb_get_periodic_pass.argtypes = []
    lib.pb_tiling_candidates.restype = ctypes.c_int
    lib.pb_tiling_candidates.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Tuning), i32, ctypes.POINTER(i32)]
    P = ctypes.POINTER(Problem)
    lib.pb_batch_workspace_bytes.restype = sz
    lib.pb_batch_workspace_bytes.argtypes = [i32, P, i32]
    lib.pb_batch_set_zchunk.restype = ctypes.c_int
    lib.pb_batch_set_zchunk.argtypes = [i32]
    lib.pb_batch_get_zchunk.restype = i32
    lib.pb_batch_get_zchunk.argtypes = []
    lib.pb_batch_autotune_workspace_bytes.restype = sz
    lib.pb_batch_autotune_workspace_bytes.argtypes = [i32, P, i32]
    lib.pb_batch_autotune.restype = ctypes.c_int
    lib.pb_batch_autotune.argtypes = [i32, P, i32, i32, vp, sz, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.pb_solve_batch.restype = ctypes.c_int
    lib.pb_solve_batch.argtypes = [i32, P, i32, vp, sz, vp, ctypes.POINTER(Info)]
    lib.pb_batch_graph_create.restype = ctypes.c_int
    lib.pb_batch_graph_create.argtypes = [i32, P, i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.pb_batch_graph_launch.restype = ctypes.c_int
    lib.pb_batch_graph_launch.argtypes = [vp, vp]
    lib.pb_batch_graph_results.restype = ctypes.c_int
    lib.pb_batch_graph_results.argtypes = [vp, vp, ctypes.POINTER(Info)]
    lib.pb_batch_graph_is_cooperative.restype = i32
    lib.pb_batch_graph_is_cooperative.argtypes = [vp]
    lib.pb_batch_graph_destroy.restype = None
    lib.pb_batch_graph_destroy.argtypes = [vp]
    lib.pb_server_request_bytes.restype = sz
    lib.pb_server_request_bytes.argtypes = [P]
    lib.pb_server_create.restype = ctypes.c_int
    lib.pb_server_create.argtypes = [vp, sz, i32, ctypes.POINTER(vp)]
    lib.pb_server_submit.restype = ctypes.c_int
    lib.pb_server_submit.argtypes = [vp, P, i32, ctypes.POINTER(i64)]
    lib.pb_server_submit_atoms.restype = ctypes.c_int
    lib.pb_server_submit_atoms.argtypes = [vp, G, i64, vp, vp, vp, dbl, dbl, dbl, dbl, i32, i32, vp,
                                           ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.pb_server_request_bytes_atoms.restype = sz
    lib.pb_server_request_bytes_atoms.argtypes = [G, i64]
    lib.pb_server_step.restype = ctypes.c_int
    lib.pb_server_step.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(Info)]
    lib.pb_server_stats.restype = ctypes.c_int
    lib.pb_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.pb_server_destroy.restype = None
    lib.pb_server_destroy.argtypes = [vp]
    lib.pb_energy_workspace_bytes.restype = sz
    lib.pb_energy_workspace_bytes.argtypes = [i64]
    lib.pb_energy.restype = ctypes.c_int
    lib.pb_energy.argtypes = [G, i64, vp, vp, vp, vp, ctypes.POINTER(dbl), vp, sz, vp]
    lib.pb_setup_ex_workspace_bytes.restype = sz
    lib.pb_setup_ex_workspace_bytes.argtypes = [G, i64, ctypes.POINTER(SetupOpts)]
    lib.pb_setup_ex.restype = ctypes.c_int
    lib.pb_setup_ex.argtypes = [G, i64, vp, vp, vp, dbl, dbl, dbl, ctypes.POINTER(SetupOpts), vp, vp, vp, vp, vp, vp,
                                vp, vp, sz, vp]
    lib.pb_solvation_workspace_bytes.restype = sz
    lib.pb_solvation_workspace_bytes.argtypes = [G, i64, ctypes.POINTER(SolveOpts)]
    lib.pb_solvation_energy.restype = ctypes.c_int
    PD, PI = ctypes.POINTER(dbl), ctypes.POINTER(Info)
    lib.pb_solvation_energy.argtypes = [G, i64, vp, vp, vp, dbl, dbl, dbl, ctypes.POINTER(SolveOpts), vp, vp,
                                        PD, PD, PD, PI, PI, vp, sz, vp]
    return lib


lib = _load()


def version() -> str:
    return lib.pb_version().decode()


def last_error() -> str:
    return lib.pb_last_error().decode()


def _check(status: int, allow=(PB_OK,)):
    if status not in allow:
        raise PBError(status, last_error())
    return status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev64(a, device) -> torch.Tensor:
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(device).contiguous()


BOUNDARIES = {"free": 0, "periodic": 1}


def make_grid(nx, ny, nz, h, origin, boundary="free") -> Grid:
    g = Grid()
    g.nx, g.ny, g.nz, g.h = int(nx), int(ny), int(nz), float(h)
    g.boundary = BOUNDARIES[boundary] if isinstance(boundary, str) else int(boundary)
    for d in range(3):
        g.origin[d] = float(origin[d])
    return g


def as_grid(grid, boundary=None) -> Grid:
    """A Grid struct from a Grid or any object with nx, ny, nz, h, origin
    (and optionally boundary); `boundary` overrides it when given."""
    if isinstance(grid, Grid) and boundary is None:
        return grid
    b = boundary if boundary is not None else getattr(grid, "boundary", 0)
    return make_grid(grid.nx, grid.ny, grid.nz, grid.h, grid.origin, b)


@dataclasses.dataclass
class System:
    """Device arrays of the linear system (layouts as in include/pbgpu.h)."""
    grid: Grid
    eps_x: torch.Tensor
    eps_y: torch.Tensor
    eps_z: torch.Tensor
    kappa2: torch.Tensor
    rhs: torch.Tensor
    qgrid: Optional[torch.Tensor] = None
    mask: Optional[torch.Tensor] = None

    @property
    def dims(self):
        return self.grid.nx, self.grid.ny, self.grid.nz


def setup(grid, xyz, radius, charge, eps_in=1.0, eps_out=80.0, kappa_d2=0.0,
          device="cuda", want_q=False, want_mask=False, stream=None, boundary=None,
          edge_model="node") -> System:
    """Build the system of Eq. 3 on the device (pb_setup_ex); boundary "free"
    (default, or the grid's own) or "periodic"; edge_model "node" (two-point
    harmonic mean) or "fraction" (weighted by the inside fraction of each edge)."""
    g = as_grid(grid, boundary)
    nx, ny, nz = g.nx, g.ny, g.nz
    xyz_t = _dev64(xyz, device).reshape(-1)
    rad_t = _dev64(radius, device)
    q_t = _dev64(charge, device)
    natoms = rad_t.numel()
    opt = dict(dtype=torch.float64, device=device)
    ex = torch.empty((nz, ny, nx + 1), **opt)
    ey = torch.empty((nz, ny + 1, nx), **opt)
    ez = torch.empty((nz + 1, ny, nx), **opt)
    k2 = torch.empty((nz, ny, nx), **opt)
    b = torch.empty((nz, ny, nx), **opt)
    qg = torch.empty((nz, ny, nx), **opt) if want_q else None
    mk = torch.empty((nz + 2, ny + 2, nx + 2), dtype=torch.uint8, device=device) if want_mask else None
    so = SetupOpts()
    so.edge_model = EDGE_MODELS[edge_model]
    wsb = lib.pb_setup_ex_workspace_bytes(ctypes.byref(g), natoms, ctypes.byref(so))
    if wsb == 0:
        raise PBError(PB_ERR_ARG, "pb_setup_ex_workspace_bytes rejected the grid / atom count / options")
    ws = torch.empty(wsb, dtype=torch.uint8, device=device)
    st = lib.pb_setup_ex(ctypes.byref(g), natoms, _ptr(xyz_t), _ptr(rad_t), _ptr(q_t), float(eps_in),
                         float(eps_out), float(kappa_d2), ctypes.byref(so), _ptr(ex), _ptr(ey), _ptr(ez), _ptr(k2),
                         _ptr(b), _ptr(qg), _ptr(mk), _ptr(ws), wsb, _stream(stream))
    _check(st)
    return System(g, ex, ey, ez, k2, b, qg, mk)


def solve_workspace_bytes(nx, ny, nz, precision="f32", op="stencil", tol=1e-6) -> int:
    o = SolveOpts()
    o.tol, o.precision, o.op = tol, PRECISIONS[precision], OPERATORS[op]
    return int(lib.pb_solve_workspace_bytes(nx, ny, nz, ctypes.byref(o)))


def solve(sysm: System, tol=1e-6, precision="f32", op="stencil", maxiter=0, x0=None,
          inner_tol=0.0, max_outer=0, workspace: Optional[torch.Tensor] = None, out=None,
          stream=None, check=True):
    """Jacobi PCG on the system. Returns (x, info dict). Raises PBError on a
    negative status (and on PB_NOT_CONVERGED when check is true)."""
    nx, ny, nz = sysm.dims
    o = SolveOpts()
    o.tol, o.maxiter = float(tol), int(maxiter)
    o.precision, o.op = PRECISIONS[precision], OPERATORS[op]
    o.warm_start = 1 if x0 is not None else 0
    o.inner_tol, o.max_outer = float(inner_tol), int(max_outer)
    o.boundary = sysm.grid.boundary
    wsb = lib.pb_solve_workspace_bytes(nx, ny, nz, ctypes.byref(o))
    if wsb == 0:
        raise PBError(PB_ERR_ARG, "pb_solve_workspace_bytes rejected the options")
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=sysm.rhs.device)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float64, device=sysm.rhs.device)
    if x0 is not None:
        out.copy_(torch.as_tensor(x0, dtype=torch.float64).reshape(nz, ny, nx))
    info = Info()
    st = lib.pb_solve(nx, ny, nz, sysm.grid.h, _ptr(sysm.eps_x), _ptr(sysm.eps_y), _ptr(sysm.eps_z),
                      _ptr(sysm.kappa2), _ptr(sysm.rhs), _ptr(out), ctypes.byref(o), _ptr(workspace),
                      workspace.numel(), _stream(stream), ctypes.byref(info))
    _check(st, allow=(PB_OK,) if check else (PB_OK, PB_NOT_CONVERGED))
    return out, info.as_dict()


def solve_noalloc(sysm: System, out: torch.Tensor, tol=1e-6, precision="f32", op="stencil", maxiter=0,
                  warm_start=False, inner_tol=0.0, max_outer=0, stream=None, check=True):
    """pb_solve_noalloc: the solve in the library's per-GPU scratch, no
    workspace and no allocation; `out` (FP64, the grid's shape) receives x
    and holds the initial guess when warm_start. Returns the info dict."""
    nx, ny, nz = sysm.dims
    o = SolveOpts()
    o.tol, o.maxiter = float(tol), int(maxiter)
    o.precision, o.op = PRECISIONS[precision], OPERATORS[op]
    o.warm_start = 1 if warm_start else 0
    o.inner_tol, o.max_outer = float(inner_tol), int(max_outer)
    o.boundary = sysm.grid.boundary
    info = Info()
    st = lib.pb_solve_noalloc(nx, ny, nz, sysm.grid.h, _ptr(sysm.eps_x), _ptr(sysm.eps_y), _ptr(sysm.eps_z),
                              _ptr(sysm.kappa2), _ptr(sysm.rhs), _ptr(out), ctypes.byref(o), _stream(stream),
                              ctypes.byref(info))
    _check(st, allow=(PB_OK,) if check else (PB_OK, PB_NOT_CONVERGED))
    return info.as_dict()


def stream_copy(src: torch.Tensor, dst: torch.Tensor, nontemporal=True, stream=None) -> None:
    """pb_stream_copy of src into dst (same size in bytes, 16-byte multiple)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib.pb_stream_copy(_ptr(src), _ptr(dst), nbytes, 1 if nontemporal else 0, _stream(stream)))


def solve_noalloc_max_bytes() -> int:
    return int(lib.pb_solve_noalloc_max_bytes())


def autotune(sysm: System, precision="f32", iters_per_trial=20,
             workspace: Optional[torch.Tensor] = None, stream=None) -> dict:
    """Time every feasible tiling of the fused kernel on this system and make
    the fastest the default for its grid shape and precision (per process)."""
    nx, ny, nz = sysm.dims
    o = SolveOpts()
    o.tol, o.precision, o.op = 1e-6, PRECISIONS[precision], OPERATORS["stencil"]
    wsb = lib.pb_solve_workspace_bytes(nx, ny, nz, ctypes.byref(o))
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=sysm.rhs.device)
    t = Tuning()
    st = lib.pb_autotune(nx, ny, nz, sysm.grid.h, _ptr(sysm.eps_x), _ptr(sysm.eps_y), _ptr(sysm.eps_z),
                         _ptr(sysm.kappa2), _ptr(sysm.rhs), ctypes.byref(o), int(iters_per_trial),
                         _ptr(workspace), workspace.numel(), _stream(stream), ctypes.byref(t))
    _check(st)
    return t.as_dict()


def set_tuning(nx, ny, nz, precision, block, groups, zchunk, grid, scheme=0, streaming=-1, segments=0) -> None:
    """Record a tiling of the fused kernel for this grid shape and precision;
    scheme 0 is the pass that stores A.p, 1 the 40-byte pass that recomputes it;
    streaming 1 / 0 selects nontemporal / cached accesses, -1 the shape's default;
    segments > 0 picks the tiling with that many in-plane segments."""
    t = Tuning()
    t.block, t.groups, t.zchunk, t.grid = int(block), int(groups), int(zchunk), int(grid)
    t.scheme, t.streaming, t.segments = int(scheme), int(streaming), int(segments)
    _check(lib.pb_set_tuning(int(nx), int(ny), int(nz), PRECISIONS[precision], ctypes.byref(t)))


def set_coded_coefficients(on: bool) -> None:
    """Process-wide switch of the coded-coefficient 40-byte FP32 pass (on by
    default; used when the operator holds at most 256 distinct FP32 values)."""
    lib.pb_set_coded_coefficients(1 if on else 0)


def get_coded_coefficients() -> bool:
    return bool(lib.pb_get_coded_coefficients())


def set_periodic_pass(form: int) -> None:
    """Pass form of periodic fused solves, process-wide: -1 the model's
    choice (the default), 0 the pass that stores A.p, 1 the 40-byte pass on
    ghost-row copies (grids with nx >= 5, ny >= 4)."""
    lib.pb_set_periodic_pass(int(form))


def get_periodic_pass() -> int:
    return int(lib.pb_get_periodic_pass())


def get_tuning(nx, ny, nz, precision="f32") -> dict:
    """The tiling (and pass form) solves of this shape and precision will use."""
    t = Tuning()
    _check(lib.pb_get_tuning(int(nx), int(ny), int(nz), PRECISIONS[precision], ctypes.byref(t)))
    d = t.as_dict()
    d.pop("us_per_iter")
    d.pop("candidates")
    return d


def tiling_candidates(nx, ny, nz, precision="f32") -> list:
    """Every feasible tiling of the fused kernel for this shape and precision
    on the current device (the autotuner's search space), as dicts."""
    n = ctypes.c_int32(0)
    _check(lib.pb_tiling_candidates(int(nx), int(ny), int(nz), PRECISIONS[precision], None, 0, ctypes.byref(n)))
    arr = (Tuning * max(1, n.value))()
    _check(lib.pb_tiling_candidates(int(nx), int(ny), int(nz), PRECISIONS[precision], arr, n.value,
                                    ctypes.byref(n)))
    return [arr[i].as_dict() for i in range(n.value)]


def save_tuning(path, entries) -> None:
    """Write autotune results [{nx, ny, nz, precision, block, groups, zchunk, grid, ...}] as JSON."""
    import json
    with open(path, "w") as f:
        json.dump(entries, f, indent=1)


def load_tuning(path) -> int:
    """Record every feasible tiling of a saved JSON table; returns how many were applied."""
    import json
    n = 0
    for e in json.load(open(path)):
        try:
            set_tuning(e["nx"], e["ny"], e["nz"], e["precision"], e["block"], e["groups"], e["zchunk"], e["grid"])
            n += 1
        except PBError:
            pass
    return n


def _problems(systems, tol, maxiter, outs, x0s):
    n = len(systems)
    arr = (Problem * n)()
    tols = tol if isinstance(tol, (list, tuple)) else [tol] * n
    for i, sm in enumerate(systems):
        nx, ny, nz = sm.dims
        p = arr[i]
        p.nx, p.ny, p.nz, p.maxiter = nx, ny, nz, int(maxiter)
        p.h, p.tol = sm.grid.h, float(tols[i])
        p.eps_x, p.eps_y, p.eps_z = sm.eps_x.data_ptr(), sm.eps_y.data_ptr(), sm.eps_z.data_ptr()
        p.kappa2, p.rhs, p.x = sm.kappa2.data_ptr(), sm.rhs.data_ptr(), outs[i].data_ptr()
        p.warm_start = 1 if (x0s is not None and x0s[i] is not None) else 0
    return arr


def _outs(systems, outs, x0s):
    if outs is None:
        outs = [torch.empty(sm.rhs.shape, dtype=torch.float64, device=sm.rhs.device) for sm in systems]
    if x0s is not None:
        for o, x0 in zip(outs, x0s):
            if x0 is not None:
                o.copy_(torch.as_tensor(x0, dtype=torch.float64).reshape(o.shape))
    return outs


def set_batch_zchunk(zchunk: int) -> None:
    """Set the batched and served kernels' z-chunk (planes per tile) on the current device."""
    _check(lib.pb_batch_set_zchunk(int(zchunk)))


def get_batch_zchunk() -> int:
    return int(lib.pb_batch_get_zchunk())


def batch_autotune(systems, precision="f32", iters_per_trial=20, stream=None) -> dict:
    """Time the batched kernel's candidate z-chunks on these systems (each
    problem capped at iters_per_trial iterations; no array of the systems is
    written) and make the fastest the device's batch z-chunk."""
    outs = _outs(systems, None, None)
    arr = _problems(systems, 1e-30, 0, outs, None)
    n = len(systems)
    prec = PRECISIONS[precision]
    wsb = lib.pb_batch_autotune_workspace_bytes(n, arr, prec)
    if wsb == 0:
        raise PBError(PB_ERR_ARG, last_error() or "pb_batch_autotune_workspace_bytes rejected the batch")
    ws = torch.empty(wsb, dtype=torch.uint8, device=systems[0].rhs.device)
    z, sec = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib.pb_batch_autotune(n, arr, prec, int(iters_per_trial), _ptr(ws), wsb, _stream(stream),
                                 ctypes.byref(z), ctypes.byref(sec)))
    return {"zchunk": z.value, "seconds": sec.value}


def solve_batch(systems, tol=1e-6, precision="f32", maxiter=0, outs=None, x0s=None,
                workspace: Optional[torch.Tensor] = None, stream=None, check=True):
    """Solve many systems in one persistent launch. Returns (list of x, list of info dicts)."""
    outs = _outs(systems, outs, x0s)
    arr = _problems(systems, tol, maxiter, outs, x0s)
    n = len(systems)
    prec = PRECISIONS[precision]
    wsb = lib.pb_batch_workspace_bytes(n, arr, prec)
    if wsb == 0:
        raise PBError(PB_ERR_ARG, last_error() or "pb_batch_workspace_bytes rejected the batch")
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=systems[0].rhs.device)
    infos = (Info * n)()
    st = lib.pb_solve_batch(n, arr, prec, _ptr(workspace), workspace.numel(), _stream(stream), infos)
    _check(st, allow=(PB_OK,) if check else (PB_OK, PB_NOT_CONVERGED) + tuple(range(-6, 0)))
    return outs, [i.as_dict() for i in infos]


class BatchGraph:
    """A batch recorded once in a HIP graph and replayed by launch(). Input
    tensors keep their addresses; their contents may change between launches."""

    def __init__(self, systems, tol=1e-6, precision="f32", maxiter=0, outs=None, stream=None):
        self.systems = list(systems)
        self.outs = _outs(self.systems, outs, None)
        self._arr = _problems(self.systems, tol, maxiter, self.outs, None)
        n = len(self.systems)
        prec = PRECISIONS[precision]
        wsb = lib.pb_batch_workspace_bytes(n, self._arr, prec)
        if wsb == 0:
            raise PBError(PB_ERR_ARG, last_error() or "pb_batch_workspace_bytes rejected the batch")
        self.workspace = torch.empty(wsb, dtype=torch.uint8, device=self.systems[0].rhs.device)
        h = ctypes.c_void_p()
        _check(lib.pb_batch_graph_create(n, self._arr, prec, _ptr(self.workspace), wsb, _stream(stream),
                                         ctypes.byref(h)))
        self._h = h

    @property
    def cooperative(self) -> bool:
        return bool(lib.pb_batch_graph_is_cooperative(self._h))

    def launch(self, stream=None):
        _check(lib.pb_batch_graph_launch(self._h, _stream(stream)))

    def results(self, stream=None, check=True):
        n = len(self.systems)
        infos = (Info * n)()
        st = lib.pb_batch_graph_results(self._h, _stream(stream), infos)
        _check(st, allow=(PB_OK,) if check else (PB_OK, PB_NOT_CONVERGED) + tuple(range(-6, 0)))
        return [i.as_dict() for i in infos]

    def close(self):
        if getattr(self, "_h", None):
            lib.pb_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server over a device arena of `arena_bytes`
    (the HBM budget). submit() queues a request; step() admits, advances every
    active request by `chunk` iterations in one launch and returns the
    requests that finished as [(id, info)]."""

    def __init__(self, arena_bytes: int, max_slots: int = 256, device="cuda", keep_outputs=True):
        self.keep_outputs = keep_outputs
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib.pb_server_create(_ptr(self.arena), self.arena.numel(), int(max_slots), ctypes.byref(h)))
        self._h = h
        self._live = {}        # id -> (system, out, problem struct): keeps request memory alive
        self.outputs = {}      # id -> potential tensor of finished requests
        self.energies = {}     # id -> energy (kcal/mol) of finished molecule requests

    @staticmethod
    def request_bytes(sysm: System) -> int:
        arr = _problems([sysm], 1e-6, 0, [sysm.rhs], None)
        return int(lib.pb_server_request_bytes(arr))

    def submit(self, sysm: System, tol=1e-6, precision="f32", maxiter=0, out=None, x0=None) -> int:
        outs = _outs([sysm], None if out is None else [out], None if x0 is None else [x0])
        arr = _problems([sysm], tol, maxiter, outs, None if x0 is None else [x0])
        rid = ctypes.c_int64()
        _check(lib.pb_server_submit(self._h, arr, PRECISIONS[precision], ctypes.byref(rid)))
        self._live[rid.value] = (sysm, outs[0], arr)
        return rid.value

    @staticmethod
    def request_bytes_atoms(grid, natoms: int) -> int:
        g = as_grid(grid)
        return int(lib.pb_server_request_bytes_atoms(ctypes.byref(g), int(natoms)))

    def submit_atoms(self, grid, xyz, radius, charge, eps_in=1.0, eps_out=80.0, kappa_d2=0.0, tol=1e-6,
                     precision="f32", maxiter=0, out=None) -> int:
        """Queue a molecule (atoms, radii, charges on `grid`): the server runs
        the setup at admission and the energy at completion. On completion
        outputs[id] is the potential and energies[id] the energy (kcal/mol)."""
        g = as_grid(grid, "free")
        dev = self.arena.device
        xyz_t = _dev64(xyz, dev).reshape(-1)
        rad_t = _dev64(radius, dev)
        q_t = _dev64(charge, dev)
        if out is None:
            out = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float64, device=dev)
        e = ctypes.c_double(float("nan"))
        rid = ctypes.c_int64()
        _check(lib.pb_server_submit_atoms(self._h, ctypes.byref(g), rad_t.numel(), _ptr(xyz_t), _ptr(rad_t),
                                          _ptr(q_t), float(eps_in), float(eps_out), float(kappa_d2), float(tol),
                                          int(maxiter), PRECISIONS[precision], _ptr(out), ctypes.byref(e),
                                          ctypes.byref(rid)))
        self._live[rid.value] = ((g, xyz_t, rad_t, q_t), out, e)
        return rid.value

    def step(self, chunk=32, stream=None, max_done=256):
        n = ctypes.c_int32()
        ids = (ctypes.c_int64 * max_done)()
        infos = (Info * max_done)()
        _check(lib.pb_server_step(self._h, int(chunk), _stream(stream), int(max_done), ctypes.byref(n), ids, infos))
        done = []
        for k in range(n.value):
            rid = ids[k]
            _, out, extra = self._live.pop(rid)
            if self.keep_outputs:
                self.outputs[rid] = out
            if isinstance(extra, ctypes.c_double):
                self.energies[rid] = extra.value
            done.append((rid, infos[k].as_dict()))
        return done

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib.pb_server_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib.pb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy(grid, xyz, charge, x: torch.Tensor, atom_phi: Optional[torch.Tensor] = None,
           stream=None, boundary=None) -> float:
    g = as_grid(grid, boundary)
    dev = x.device
    xyz_t = _dev64(xyz, dev).reshape(-1)
    q_t = _dev64(charge, dev)
    natoms = q_t.numel()
    wsb = lib.pb_energy_workspace_bytes(natoms)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    e = ctypes.c_double(0.0)
    st = lib.pb_energy(ctypes.byref(g), natoms, _ptr(xyz_t), _ptr(q_t), _ptr(x), _ptr(atom_phi),
                       ctypes.byref(e), _ptr(ws), wsb, _stream(stream))
    _check(st)
    return float(e.value)


def solvation_energy(grid, xyz, radius, charge, eps_in=1.0, eps_out=80.0, kappa_d2=0.0, tol=1e-6,
                     precision="f32", op="stencil", maxiter=0, inner_tol=0.0, max_outer=0, device="cuda",
                     want_phi=False, stream=None, check=True, boundary=None) -> dict:
    """Solvation energy dG = E(solvent) - E(uniform eps_in reference) in
    kcal/mol from two solves on the same grid (pb_solvation_energy)."""
    g = as_grid(grid, boundary)
    nx, ny, nz = g.nx, g.ny, g.nz
    xyz_t = _dev64(xyz, device).reshape(-1)
    rad_t = _dev64(radius, device)
    q_t = _dev64(charge, device)
    natoms = rad_t.numel()
    o = SolveOpts()
    o.tol, o.maxiter = float(tol), int(maxiter)
    o.precision, o.op = PRECISIONS[precision], OPERATORS[op]
    o.inner_tol, o.max_outer = float(inner_tol), int(max_outer)
    wsb = lib.pb_solvation_workspace_bytes(ctypes.byref(g), natoms, ctypes.byref(o))
    if wsb == 0:
        raise PBError(PB_ERR_ARG, "pb_solvation_workspace_bytes rejected the grid / atoms / options")
    ws = torch.empty(wsb, dtype=torch.uint8, device=device)
    phs = [torch.empty((nz, ny, nx), dtype=torch.float64, device=device) for _ in range(2)] if want_phi \
        else [None, None]
    dg, es, er = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    i_s, i_r = Info(), Info()
    st = lib.pb_solvation_energy(ctypes.byref(g), natoms, _ptr(xyz_t), _ptr(rad_t), _ptr(q_t), float(eps_in),
                                 float(eps_out), float(kappa_d2), ctypes.byref(o), _ptr(phs[0]), _ptr(phs[1]),
                                 ctypes.byref(dg), ctypes.byref(es), ctypes.byref(er), ctypes.byref(i_s),
                                 ctypes.byref(i_r), _ptr(ws), wsb, _stream(stream))
    _check(st, allow=(PB_OK,) if check else (PB_OK, PB_NOT_CONVERGED))
    out = {"dG": dg.value, "e_solv": es.value, "e_ref": er.value, "info_solv": i_s.as_dict(),
           "info_ref": i_r.as_dict(), "status": st}
    if want_phi:
        out["phi_solv"], out["phi_ref"] = phs
    return out

"""Python binding of the C ABI in include/ftc.h (argument marshalling only).

Every function here has the name of a C entry point without the ``ftc_``
prefix, checks that the torch tensors it is given are CUDA (HIP) tensors of
the right dtype and size, and passes their device pointers and torch's current
stream to ``libftc.so``.  All arithmetic happens in the library's kernels;
there is no CPU fallback: if the library is missing or no GPU is present, the
calls raise.

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already loaded (same soname): device pointers and
stream handles from torch are then valid in the library.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import inputs as _inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftc.so")

FTC_OK, FTC_EINVAL, FTC_EDOMAIN, FTC_EMESH, FTC_ECAPACITY, FTC_ENOMEM, FTC_EHIP = 0, -1, -2, -3, -4, -5, -6
FTC_CELL_RANK, FTC_CELL_OVERFLOW, FTC_CELL_SURROGATE = 1, 2, 4
# learned curvature: feature row width, parameter count, loss-gradient work floats
MLP_FEATURES, MLP_PARAMS = 32, 6209
MLP_WORK_FLOATS = 256 * (MLP_PARAMS + 3)

EXPORTED = ["ftc_cells_create", "ftc_cells_destroy", "ftc_build_cell_lists", "ftc_cells_count",
            "ftc_cells_view", "ftc_volume_fraction", "ftc_ppic_curvature", "ftc_csf_force",
            "ftc_interp_vertex_velocity", "ftc_last_device_error", "ftc_set_timing", "ftc_kernel_time",
            "ftc_csf_force_band", "ftc_advect_vertices_rk4", "ftc_curvature_features", "ftc_mlp_forward",
            "ftc_mlp_loss_grad", "ftc_mlp_loss_grad_static", "ftc_mlp_adam", "ftc_learned_curvature", "ftc_front_roughness",
            "ftc_smooth_rough_edges", "ftc_get_tuning", "ftc_set_tuning", "ftc_surface_tension_flux",
            "ftc_paraboloid_cell", "ftc_status_str"]

# ftc_kernel values (timing)
KERNELS = {"tri_pieces": 0, "piece_rank": 1, "columns": 2, "ppic": 3, "csf": 4, "interp": 5, "surrogate": 6}


class _CGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double), ("h", C.c_double)]


class _CMesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("t0", C.c_void_p), ("t1", C.c_void_p), ("t2", C.c_void_p)]


class _CParams(C.Structure):
    _fields_ = [("delta_over_h", C.c_double), ("rings", C.c_int32), ("n_min", C.c_int32),
                ("grow", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32)]


@dataclass(frozen=True)
class PPICParams:
    """Volume-fit parameters; defaults are the paper's (section 3.2).
    precision 0: normal equations in double precision; 1: formed and
    factored in single precision, refined with double-precision residuals."""
    delta_over_h: float = 2.5
    rings: int = 3
    n_min: int = 24
    grow: float = 1.1
    max_iter: int = 16
    precision: int = 0


class _CTuning(C.Structure):
    _fields_ = [("ring_lanes", C.c_int32), ("column_chunks", C.c_int32), ("ring_blocks", C.c_int32),
                ("queue_chunk", C.c_int32)]


@dataclass(frozen=True)
class Tuning:
    """Launch shapes of a workspace (see ftc_tuning in include/ftc.h)."""
    ring_lanes: int = 8
    column_chunks: int = 16
    ring_blocks: int = 0
    queue_chunk: int = 0


class FTCError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_str(code)} ({code})")
        self.code = code


_lib = None
_hip = None


def lib() -> C.CDLL:
    """The loaded libftc.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_06932_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    L.ftc_cells_create.argtypes = [P(vp), P(_CGrid), C.c_int32, C.c_int32, C.c_int64, C.c_int32]
    L.ftc_cells_create.restype = C.c_int32
    L.ftc_cells_destroy.argtypes = [vp]
    L.ftc_cells_destroy.restype = None
    L.ftc_build_cell_lists.argtypes = [vp, P(_CGrid), P(_CMesh), vp]
    L.ftc_build_cell_lists.restype = C.c_int32
    L.ftc_cells_count.argtypes = [vp, P(C.c_int32), P(C.c_int64), vp]
    L.ftc_cells_count.restype = C.c_int32
    L.ftc_cells_view.argtypes = [vp, P(vp), P(vp), P(vp), P(vp)]
    L.ftc_cells_view.restype = C.c_int32
    L.ftc_volume_fraction.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, vp]
    L.ftc_volume_fraction.restype = C.c_int32
    L.ftc_ppic_curvature.argtypes = [vp, P(_CGrid), P(_CMesh), P(_CParams), vp, vp, vp, vp, vp, vp, vp, vp]
    L.ftc_ppic_curvature.restype = C.c_int32
    L.ftc_csf_force.argtypes = [vp, P(_CGrid), vp, vp, C.c_double, vp, vp, vp, vp]
    L.ftc_csf_force.restype = C.c_int32
    L.ftc_csf_force_band.argtypes = [vp, P(_CGrid), vp, vp, vp, vp, vp, C.c_double, C.c_int32, vp, vp, vp, vp, vp,
                                     vp, vp]
    L.ftc_csf_force_band.restype = C.c_int32
    L.ftc_surface_tension_flux.argtypes = [vp, P(_CGrid), vp, vp, C.c_int32, vp, vp, vp, C.c_double, C.c_double,
                                           C.c_double, vp, vp, vp]
    L.ftc_surface_tension_flux.restype = C.c_int32
    L.ftc_paraboloid_cell.argtypes = [vp, P(_CGrid), vp, vp, vp, vp, vp]
    L.ftc_paraboloid_cell.restype = C.c_int32
    L.ftc_interp_vertex_velocity.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, vp, vp, vp, vp, vp]
    L.ftc_interp_vertex_velocity.restype = C.c_int32
    L.ftc_advect_vertices_rk4.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, vp, C.c_double, vp, vp, vp, vp]
    L.ftc_advect_vertices_rk4.restype = C.c_int32
    L.ftc_curvature_features.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, vp, vp]
    L.ftc_curvature_features.restype = C.c_int32
    L.ftc_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_int32, vp, vp]
    L.ftc_mlp_forward.restype = C.c_int32
    L.ftc_mlp_loss_grad.argtypes = [vp, vp, C.c_int64, vp, vp, vp, C.c_int32, vp, vp, vp, vp]
    L.ftc_mlp_loss_grad.restype = C.c_int32
    L.ftc_mlp_loss_grad_static.argtypes = [vp, vp, C.c_int64, vp, vp, vp, C.c_int32, vp, vp, vp]
    L.ftc_mlp_loss_grad_static.restype = C.c_int32
    L.ftc_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.ftc_mlp_adam.restype = C.c_int32
    L.ftc_learned_curvature.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, C.c_double, P(_CParams), vp, vp, vp, vp,
                                        vp, vp, vp, vp]
    L.ftc_learned_curvature.restype = C.c_int32
    L.ftc_front_roughness.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, vp]
    L.ftc_front_roughness.restype = C.c_int32
    L.ftc_smooth_rough_edges.argtypes = [vp, P(_CGrid), P(_CMesh), vp, vp, C.c_double, C.c_double, C.c_int32, vp, vp,
                                         vp, vp, vp]
    L.ftc_smooth_rough_edges.restype = C.c_int32
    L.ftc_get_tuning.argtypes = [vp, P(_CTuning)]
    L.ftc_get_tuning.restype = C.c_int32
    L.ftc_set_tuning.argtypes = [vp, P(_CTuning)]
    L.ftc_set_tuning.restype = C.c_int32
    L.ftc_last_device_error.argtypes = [vp, P(C.c_int32), vp]
    L.ftc_last_device_error.restype = C.c_int32
    L.ftc_set_timing.argtypes = [vp, C.c_int32]
    L.ftc_set_timing.restype = C.c_int32
    L.ftc_kernel_time.argtypes = [vp, C.c_int32, P(C.c_float)]
    L.ftc_kernel_time.restype = C.c_int32
    L.ftc_status_str.argtypes = [C.c_int32]
    L.ftc_status_str.restype = C.c_char_p
    _lib = L
    return L


def _hip_rt() -> C.CDLL:
    """torch's HIP runtime (already loaded), for device-to-device copies."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so.7")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    return _hip


def status_str(code: int) -> str:
    try:
        return lib().ftc_status_str(int(code)).decode()
    except ImportError:
        return "library missing"


def _check(code: int, what: str) -> None:
    if code != FTC_OK:
        raise FTCError(code, what)


def _stream(stream) -> C.c_void_p:
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the coupling library runs only on the GPU")
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t, dtype, n, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return C.c_void_p(t.data_ptr())


def c_grid(grid: _inputs.Grid) -> _CGrid:
    return _CGrid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0, grid.h)


class DeviceMesh:
    """A front held in device memory (torch tensors) plus its C descriptor."""

    def __init__(self, x, y, z, t0, t1, t2):
        self.x, self.y, self.z, self.t0, self.t1, self.t2 = x, y, z, t0, t1, t2
        nv, nt = x.numel(), t0.numel()
        for name, t, dt, n in (("x", x, torch.float64, nv), ("y", y, torch.float64, nv),
                               ("z", z, torch.float64, nv), ("t0", t0, torch.int32, nt),
                               ("t1", t1, torch.int32, nt), ("t2", t2, torch.int32, nt)):
            _ptr(t, dt, n, name)
        self.c = _CMesh(nv, nt, x.data_ptr(), y.data_ptr(), z.data_ptr(), t0.data_ptr(),
                        t1.data_ptr(), t2.data_ptr())

    @property
    def nv(self) -> int:
        return self.c.nv

    @property
    def nt(self) -> int:
        return self.c.nt

    @staticmethod
    def from_host(mesh: _inputs.Mesh, device="cuda") -> "DeviceMesh":
        f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        return DeviceMesh(f(mesh.x, torch.float64), f(mesh.y, torch.float64), f(mesh.z, torch.float64),
                          f(mesh.t0, torch.int32), f(mesh.t1, torch.int32), f(mesh.t2, torch.int32))


class Cells:
    """The opaque workspace (ftc_cells_create / ftc_cells_destroy)."""

    def __init__(self, grid: _inputs.Grid, nv_capacity: int, nt_capacity: int, pair_capacity: int,
                 cell_capacity: int):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the coupling library runs only on the GPU")
        torch.cuda.init()
        self._lib = lib()
        self.grid = grid
        self.cg = c_grid(grid)
        self.nv_capacity, self.nt_capacity = int(nv_capacity), int(nt_capacity)
        self.pair_capacity, self.cell_capacity = int(pair_capacity), int(cell_capacity)
        h = C.c_void_p()
        _check(self._lib.ftc_cells_create(C.byref(h), C.byref(self.cg), self.nv_capacity,
                                          self.nt_capacity, self.pair_capacity, self.cell_capacity),
               "ftc_cells_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.ftc_cells_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def count(self, stream=None):
        n_if, n_p = C.c_int32(), C.c_int64()
        _check(self._lib.ftc_cells_count(self.handle, C.byref(n_if), C.byref(n_p), _stream(stream)),
               "ftc_cells_count")
        return int(n_if.value), int(n_p.value)

    def lists(self, stream=None):
        """(cell_ids, offsets, tri_ids) of the last build, copied into new
        int32 tensors sized by the current counts."""
        n_if, n_p = self.count(stream)
        pc, po, pt, pn = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(self._lib.ftc_cells_view(self.handle, C.byref(pc), C.byref(po), C.byref(pt), C.byref(pn)),
               "ftc_cells_view")
        s = _stream(stream)
        out = []
        for p, n in ((pc, n_if), (po, n_if + 1), (pt, n_p)):
            t = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            if n > 0:
                r = _hip_rt().hipMemcpyAsync(C.c_void_p(t.data_ptr()), p, 4 * n, 3, s)  # device to device
                if r != 0:
                    raise FTCError(FTC_EHIP, "hipMemcpyAsync")
            out.append(t[:n])
        torch.cuda.current_stream().synchronize()
        return tuple(out)

    def set_timing(self, enable: bool) -> None:
        _check(self._lib.ftc_set_timing(self.handle, 1 if enable else 0), "ftc_set_timing")

    def kernel_time(self, kernel: str) -> float:
        """Milliseconds of the last timed launch of `kernel` (see KERNELS)."""
        ms = C.c_float()
        _check(self._lib.ftc_kernel_time(self.handle, KERNELS[kernel], C.byref(ms)), "ftc_kernel_time")
        return float(ms.value)

    def last_device_error(self, stream=None) -> int:
        code = C.c_int32()
        _check(self._lib.ftc_last_device_error(self.handle, C.byref(code), _stream(stream)),
               "ftc_last_device_error")
        return int(code.value)


def build_cell_lists(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, stream=None) -> None:
    cg = c_grid(grid)
    _check(lib().ftc_build_cell_lists(cells.handle, C.byref(cg), C.byref(mesh.c), _stream(stream)),
           "ftc_build_cell_lists")


def volume_fraction(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, alpha_if, alpha_dense=None,
                    stream=None) -> None:
    cg = c_grid(grid)
    a = _ptr(alpha_if, torch.float64, cells.cell_capacity, "alpha_if")
    d = _ptr(alpha_dense, torch.float64, grid.ncell, "alpha_dense")
    _check(lib().ftc_volume_fraction(cells.handle, C.byref(cg), C.byref(mesh.c), a, d, _stream(stream)),
           "ftc_volume_fraction")


def ppic_curvature(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, kappa, nx, ny, nz, coeff=None,
                   cell_status=None, diag=None, params: PPICParams | None = None, stream=None) -> None:
    cg = c_grid(grid)
    cap = cells.cell_capacity
    p = None
    if params is not None:
        p = C.byref(_CParams(params.delta_over_h, params.rings, params.n_min, params.grow, params.max_iter,
                             params.precision))
    _check(lib().ftc_ppic_curvature(cells.handle, C.byref(cg), C.byref(mesh.c), p,
                                    _ptr(kappa, torch.float64, cap, "kappa"),
                                    _ptr(nx, torch.float64, cap, "nx"), _ptr(ny, torch.float64, cap, "ny"),
                                    _ptr(nz, torch.float64, cap, "nz"),
                                    _ptr(coeff, torch.float64, 6 * cap, "coeff"),
                                    _ptr(cell_status, torch.int32, cap, "cell_status"),
                                    _ptr(diag, torch.int32, 4 * cap, "diag"), _stream(stream)),
           "ftc_ppic_curvature")


def csf_force(cells: Cells, grid: _inputs.Grid, alpha_dense, kappa, sigma: float, fx, fy, fz,
              stream=None) -> None:
    cg = c_grid(grid)
    cap = cells.cell_capacity
    _check(lib().ftc_csf_force(cells.handle, C.byref(cg), _ptr(alpha_dense, torch.float64, grid.ncell, "alpha"),
                               _ptr(kappa, torch.float64, cap, "kappa"), float(sigma),
                               _ptr(fx, torch.float64, cap, "fx"), _ptr(fy, torch.float64, cap, "fy"),
                               _ptr(fz, torch.float64, cap, "fz"), _stream(stream)),
           "ftc_csf_force")


def csf_force_band(cells: Cells, grid: _inputs.Grid, alpha_dense, kappa, nx, ny, nz, sigma: float, band_ids,
                   kappa_band, fx, fy, fz, n_band, stream=None) -> None:
    """Band mode: outputs sized by band_ids.numel() (the band capacity);
    n_band is a one-element int32 device tensor receiving the band count."""
    cg = c_grid(grid)
    cap = cells.cell_capacity
    bcap = int(band_ids.numel())
    _check(lib().ftc_csf_force_band(cells.handle, C.byref(cg),
                                    _ptr(alpha_dense, torch.float64, grid.ncell, "alpha"),
                                    _ptr(kappa, torch.float64, cap, "kappa"), _ptr(nx, torch.float64, cap, "nx"),
                                    _ptr(ny, torch.float64, cap, "ny"), _ptr(nz, torch.float64, cap, "nz"),
                                    float(sigma), bcap, _ptr(band_ids, torch.int32, bcap, "band_ids"),
                                    _ptr(kappa_band, torch.float64, bcap, "kappa_band"),
                                    _ptr(fx, torch.float64, bcap, "fx"), _ptr(fy, torch.float64, bcap, "fy"),
                                    _ptr(fz, torch.float64, bcap, "fz"), _ptr(n_band, torch.int32, 1, "n_band"),
                                    _stream(stream)),
           "ftc_csf_force_band")


def paraboloid_cell(cells: Cells, grid: _inputs.Grid, coeff, alpha_out, kappa_out=None, normal_out=None,
                    stream=None) -> None:
    """alpha under each interfacial cell's fitted paraboloid and, if asked,
    the curvature and normal integrated over its part inside the cell; coeff
    [6, cell_capacity] from the last ppic_curvature, alpha_out and kappa_out
    [cell_capacity], normal_out [3, cell_capacity]."""
    cg = c_grid(grid)
    cap = cells.cell_capacity
    _check(lib().ftc_paraboloid_cell(cells.handle, C.byref(cg), _ptr(coeff, torch.float64, 6 * cap, "coeff"),
                                     _ptr(alpha_out, torch.float64, cap, "alpha_out"),
                                     _ptr(kappa_out, torch.float64, cap, "kappa_out"),
                                     _ptr(normal_out, torch.float64, 3 * cap, "normal_out"), _stream(stream)),
           "ftc_paraboloid_cell")


def surface_tension_flux(cells: Cells, grid: _inputs.Grid, alpha_dense, kappa, band_ids, kappa_band, n_band,
                         rho_a: float, rho_b: float, sigma: float, flux_if, flux_band, stream=None) -> None:
    """Surface-tension part of the face flux (Eq. mwi_disc) over d_f A_f:
    flux_if [6, cell_capacity], flux_band [6, band capacity]; band_ids,
    kappa_band and n_band as written by the last csf_force_band."""
    cg = c_grid(grid)
    cap = cells.cell_capacity
    bcap = int(band_ids.numel())
    _check(lib().ftc_surface_tension_flux(cells.handle, C.byref(cg),
                                          _ptr(alpha_dense, torch.float64, grid.ncell, "alpha"),
                                          _ptr(kappa, torch.float64, cap, "kappa"), bcap,
                                          _ptr(band_ids, torch.int32, bcap, "band_ids"),
                                          _ptr(kappa_band, torch.float64, bcap, "kappa_band"),
                                          _ptr(n_band, torch.int32, 1, "n_band"), float(rho_a), float(rho_b),
                                          float(sigma), _ptr(flux_if, torch.float64, 6 * cap, "flux_if"),
                                          _ptr(flux_band, torch.float64, 6 * bcap, "flux_band"), _stream(stream)),
           "ftc_surface_tension_flux")


def advect_vertices_rk4(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, U, V, W, dt: float, x_out, y_out, z_out,
                        stream=None) -> None:
    cg = c_grid(grid)
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    nv = mesh.nv
    _check(lib().ftc_advect_vertices_rk4(cells.handle, C.byref(cg), C.byref(mesh.c),
                                         _ptr(U, torch.float64, (nx + 1) * ny * nz, "U"),
                                         _ptr(V, torch.float64, nx * (ny + 1) * nz, "V"),
                                         _ptr(W, torch.float64, nx * ny * (nz + 1), "W"), float(dt),
                                         _ptr(x_out, torch.float64, nv, "x_out"), _ptr(y_out, torch.float64, nv, "y_out"),
                                         _ptr(z_out, torch.float64, nv, "z_out"), _stream(stream)),
           "ftc_advect_vertices_rk4")


def interp_vertex_velocity(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, U, V, W, ux, uy, uz,
                           stream=None) -> None:
    cg = c_grid(grid)
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    nv = mesh.nv
    _check(lib().ftc_interp_vertex_velocity(cells.handle, C.byref(cg), C.byref(mesh.c),
                                            _ptr(U, torch.float64, (nx + 1) * ny * nz, "U"),
                                            _ptr(V, torch.float64, nx * (ny + 1) * nz, "V"),
                                            _ptr(W, torch.float64, nx * ny * (nz + 1), "W"),
                                            _ptr(ux, torch.float64, nv, "ux"), _ptr(uy, torch.float64, nv, "uy"),
                                            _ptr(uz, torch.float64, nv, "uz"), _stream(stream)),
           "ftc_interp_vertex_velocity")


# ------------------------------------------------------------ learned curvature
def curvature_features(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, alpha_dense, features,
                       final_flags=None, stream=None) -> None:
    """Feature rows [cell_capacity, 32] (float32) of the interfacial cells."""
    cg = c_grid(grid)
    cap = cells.cell_capacity
    _check(lib().ftc_curvature_features(cells.handle, C.byref(cg), C.byref(mesh.c),
                                        _ptr(alpha_dense, torch.float64, grid.ncell, "alpha_dense"),
                                        _ptr(features, torch.float32, cap * MLP_FEATURES, "features"),
                                        _ptr(final_flags, torch.int32, cap, "final_flags"), _stream(stream)),
           "ftc_curvature_features")


def _rows(X):
    if X.dim() != 2 or X.shape[1] != MLP_FEATURES:
        raise ValueError(f"X must be [rows, {MLP_FEATURES}]")
    return X.shape[0]


def mlp_forward(theta, X, y, n=None, idx=None, sym=None, stream=None) -> None:
    rows = _rows(X)
    n = rows if n is None and idx is None else (int(idx.numel()) if n is None else int(n))
    _check(lib().ftc_mlp_forward(_ptr(theta, torch.float32, MLP_PARAMS, "theta"),
                                 _ptr(X, torch.float32, rows * MLP_FEATURES, "X"), rows,
                                 _ptr(idx, torch.int32, n, "idx"), _ptr(sym, torch.int32, n, "sym"), n,
                                 _ptr(y, torch.float32, n, "y"), _stream(stream)), "ftc_mlp_forward")


def mlp_loss_grad(theta, X, t, grad, work, loss=None, n=None, idx=None, sym=None, stream=None) -> None:
    rows = _rows(X)
    n = rows if n is None and idx is None else (int(idx.numel()) if n is None else int(n))
    _check(lib().ftc_mlp_loss_grad(_ptr(theta, torch.float32, MLP_PARAMS, "theta"),
                                   _ptr(X, torch.float32, rows * MLP_FEATURES, "X"), rows,
                                   _ptr(idx, torch.int32, n, "idx"), _ptr(sym, torch.int32, n, "sym"),
                                   _ptr(t, torch.float32, rows, "t"), n, _ptr(grad, torch.float32, MLP_PARAMS, "grad"),
                                   _ptr(loss, torch.float32, 1, "loss"),
                                   _ptr(work, torch.float32, MLP_WORK_FLOATS, "work"), _stream(stream)),
           "ftc_mlp_loss_grad")


def mlp_loss_grad_static(theta, X, t, grad, loss=None, n=None, idx=None, sym=None, stream=None) -> None:
    """mlp_loss_grad with the partial rows in the library's own scratch (the
    entry point that allocates nothing)."""
    rows = _rows(X)
    n = rows if n is None and idx is None else (int(idx.numel()) if n is None else int(n))
    _check(lib().ftc_mlp_loss_grad_static(_ptr(theta, torch.float32, MLP_PARAMS, "theta"),
                                          _ptr(X, torch.float32, rows * MLP_FEATURES, "X"), rows,
                                          _ptr(idx, torch.int32, n, "idx"), _ptr(sym, torch.int32, n, "sym"),
                                          _ptr(t, torch.float32, rows, "t"), n,
                                          _ptr(grad, torch.float32, MLP_PARAMS, "grad"),
                                          _ptr(loss, torch.float32, 1, "loss"), _stream(stream)),
           "ftc_mlp_loss_grad_static")


def mlp_adam(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             stream=None) -> None:
    _check(lib().ftc_mlp_adam(_ptr(theta, torch.float32, MLP_PARAMS, "theta"), _ptr(m, torch.float32, MLP_PARAMS, "m"),
                              _ptr(v, torch.float32, MLP_PARAMS, "v"), _ptr(grad, torch.float32, MLP_PARAMS, "grad"),
                              int(step), float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
           "ftc_mlp_adam")


def learned_curvature(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, alpha_dense, theta, bound: float, kappa,
                      nx, ny, nz, spread=None, cell_status=None, n_fallback=None, params: PPICParams | None = None,
                      stream=None) -> None:
    cg = c_grid(grid)
    cap = cells.cell_capacity
    p = None
    if params is not None:
        p = C.byref(_CParams(params.delta_over_h, params.rings, params.n_min, params.grow, params.max_iter,
                             params.precision))
    _check(lib().ftc_learned_curvature(cells.handle, C.byref(cg), C.byref(mesh.c),
                                       _ptr(alpha_dense, torch.float64, grid.ncell, "alpha_dense"),
                                       _ptr(theta, torch.float32, MLP_PARAMS, "theta"), float(bound), p,
                                       _ptr(kappa, torch.float64, cap, "kappa"), _ptr(nx, torch.float64, cap, "nx"),
                                       _ptr(ny, torch.float64, cap, "ny"), _ptr(nz, torch.float64, cap, "nz"),
                                       _ptr(spread, torch.float32, cap, "spread"),
                                       _ptr(cell_status, torch.int32, cap, "cell_status"),
                                       _ptr(n_fallback, torch.int32, 1, "n_fallback"), _stream(stream)),
           "ftc_learned_curvature")


# ------------------------------------------------------------------ roughness
def front_roughness(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, gl_mag, rough, stream=None) -> None:
    nv = mesh.c.nv
    _check(lib().ftc_front_roughness(cells.handle, C.byref(c_grid(grid)), C.byref(mesh.c),
                                     _ptr(gl_mag, torch.float64, nv, "gl_mag"), _ptr(rough, torch.float64, nv, "rough"),
                                     _stream(stream)), "ftc_front_roughness")


def smooth_rough_edges(cells: Cells, grid: _inputs.Grid, mesh: DeviceMesh, gl_mag, rough, gl_threshold: float,
                       rough_threshold: float, x_out, y_out, z_out, counts, max_rounds: int = 64, stream=None) -> None:
    nv = mesh.c.nv
    _check(lib().ftc_smooth_rough_edges(cells.handle, C.byref(c_grid(grid)), C.byref(mesh.c),
                                        _ptr(gl_mag, torch.float64, nv, "gl_mag"),
                                        _ptr(rough, torch.float64, nv, "rough"), float(gl_threshold),
                                        float(rough_threshold), int(max_rounds),
                                        _ptr(x_out, torch.float64, nv, "x_out"), _ptr(y_out, torch.float64, nv, "y_out"),
                                        _ptr(z_out, torch.float64, nv, "z_out"), _ptr(counts, torch.int32, 3, "counts"),
                                        _stream(stream)), "ftc_smooth_rough_edges")


# -------------------------------------------------------------------- tuning
def get_tuning(cells: Cells) -> Tuning:
    t = _CTuning()
    _check(lib().ftc_get_tuning(cells.handle, C.byref(t)), "ftc_get_tuning")
    return Tuning(t.ring_lanes, t.column_chunks, t.ring_blocks, t.queue_chunk)


def set_tuning(cells: Cells, tuning: Tuning) -> None:
    _check(lib().ftc_set_tuning(cells.handle, C.byref(_CTuning(tuning.ring_lanes, tuning.column_chunks,
                                                               tuning.ring_blocks, tuning.queue_chunk))),
           "ftc_set_tuning")

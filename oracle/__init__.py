"""ctypes front end of the FP64 CPU oracle (``oracle/ftc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The oracle shares no code with the HIP
library; it takes plain numpy arrays (host memory) built by the seeded input
generators.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libftc_oracle.so")
_lib = None

ORA_OK, ORA_EINVAL, ORA_EDOMAIN, ORA_EMESH, ORA_ECAPACITY = 0, -1, -2, -3, -4


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double), ("h", C.c_double)]


class _Mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("z", C.POINTER(C.c_double)),
                ("t0", C.POINTER(C.c_int32)), ("t1", C.POINTER(C.c_int32)),
                ("t2", C.POINTER(C.c_int32))]


class _Params(C.Structure):
    _fields_ = [("delta_over_h", C.c_double), ("rings", C.c_int32), ("n_min", C.c_int32),
                ("grow", C.c_double), ("max_iter", C.c_int32)]


@dataclass(frozen=True)
class PPICParams:
    """Volume-fit parameters (paper sec. 3.2): support radius 2.5 cells, the
    3-ring around the closest vertex, at least 24 weighted triangles, support
    grown by 10% per adjustment, at most 16 adjustments."""
    delta_over_h: float = 2.5
    rings: int = 3
    n_min: int = 24
    grow: float = 1.1
    max_iter: int = 16


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: F401  (oracle/build.py)
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    lib.ora_candidate_bound.argtypes = [P(_Grid), P(_Mesh)]
    lib.ora_candidate_bound.restype = C.c_int64
    lib.ora_cell_lists.argtypes = [P(_Grid), P(_Mesh), C.c_int64, P(C.c_int64), P(C.c_int32)]
    lib.ora_cell_lists.restype = C.c_int64
    lib.ora_volume_fraction.argtypes = [P(_Grid), P(_Mesh), C.c_int32, P(C.c_double), P(C.c_uint8)]
    lib.ora_volume_fraction.restype = C.c_int32
    lib.ora_piece.argtypes = [P(_Grid), P(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                              P(C.c_double)]
    lib.ora_piece.restype = C.c_int32
    lib.ora_ppic.argtypes = [P(_Grid), P(_Mesh), P(_Params), C.c_int64, P(C.c_int64),
                             P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_int32), P(C.c_int32)]
    lib.ora_ppic.restype = C.c_int32
    lib.ora_ppic_support.argtypes = [P(_Grid), P(_Mesh), P(_Params), C.c_int64, C.c_int32, P(C.c_int32),
                                     P(C.c_double), P(C.c_double), P(C.c_double)]
    lib.ora_ppic_support.restype = C.c_int32
    lib.ora_fit.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_int32, P(C.c_double),
                            P(C.c_double), P(C.c_double)]
    lib.ora_fit.restype = C.c_int32
    lib.ora_kappa.argtypes = [P(C.c_double)]
    lib.ora_kappa.restype = C.c_double
    lib.ora_frame_normal.argtypes = [P(_Grid), P(_Mesh), C.c_int64, P(C.c_int64), P(C.c_int32),
                                     P(C.c_double), P(C.c_double)]
    lib.ora_frame_normal.restype = C.c_int32
    lib.ora_csf.argtypes = [P(_Grid), P(C.c_double), C.c_int64, P(C.c_int64), P(C.c_double),
                            C.c_double, P(C.c_double)]
    lib.ora_csf.restype = C.c_int32
    lib.ora_csf_band.argtypes = [P(_Grid), P(C.c_double), C.c_int64, P(C.c_int64), P(C.c_double),
                                 P(C.c_double), C.c_double, C.c_int64, P(C.c_int64), P(C.c_double),
                                 P(C.c_double)]
    lib.ora_csf_band.restype = C.c_int64
    lib.ora_advect_rk4.argtypes = [P(_Grid), C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double),
                                   P(C.c_double), P(C.c_double), P(C.c_double), C.c_double, P(C.c_double)]
    lib.ora_advect_rk4.restype = C.c_int32
    lib.ora_interp.argtypes = [P(_Grid), C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double),
                               P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)]
    lib.ora_interp.restype = C.c_int32
    lib.ora_interp_in_cell.argtypes = [P(_Grid), C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                       C.c_double, C.c_double, P(C.c_double), P(C.c_double),
                                       P(C.c_double), P(C.c_double)]
    lib.ora_interp_in_cell.restype = None
    lib.ora_threads.argtypes = []
    lib.ora_threads.restype = C.c_int32
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self, grid, mesh=None):
        self.g = _Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0, grid.h)
        self.m = None
        if mesh is not None:
            self.arrs = [_f64(mesh.x), _f64(mesh.y), _f64(mesh.z), _i32(mesh.t0), _i32(mesh.t1),
                         _i32(mesh.t2)]
            x, y, z, t0, t1, t2 = self.arrs
            self.m = _Mesh(len(x), len(t0), _dp(x), _dp(y), _dp(z), _ip(t0), _ip(t1), _ip(t2))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def threads() -> int:
    return int(_load().ora_threads())


def set_threads(n: int) -> None:
    """Threads of the following oracle calls (n <= 0: one per processor)."""
    lib = _load()
    lib.ora_set_threads.argtypes = [C.c_int32]
    lib.ora_set_threads.restype = None
    lib.ora_set_threads(int(n))


def candidate_bound(grid, mesh) -> int:
    k = _Keep(grid, mesh)
    return int(_load().ora_candidate_bound(C.byref(k.g), C.byref(k.m)))


def cell_lists(grid, mesh):
    """(cell_ids, offsets, tri_ids): the interfacial cells in ascending linear
    id and, for each, its triangles in ascending id (CSR)."""
    lib = _load()
    k = _Keep(grid, mesh)
    cap = int(lib.ora_candidate_bound(C.byref(k.g), C.byref(k.m)))
    if cap < 0:
        raise OracleError(cap, "cell_lists")
    pc = np.empty(max(cap, 1), np.int64)
    pt = np.empty(max(cap, 1), np.int32)
    n = int(lib.ora_cell_lists(C.byref(k.g), C.byref(k.m), cap, _lp(pc), _ip(pt)))
    if n < 0:
        raise OracleError(n, "cell_lists")
    pc, pt = pc[:n], pt[:n]
    cells, starts = np.unique(pc, return_index=True)
    offsets = np.append(starts, n).astype(np.int64)
    return cells.astype(np.int64), offsets, pt.copy()


def volume_fraction(grid, mesh, axis: int = 2):
    """(alpha, is_interfacial) for every cell, shape (nz, ny, nx)."""
    lib = _load()
    k = _Keep(grid, mesh)
    alpha = np.empty(grid.ncell, np.float64)
    isif = np.empty(grid.ncell, np.uint8)
    st = int(lib.ora_volume_fraction(C.byref(k.g), C.byref(k.m), axis, _dp(alpha),
                                     isif.ctypes.data_as(C.POINTER(C.c_uint8))))
    if st != 0:
        raise OracleError(st, "volume_fraction")
    shp = (grid.nz, grid.ny, grid.nx)
    return alpha.reshape(shp), isif.reshape(shp).astype(bool)


def piece(grid, tri, ijk, axis: int = 2):
    """(counts, flux, vol) of one triangle clipped to cell ijk."""
    out = np.zeros(2)
    k = _Keep(grid)
    t = _f64(np.asarray(tri).reshape(9))
    r = int(_load().ora_piece(C.byref(k.g), _dp(t), int(ijk[0]), int(ijk[1]), int(ijk[2]), axis,
                              _dp(out)))
    return bool(r), float(out[0]), float(out[1])


def ppic(grid, mesh, cell_ids, params: PPICParams = PPICParams()):
    """Per listed cell: dict(kappa, normal[n,3], coeff[n,6], status, diag[n,4])."""
    lib = _load()
    k = _Keep(grid, mesh)
    ids = np.ascontiguousarray(cell_ids, dtype=np.int64)
    n = len(ids)
    kap = np.empty(n)
    nrm = np.empty((n, 3))
    co = np.empty((n, 6))
    st = np.empty(n, np.int32)
    dg = np.empty((n, 4), np.int32)
    p = _Params(params.delta_over_h, params.rings, params.n_min, params.grow, params.max_iter)
    r = int(lib.ora_ppic(C.byref(k.g), C.byref(k.m), C.byref(p), n, _lp(ids), _dp(kap), _dp(nrm),
                         _dp(co), _ip(st), _ip(dg)))
    if r != 0:
        raise OracleError(r, "ppic")
    return dict(kappa=kap, normal=nrm, coeff=co, status=st, diag=dg)


def ppic_support(grid, mesh, cell_id, params: PPICParams = PPICParams()):
    """The support of one cell's volume fit, as ppic computes it: dict(tri
    [ring triangles, ascending], d2 [squared centre distances], w [Wendland
    weights], delta [support radius])."""
    k = _Keep(grid, mesh)
    p = _Params(params.delta_over_h, params.rings, params.n_min, params.grow, params.max_iter)
    cap = mesh.nt
    tri = np.empty(cap, np.int32)
    d2 = np.empty(cap)
    w = np.empty(cap)
    delta = np.empty(1)
    n = int(_load().ora_ppic_support(C.byref(k.g), C.byref(k.m), C.byref(p), int(cell_id), cap, _ip(tri),
                                     _dp(d2), _dp(w), _dp(delta)))
    if n < 0:
        raise OracleError(n, "ppic_support")
    return dict(tri=tri[:n].copy(), d2=d2[:n].copy(), w=w[:n].copy(), delta=float(delta[0]))


def frame_normal(grid, mesh, cell_ids):
    """Per listed cell: (closest vertex, its squared distance to the cell
    centre, that vertex's area-weighted normal [n, 3])."""
    k = _Keep(grid, mesh)
    ids = np.ascontiguousarray(cell_ids, dtype=np.int64)
    n = len(ids)
    vs = np.empty(n, np.int32)
    d2 = np.empty(n)
    nrm = np.empty((n, 3))
    r = int(_load().ora_frame_normal(C.byref(k.g), C.byref(k.m), n, _lp(ids), _ip(vs), _dp(d2), _dp(nrm)))
    if r != 0:
        raise OracleError(r, "frame_normal")
    return vs, d2, nrm


def fit(frame, xc, h, tris, w):
    """One volume fit: frame rows (t1, t2, n), origin xc, triangles
    [ntri, 3, 3] in world coordinates, weights [ntri] -> (a[6], status)."""
    fr = _f64(np.asarray(frame).reshape(9))
    x = _f64(np.asarray(xc).reshape(3))
    t = _f64(np.asarray(tris).reshape(-1))
    ww = _f64(w)
    a = np.empty(6)
    st = int(_load().ora_fit(_dp(fr), _dp(x), float(h), len(ww), _dp(t), _dp(ww), _dp(a)))
    return a, st


def kappa_of(a) -> float:
    aa = _f64(a)
    return float(_load().ora_kappa(_dp(aa)))


def csf(grid, alpha, cell_ids, kappa, sigma: float):
    lib = _load()
    k = _Keep(grid)
    al = _f64(alpha).reshape(-1)
    ids = np.ascontiguousarray(cell_ids, dtype=np.int64)
    kp = _f64(kappa)
    f = np.empty((len(ids), 3))
    r = int(lib.ora_csf(C.byref(k.g), _dp(al), len(ids), _lp(ids), _dp(kp), float(sigma), _dp(f)))
    if r != 0:
        raise OracleError(r, "csf")
    return f


def csf_band(grid, alpha, cell_ids, kappa, normal, sigma: float):
    """BAND mode: (band_ids, kappa_bar, force[n,3]) for the face neighbours of
    the interfacial cells that are not interfacial themselves."""
    lib = _load()
    k = _Keep(grid)
    al = _f64(alpha).reshape(-1)
    ids = np.ascontiguousarray(cell_ids, dtype=np.int64)
    kp = _f64(kappa)
    nr = np.ascontiguousarray(normal, dtype=np.float64).reshape(-1)
    cap = 6 * len(ids)
    bid = np.empty(cap, np.int64)
    kb = np.empty(cap)
    f = np.empty((cap, 3))
    n = int(lib.ora_csf_band(C.byref(k.g), _dp(al), len(ids), _lp(ids), _dp(kp), _dp(nr), float(sigma), cap,
                             _lp(bid), _dp(kb), _dp(f)))
    if n < 0:
        raise OracleError(n, "csf_band")
    return bid[:n], kb[:n], f[:n]


def interp(grid, x, y, z, U, V, W):
    lib = _load()
    k = _Keep(grid)
    x, y, z = _f64(x), _f64(y), _f64(z)
    U, V, W = _f64(U).reshape(-1), _f64(V).reshape(-1), _f64(W).reshape(-1)
    u = np.empty((len(x), 3))
    r = int(lib.ora_interp(C.byref(k.g), len(x), _dp(x), _dp(y), _dp(z), _dp(U), _dp(V), _dp(W),
                           _dp(u)))
    if r != 0:
        raise OracleError(r, "interp")
    return u


def advect_rk4(grid, x, y, z, U, V, W, dt: float, check: bool = True):
    """One RK4 step of the points through the interpolated field: new
    positions [n, 3] (NaN where a stage point left the grid)."""
    lib = _load()
    k = _Keep(grid)
    x, y, z = _f64(x), _f64(y), _f64(z)
    U, V, W = _f64(U).reshape(-1), _f64(V).reshape(-1), _f64(W).reshape(-1)
    out = np.empty((len(x), 3))
    r = int(lib.ora_advect_rk4(C.byref(k.g), len(x), _dp(x), _dp(y), _dp(z), _dp(U), _dp(V), _dp(W), float(dt),
                               _dp(out)))
    if r != 0 and check:
        raise OracleError(r, "advect_rk4")
    return out


def interp_in_cell(grid, ijk, p, U, V, W):
    k = _Keep(grid)
    U, V, W = _f64(U).reshape(-1), _f64(V).reshape(-1), _f64(W).reshape(-1)
    out = np.empty(3)
    _load().ora_interp_in_cell(C.byref(k.g), int(ijk[0]), int(ijk[1]), int(ijk[2]), float(p[0]),
                               float(p[1]), float(p[2]), _dp(U), _dp(V), _dp(W), _dp(out))
    return out

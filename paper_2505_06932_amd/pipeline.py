"""One coupling step over device-resident inputs: the five library calls in
order (cell lists, volume fraction, PPIC curvature, CSF, vertex velocities),
with every output allocated once so that a step allocates nothing and can be
captured into a HIP graph."""
from __future__ import annotations

import numpy as np
import torch

from . import ftc
from . import inputs as I


class CouplingStep:
    def __init__(self, grid: I.Grid, mesh: I.Mesh, U=None, V=None, W=None, sigma: float = 1.0,
                 params: ftc.PPICParams | None = None, margin: float = 1.25,
                 pair_capacity: int | None = None, cell_capacity: int | None = None, band: bool = False,
                 learned=None, bound: float | None = None, tuning: ftc.Tuning | None = None,
                 densities: tuple[float, float] | None = None):
        """learned: surrogate parameters (device float32 tensor of
        ftc.MLP_PARAMS values); the curvature is then the learned surrogate
        with its PPIC fallback above the spread `bound`.  densities: (rho_a,
        rho_b) adds the surface-tension part of the face flux of every
        interfacial and band cell (needs band=True)."""
        if densities is not None and not band:
            raise ValueError("the face flux needs the band (band=True)")
        self.grid = grid
        self.sigma = float(sigma)
        self.params = params
        self.mesh = ftc.DeviceMesh.from_host(mesh)
        dev = "cuda"
        if U is None:
            U, V, W = I.uniform_face_velocity(grid, (0.0, 0.0, 0.0))
        f64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        self.U, self.V, self.W = f64(U).reshape(-1), f64(V).reshape(-1), f64(W).reshape(-1)
        nv, nt = mesh.nv, mesh.nt
        if pair_capacity is None or cell_capacity is None:
            # size the workspace from probing builds, doubling the capacities
            # while they overflow
            pc, cc = 8 * nt + 4096, int(min(grid.ncell, 4 * nt + 4096))
            for _ in range(12):
                probe = ftc.Cells(grid, nv, nt, pc, cc)
                ftc.build_cell_lists(probe, grid, self.mesh)
                n_if, n_p = probe.count()
                err = probe.last_device_error()
                probe.close()
                if err != ftc.FTC_ECAPACITY:
                    break
                pc, cc = 2 * pc, int(min(grid.ncell, 2 * cc))
            if err != ftc.FTC_OK:
                raise ftc.FTCError(err, "probing build")
            pair_capacity = pair_capacity or int(n_p * margin) + 256
            cell_capacity = cell_capacity or int(min(grid.ncell, n_if * margin + 256))
        self.cells = ftc.Cells(grid, nv, nt, pair_capacity, cell_capacity)
        if tuning is not None:
            ftc.set_tuning(self.cells, tuning)
        cap = self.cells.cell_capacity
        z = lambda n, dt=torch.float64: torch.zeros(n, dtype=dt, device=dev)
        self.alpha_if = z(cap)
        self.alpha = z(grid.ncell)
        self.kappa, self.nx, self.ny, self.nz = z(cap), z(cap), z(cap), z(cap)
        self.coeff = z(6 * cap)
        self.status = z(cap, torch.int32)
        self.diag = z(4 * cap, torch.int32)
        self.fx, self.fy, self.fz = z(cap), z(cap), z(cap)
        self.ux, self.uy, self.uz = z(nv), z(nv), z(nv)
        self.band = band
        self.learned = learned
        if learned is not None:
            from . import surrogate
            self.bound = surrogate.DEFAULT_BOUND if bound is None else float(bound)
            self.spread = z(cap, torch.float32)
            self.n_fallback = z(1, torch.int32)
        if band:
            # every band cell is a face neighbour of an interfacial cell
            bcap = 6 * cap
            self.band_ids = z(bcap, torch.int32)
            self.kappa_band = z(bcap)
            self.bx, self.by, self.bz = z(bcap), z(bcap), z(bcap)
            self.n_band = z(1, torch.int32)
        self.densities = densities
        if densities is not None:
            self.flux_if, self.flux_band = z(6 * cap), z(6 * bcap)

    # the hot path, split so that callers can time its parts
    def cells_and_alpha(self, stream=None):
        ftc.build_cell_lists(self.cells, self.grid, self.mesh, stream)
        ftc.volume_fraction(self.cells, self.grid, self.mesh, self.alpha_if, self.alpha, stream)

    def curvature(self, stream=None, diagnostics=True):
        if self.learned is not None:
            ftc.learned_curvature(self.cells, self.grid, self.mesh, self.alpha, self.learned, self.bound, self.kappa,
                                  self.nx, self.ny, self.nz, spread=self.spread, cell_status=self.status,
                                  n_fallback=self.n_fallback, params=self.params, stream=stream)
            return
        ftc.ppic_curvature(self.cells, self.grid, self.mesh, self.kappa, self.nx, self.ny, self.nz,
                           self.coeff if diagnostics else None, self.status,
                           self.diag if diagnostics else None, self.params, stream)

    def forces_and_velocities(self, stream=None):
        ftc.csf_force(self.cells, self.grid, self.alpha, self.kappa, self.sigma, self.fx, self.fy, self.fz,
                      stream)
        if self.band:
            ftc.csf_force_band(self.cells, self.grid, self.alpha, self.kappa, self.nx, self.ny, self.nz, self.sigma,
                               self.band_ids, self.kappa_band, self.bx, self.by, self.bz, self.n_band, stream)
        if self.densities is not None:
            ftc.surface_tension_flux(self.cells, self.grid, self.alpha, self.kappa, self.band_ids, self.kappa_band,
                                     self.n_band, self.densities[0], self.densities[1], self.sigma, self.flux_if,
                                     self.flux_band, stream)
        ftc.interp_vertex_velocity(self.cells, self.grid, self.mesh, self.U, self.V, self.W, self.ux,
                                   self.uy, self.uz, stream)

    def run(self, stream=None, diagnostics=True):
        self.cells_and_alpha(stream)
        self.curvature(stream, diagnostics)
        self.forces_and_velocities(stream)

    def results(self):
        """Host copies of every output, trimmed to the live counts."""
        torch.cuda.synchronize()
        n_if, n_p = self.cells.count()
        cap = self.cells.cell_capacity
        cell_ids, offsets, tri_ids = self.cells.lists()
        h = lambda t: t.detach().cpu().numpy()
        return dict(
            n_if=n_if, n_pairs=n_p, cell_ids=h(cell_ids).astype(np.int64), offsets=h(offsets).astype(np.int64),
            tri_ids=h(tri_ids), alpha_if=h(self.alpha_if)[:n_if],
            alpha=h(self.alpha).reshape(self.grid.nz, self.grid.ny, self.grid.nx),
            kappa=h(self.kappa)[:n_if],
            normal=np.stack([h(self.nx)[:n_if], h(self.ny)[:n_if], h(self.nz)[:n_if]], 1),
            coeff=h(self.coeff).reshape(6, cap)[:, :n_if].T, status=h(self.status)[:n_if],
            diag=h(self.diag).reshape(4, cap)[:, :n_if].T,
            force=np.stack([h(self.fx)[:n_if], h(self.fy)[:n_if], h(self.fz)[:n_if]], 1),
            u=np.stack([h(self.ux), h(self.uy), h(self.uz)], 1),
            **(self._band_results(h) if self.band else {}),
            **(dict(spread=h(self.spread)[:n_if], n_fallback=int(h(self.n_fallback)[0]))
               if self.learned is not None else {}),
            error=self.cells.last_device_error())

    def _band_results(self, h):
        nb = int(h(self.n_band)[0])
        nb = min(nb, self.band_ids.numel())
        out = dict(n_band=nb, band_ids=h(self.band_ids)[:nb].astype(np.int64), kappa_band=h(self.kappa_band)[:nb],
                   band_force=np.stack([h(self.bx)[:nb], h(self.by)[:nb], h(self.bz)[:nb]], 1))
        if self.densities is not None:
            n_if = self.cells.count()[0]
            out["flux_if"] = h(self.flux_if).reshape(6, -1)[:, :n_if].T
            out["flux_band"] = h(self.flux_band).reshape(6, -1)[:, :nb].T
        return out

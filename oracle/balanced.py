"""Surface-tension part of the face flux of the momentum-weighted interpolation
(paper section 3.3, Eq. mwi_disc): the plain CPU definition the GPU kernel is
checked against.  Test infrastructure only.

For a face f between cells P (lower) and Q (upper) along axis d, n_f = +e_d,
the surface-tension term of F_f divided by the solver's coefficients
d_f A_f is

    Phi_f = sigma [ kbar_f (alpha_Q - alpha_P) / h
                    - rho*_f / 2 (k_P g_P / rho_P + k_Q g_Q / rho_Q) ],

with
  * rho_C = rho_a + alpha_C (rho_b - rho_a), the mixture density of the
    indicator (sec. 2), and rho*_f = 2 rho_P rho_Q / (rho_P + rho_Q), the
    harmonic face density (sec. 2);
  * g_C = (alpha[C + e_d] - alpha[C - e_d]) / (2 h), the d-component of the
    central-difference gradient the CSF source uses (Eq. csf);
  * k_C the curvature the CSF source uses in C: the PPIC curvature of an
    interfacial cell, the weighted average kbar of a band cell (a face
    neighbour of an interfacial cell that is not interfacial itself,
    Eq. for kbar_P), and 0 in every other cell, which carries no surface
    force;
  * kbar_f the mean of k_P and k_Q over those of the two cells that carry a
    curvature (interfacial or band), 0 if neither does.

Readings (the paper names kbar_f without defining it): the face curvature is
the arithmetic mean of the two cell curvatures, and a cell outside the band
contributes neither a curvature nor a source.  With a constant curvature and
p = sigma k alpha the term equals the pressure term of the same flux exactly,
which is the force balance the paper claims for this discretisation.

Output layout: per listed cell C (the interfacial cells in ascending linear
id, then the band cells in ascending linear id) the values of its six faces,
slot 2d for the face towards C - e_d (P = C - e_d, Q = C) and slot 2d + 1
for the face towards C + e_d (P = C, Q = C + e_d).
"""
from __future__ import annotations

import numpy as np


def surface_tension_face_flux(grid, alpha, cell_ids, kappa, band_ids, kappa_band, rho_a, rho_b, sigma):
    """(flux of the interfacial cells [n_if, 6], flux of the band cells [n_band, 6])."""
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    a = np.asarray(alpha, dtype=np.float64).reshape(-1)
    stride = (1, nx, nx * ny)
    curv = {}
    for lin, k in zip(np.asarray(cell_ids).tolist(), np.asarray(kappa, dtype=np.float64).tolist()):
        curv[int(lin)] = k
    for lin, k in zip(np.asarray(band_ids).tolist(), np.asarray(kappa_band, dtype=np.float64).tolist()):
        curv[int(lin)] = k

    def rho(c):
        return rho_a + a[c] * (rho_b - rho_a)

    def source_part(c, d):
        """k_C g_C / rho_C along d, 0 outside the band."""
        if c not in curv:
            return 0.0
        g = (a[c + stride[d]] - a[c - stride[d]]) / (2.0 * h)
        return curv[c] * g / rho(c)

    def face(p, q, d):
        ks = [curv[c] for c in (p, q) if c in curv]
        kf = sum(ks) / len(ks) if ks else 0.0
        rp, rq = rho(p), rho(q)
        rs = 2.0 * rp * rq / (rp + rq)
        return sigma * (kf * (a[q] - a[p]) / h - 0.5 * rs * (source_part(p, d) + source_part(q, d)))

    def rows(ids):
        out = np.empty((len(ids), 6))
        for r, c in enumerate(np.asarray(ids).tolist()):
            c = int(c)
            for d in range(3):
                out[r, 2 * d] = face(c - stride[d], c, d)
                out[r, 2 * d + 1] = face(c, c + stride[d], d)
        return out

    return rows(cell_ids), rows(band_ids)


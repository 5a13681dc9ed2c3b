"""FP64 reference of the Fourier's-law heat spreading outside the phonon
Monte Carlo domain (coupling paragraph of Hao, Zhao, Xiao and Kronenfeld,
arXiv:1707.09073): steady conduction, cell-centred finite volumes on a
tensor-product grid, the GaN-substrate interface resistance of Eq. (3) on
one plane, and conductivities whose bulk mean free paths are limited by the
structure size (the wire's diameter, the film's thickness).

TEST INFRASTRUCTURE ONLY: used by the tests; the GPU product path never
imports it.  The linear system is assembled from its definition with
scipy.sparse and solved directly (no iteration).

Definitions (both sides): cells (i, j, k), index (i*ny + j)*nz + k, widths
d from the edge coordinates.  Between neighbours c, c' across a face of
area A the conductance is A / (d_c/(2 kappa_c) + d_c'/(2 kappa_c') [+ R_K
on the interface plane]), zero if either conductivity is zero (void).  A
Dirichlet face holds the rise at zero with conductance A / (d/(2 kappa)).
The rise u = T - T_sink solves sum_faces G (u_c - u_nb) = q_c; a void cell
takes u = 0.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse
from scipy.sparse import linalg as spla

from oracle import phonon_oracle as P


def assemble(n, dirichlet, k_interface, R_K, edges, kappa, q):
    """The sparse matrix and right-hand side of the rise."""
    nx, ny, nz = (int(v) for v in n)
    ex, ey, ez = (np.asarray(e, np.float64) for e in edges)
    dx, dy, dz = np.diff(ex), np.diff(ey), np.diff(ez)
    kap = np.asarray(kappa, np.float64).reshape(nx, ny, nz)
    nc = nx * ny * nz
    idx = np.arange(nc).reshape(nx, ny, nz)
    rows, cols, vals = [], [], []
    diag = np.zeros((nx, ny, nz))

    def couple(a_idx, b_idx, G):
        # symmetric off-diagonal pair and the diagonal contributions
        rows.extend([a_idx.ravel(), b_idx.ravel()])
        cols.extend([b_idx.ravel(), a_idx.ravel()])
        vals.extend([-G.ravel(), -G.ravel()])

    def face_G(k1, k2, d1, d2, area, extra=0.0):
        with np.errstate(divide="ignore", invalid="ignore"):
            G = area / (d1 / (2.0 * k1) + d2 / (2.0 * k2) + extra)
        return np.where((k1 > 0) & (k2 > 0), G, 0.0)

    # x faces
    A = (dy[:, None] * dz[None, :])[None, :, :]
    G = face_G(kap[:-1], kap[1:], dx[:-1, None, None], dx[1:, None, None], A)
    couple(idx[:-1], idx[1:], G)
    diag[:-1] += G
    diag[1:] += G
    # y faces
    A = (dx[:, None] * dz[None, :])[:, None, :]
    G = face_G(kap[:, :-1], kap[:, 1:], dy[None, :-1, None], dy[None, 1:, None], A)
    couple(idx[:, :-1], idx[:, 1:], G)
    diag[:, :-1] += G
    diag[:, 1:] += G
    # z faces (the interface plane carries R_K)
    A = (dx[:, None] * dy[None, :])[:, :, None]
    extra = np.zeros(nz - 1)
    if 0 < k_interface < nz:
        extra[k_interface - 1] = R_K
    G = face_G(kap[:, :, :-1], kap[:, :, 1:], dz[None, None, :-1], dz[None, None, 1:], A * np.ones((1, 1, nz - 1)),
               extra[None, None, :])
    couple(idx[:, :, :-1], idx[:, :, 1:], G)
    diag[:, :, :-1] += G
    diag[:, :, 1:] += G
    # Dirichlet faces: half a cell from the centre to the face
    for f, held in enumerate(dirichlet):
        if not held:
            continue
        ax, hi = f // 2, f % 2
        sl = [slice(None)] * 3
        sl[ax] = -1 if hi else 0
        sl = tuple(sl)
        d = (dx, dy, dz)[ax][-1 if hi else 0]
        area = {0: dy[:, None] * dz[None, :], 1: dx[:, None] * dz[None, :], 2: dx[:, None] * dy[None, :]}[ax]
        k = kap[sl]
        with np.errstate(divide="ignore"):
            Gb = np.where(k > 0, area / (d / (2.0 * np.where(k > 0, k, 1.0))), 0.0)
        diag[sl] += Gb
    void = kap <= 0
    diag = np.where(void, 1.0, diag)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    M = sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nc, nc))
    b = np.where(void.ravel(), 0.0, np.asarray(q, np.float64).ravel())
    return M, b


def solve(cfg: dict, edges, kappa, q) -> np.ndarray:
    """Temperature per cell (K): cfg has n, dirichlet (six flags), k_interface,
    R_K_m2KW, T_sink_K."""
    M, b = assemble(cfg["n"], cfg["dirichlet"], cfg.get("k_interface", -1), cfg.get("R_K_m2KW", 0.0), edges, kappa, q)
    u = spla.spsolve(M.tocsc(), b, permc_spec="MMD_AT_PLUS_A")   # a fill-reducing order for symmetric structure
    return cfg["T_sink_K"] + u


def boundary_flux(cfg: dict, edges, kappa, T) -> float:
    """Heat leaving through the Dirichlet faces (W)."""
    nx, ny, nz = cfg["n"]
    ex, ey, ez = (np.asarray(e, np.float64) for e in edges)
    dx, dy, dz = np.diff(ex), np.diff(ey), np.diff(ez)
    kap = np.asarray(kappa, np.float64).reshape(nx, ny, nz)
    u = (np.asarray(T) - cfg["T_sink_K"]).reshape(nx, ny, nz)
    out = 0.0
    for f, held in enumerate(cfg["dirichlet"]):
        if not held:
            continue
        ax, hi = f // 2, f % 2
        sl = [slice(None)] * 3
        sl[ax] = -1 if hi else 0
        sl = tuple(sl)
        d = (dx, dy, dz)[ax][-1 if hi else 0]
        area = {0: dy[:, None] * dz[None, :], 1: dx[:, None] * dz[None, :], 2: dx[:, None] * dy[None, :]}[ax]
        k = kap[sl]
        Gb = np.where(k > 0, area * 2.0 * np.where(k > 0, k, 1.0) / d, 0.0)
        out += float((Gb * u[sl]).sum())
    return out


def size_limited_kappa(m: dict, T: float, d_m: float, electrons=None) -> float:
    """Conductivity (W/m/K) with the bulk mean free paths limited by a
    structure size d (Matthiessen's rule, 1/tau + v/d), by quadrature;
    d <= 0 gives the bulk value."""
    ef = None
    if electrons:
        ef = P.fermi_level(electrons["n_m3"], electrons["m_dos"], T)

    def extra(w):
        e = 0.0
        if electrons:
            e += float(P.inv_tau_electron(w, T, ef, electrons["m_dos"], electrons["D_a_eV"], electrons["rho"],
                                          electrons["v_g"]))
        if d_m > 0:
            e += float(P.vg_of_w(m, w)) / d_m
        return e

    return P.kappa(m, T, extra_inv_tau=extra)

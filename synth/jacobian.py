"""Seeded synthetic Jacobians of a thermal CO2-brine system with 3x3 blocks.

This module only builds inputs.  It holds none of the preconditioner's or the
Krylov solver's arithmetic, and both the CPU oracle and the GPU library read
what it writes.

The paper's test cases are reservoir models that are not available here; the
Jacobians below stand in for them.  They follow the structure of the mass
conservation equation (Eq. 1) and the energy conservation equation (Eq. 2):
accumulation, upwinded advection of mass, CO2 and enthalpy, and heat
conduction, discretised with two-point flux approximation (TPFA) on a
Cartesian grid.  After the exact local elimination the paper performs before
building CPTR (Sec. 3.4), three unknowns per cell remain; here they are
(p, T, z_CO2) with equations (total mass, energy, CO2 mass), interleaved per
cell (Sec. 3.1 notes the variables are interleaved), so that p and T form the
elliptic pair and z the hyperbolic unknown (Sec. 3.2).

The thermal Peclet number of Eq. (4) is the knob used to sweep the thermal
regime (Sec. 5.3): it is measured per face and the conductivity is rescaled
to reach a target value.

Output: block-CSR (BSR) arrays with block size 3, blocks row-major, sorted
column indices, the diagonal block present in every row.
"""
from __future__ import annotations

import dataclasses
import json
import math

import numpy as np

BLOCK = 3
SEED_BASE = 11892

# Physical constants of the synthetic state (recorded in meta).
DX, DY, DZ = 10.0, 10.0, 2.0          # m
PORO = 0.2
CT = 1e-9                             # 1/Pa
MU_C = 5e-5                           # Pa s, CO2-rich phase
CF = 4.0e6                            # J/m^3/K, fluid volumetric heat capacity
CR = 2.5e6                            # J/m^3/K, rock
KAPPA0 = 2.0                          # W/m/K
DT = 86400.0                          # s
T_RES = 343.15                        # K (70 C)
DT_INJ = 30.0                         # K: injected at 40 C
P0 = 20e6                             # Pa
DP_WELL = 2e6                         # Pa
R_WELL = 0.5                          # cells
P_SCALE = 1e6                         # pressure column unit: MPa
K_REF = 1e-13                         # m^2, reference medium of the flow state
LAM_REF = 1.0 / 5e-4                  # 1/(Pa s), brine mobility at reservoir T


@dataclasses.dataclass
class Case:
    """One synthetic linear system (a Newton-step Jacobian and a right-hand side)."""
    name: str
    nx: int
    ny: int
    nz: int
    row_ptr: np.ndarray    # int32 [n+1]
    col_idx: np.ndarray    # int32 [nnzb]
    values: np.ndarray     # float64 [nnzb, 3, 3]
    b: np.ndarray          # float64 [3n]
    x_star: np.ndarray     # float64 [3n], b = A x_star
    tol: float
    meta: dict

    @property
    def n_cells(self) -> int:
        return self.row_ptr.shape[0] - 1

    @property
    def n_dof(self) -> int:
        return BLOCK * self.n_cells

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.bsr_matrix((self.values, self.col_idx, self.row_ptr),
                             shape=(self.n_dof, self.n_dof))


def _gauss_field(rng, shape, corr_cells):
    g = rng.standard_normal(shape)
    if corr_cells and corr_cells > 0:
        from scipy.ndimage import gaussian_filter
        # shape is (nz, ny, nx); filter isotropically in cell units
        g = gaussian_filter(g, sigma=corr_cells, mode="wrap")
        g = (g - g.mean()) / max(g.std(), 1e-300)
    return g


def _wells(nx, ny, n_wells):
    if n_wells == 1:
        return [(0, 0)]
    if n_wells == 4:
        return [(nx // 4, ny // 4), (3 * nx // 4, ny // 4),
                (nx // 4, 3 * ny // 4), (3 * nx // 4, 3 * ny // 4)]
    raise ValueError("n_wells must be 1 or 4")


def _mobility(z, T):
    inv_mw = np.exp(-0.02 * (T_RES - T)) / 5e-4
    lam = (1.0 - z) * inv_mw + z / MU_C
    dlam_dT = (1.0 - z) * inv_mw * 0.02
    dlam_dz = 1.0 / MU_C - inv_mw
    return lam, dlam_dT, dlam_dz


def _radial_p(ii, jj, wells, R):
    """Superposed radial pressure of the injectors at cell coordinates (ii, jj)."""
    p = np.full(np.broadcast(ii, jj).shape, P0)
    for (iw, jw) in wells:
        r = np.sqrt((ii - iw) ** 2 + (jj - jw) ** 2)
        p = p + DP_WELL * np.log(R / np.maximum(R_WELL, r)) / math.log(R / R_WELL)
    return p


def _state(nx, ny, nz, wells, r_front):
    i = np.arange(nx, dtype=np.float64)[None, None, :]
    j = np.arange(ny, dtype=np.float64)[None, :, None]
    R = math.hypot(nx, ny)
    p = np.broadcast_to(_radial_p(i, j, wells, R), (nz, ny, nx))
    dmin = np.full((1, ny, nx), np.inf)
    for (iw, jw) in wells:
        dmin = np.minimum(dmin, np.sqrt((i - iw) ** 2 + (j - jw) ** 2))
    dmin = np.broadcast_to(dmin, (nz, ny, nx))
    T = T_RES - DT_INJ * 0.5 * (1.0 - np.tanh(dmin - r_front))
    z = 0.5 * (1.0 - np.tanh(dmin - 2.0 * r_front))
    return p, T, z


def _faces(nx, ny, nz):
    """Yield (direction, left cell ids, right cell ids, area, distance)."""
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    out = []
    if nx > 1:
        out.append((0, idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel(), DY * DZ, DX))
    if ny > 1:
        out.append((1, idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel(), DX * DZ, DY))
    if nz > 1:
        out.append((2, idx[:-1, :, :].ravel(), idx[1:, :, :].ravel(), DX * DY, DZ))
    return out


def _face_fluxes(p, faces):
    """Volumetric face fluxes of the linearisation state.

    They come from the superposed radial flow of the injectors through the
    reference medium (K_REF, LAM_REF), so the flux field is conservative away
    from the wells, as the converged Newton state of a simulator would be;
    the heterogeneity enters the Jacobian through the transmissibilities and
    the Darcy-consistent face pressure differences dp_f = F_f / (T_f lam_u)."""
    res = []
    for (d, a, b, area, dist) in faces:
        res.append((area / dist) * K_REF * LAM_REF * (p[a] - p[b]))
    return res


def peclet(fluxes, faces, kappa):
    """Median over faces with nonzero flux of |F| C_f d / (kappa A)  (Eq. 4, per face)."""
    vals = []
    for F, (d, a, b, area, dist) in zip(fluxes, faces):
        nz_ = F != 0
        area_ = np.broadcast_to(area, F.shape)[nz_]
        dist_ = np.broadcast_to(dist, F.shape)[nz_]
        vals.append(np.abs(F[nz_]) * CF * dist_ / (kappa * area_))
    v = np.concatenate(vals) if vals else np.zeros(0)
    return float(np.median(v)) if v.size else 0.0


def _boundary_outflow(nx, ny, nz, wells):
    """Open lateral boundaries: (cell ids, outward flux > 0) of the radial flow
    leaving the domain through its x and y boundary faces."""
    R = math.hypot(nx, ny)
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    cells, flux = [], []
    jj = np.arange(ny, dtype=np.float64)
    ii = np.arange(nx, dtype=np.float64)
    sides = [
        (idx[:, :, 0], _radial_p(0.0, jj, wells, R) - _radial_p(-1.0, jj, wells, R), DY * DZ / DX),
        (idx[:, :, nx - 1], _radial_p(nx - 1.0, jj, wells, R) - _radial_p(float(nx), jj, wells, R), DY * DZ / DX),
        (idx[:, 0, :], _radial_p(ii, 0.0, wells, R) - _radial_p(ii, -1.0, wells, R), DX * DZ / DY),
        (idx[:, ny - 1, :], _radial_p(ii, ny - 1.0, wells, R) - _radial_p(ii, float(ny), wells, R), DX * DZ / DY),
    ]
    for cell_ids, dp, geo in sides:
        F = np.broadcast_to(geo * K_REF * LAM_REF * dp, cell_ids.shape)
        cells.append(cell_ids.ravel())
        flux.append(np.maximum(F, 0.0).ravel())
    return np.concatenate(cells), np.concatenate(flux)


def _face_blocks(F, a_up, up, tf, kf, z, T):
    """Derivatives of the a->b face terms (rows: mass, energy, CO2) with respect
    to the unknowns of cell a (Da) and of cell b (Db).  F is the volumetric flux
    a->b, a_up marks faces upwinded from a, up the upwind cell, tf the
    transmissibility and kf the conductive transmissibility."""
    lam, lT, lz = _mobility(z[up], T[up])
    Tu, zu = T[up], z[up]
    # Darcy: F = tf lam (p_a - p_b); the derivatives follow from that law
    dF_dpa = tf * lam
    dF_dpb = -tf * lam
    dF_dTu = F * lT / lam
    dF_dzu = F * lz / lam
    m = F.shape[0]
    Da = np.zeros((m, 3, 3))   # d(flux a->b)/d(vars of a); rows mass, energy, CO2
    Db = np.zeros((m, 3, 3))
    ua = a_up.astype(np.float64)
    ub = 1.0 - ua
    for (D, dpv, u) in ((Da, dF_dpa, ua), (Db, dF_dpb, ub)):
        dFdT = dF_dTu * u
        dFdz = dF_dzu * u
        # mass
        D[:, 0, 0] = dpv
        D[:, 0, 1] = dFdT
        D[:, 0, 2] = dFdz
        # energy: F Cf Tu + kf (Ta - Tb)
        D[:, 1, 0] = CF * Tu * dpv
        D[:, 1, 1] = CF * Tu * dFdT + F * CF * u
        D[:, 1, 2] = CF * Tu * dFdz
        # CO2: F zu
        D[:, 2, 0] = zu * dpv
        D[:, 2, 1] = zu * dFdT
        D[:, 2, 2] = zu * dFdz + F * u
    Da[:, 1, 1] += kf
    Db[:, 1, 1] -= kf
    return Da, Db


def cartesian(name, nx, ny, nz, *, seed, sigma, corr, n_wells, r_front,
              kappa=KAPPA0, pe_target=None, tol=1e-6, rhs=True, dt=DT):
    """Assemble the thermal TPFA Jacobian on an nx*ny*nz grid (x fastest).
    `dt` is the time step dividing the accumulation terms."""
    rng = np.random.default_rng(seed)
    nc = nx * ny * nz
    g = _gauss_field(rng, (nz, ny, nx), corr)
    perm = (10.0 ** (-13.0 + sigma * g)).ravel()
    wells = _wells(nx, ny, n_wells)
    p3, T3, z3 = _state(nx, ny, nz, wells, r_front)
    p, T, z = p3.ravel(), T3.ravel(), z3.ravel()
    faces = _faces(nx, ny, nz)
    fluxes = _face_fluxes(p, faces)
    pe0 = peclet(fluxes, faces, kappa)
    if pe_target is not None:
        kappa = kappa * pe0 / pe_target
    pe = peclet(fluxes, faces, kappa)

    # Seven slots per row in sorted column order: -z, -y, -x, diag, +x, +y, +z.
    SLOT = {(2, -1): 0, (1, -1): 1, (0, -1): 2, (0, 1): 4, (1, 1): 5, (2, 1): 6}
    val7 = np.zeros((nc, 7, 3, 3))
    has7 = np.zeros((nc, 7), dtype=bool)
    has7[:, 3] = True
    vol = DX * DY * DZ
    val7[:, 3, 0, 0] += vol * PORO * CT / dt
    val7[:, 3, 1, 1] += vol * (PORO * CF + (1.0 - PORO) * CR) / dt
    val7[:, 3, 2, 2] += vol * PORO / dt

    for F, (d, a, b, area, dist) in zip(fluxes, faces):
        ka, kb = perm[a], perm[b]
        tf = (area / dist) * 2.0 * ka * kb / (ka + kb)
        kf = kappa * area / dist
        a_up = (F > 0) | ((F == 0) & (a < b))
        up = np.where(a_up, a, b)
        Da, Db = _face_blocks(F, a_up, up, tf, kf, z, T)
        s_ab = SLOT[(d, 1)]    # in row a, neighbour b is on the + side
        s_ba = SLOT[(d, -1)]
        # within one direction every cell is a left (right) end at most once
        val7[a, 3] += Da
        val7[a, s_ab] += Db
        val7[b, s_ba] -= Da
        val7[b, 3] -= Db
        has7[a, s_ab] = True
        has7[b, s_ba] = True

    # Open lateral boundaries: outflow leaves at the cell's own state.
    bc, bF = _boundary_outflow(nx, ny, nz, wells)
    keep = bF > 0
    bc, bF = bc[keep], bF[keep]
    lam, lT, lz = _mobility(z[bc], T[bc])
    tb = (DY * DZ / DX) * perm[bc]      # x and y boundary faces share area/distance (DX = DY)
    D = np.zeros((bc.shape[0], 3, 3))
    dFdp, dFdT, dFdz = tb * lam, bF * lT / lam, bF * lz / lam
    D[:, 0, 0], D[:, 0, 1], D[:, 0, 2] = dFdp, dFdT, dFdz
    D[:, 1, 0] = CF * T[bc] * dFdp
    D[:, 1, 1] = CF * T[bc] * dFdT + bF * CF
    D[:, 1, 2] = CF * T[bc] * dFdz
    D[:, 2, 0], D[:, 2, 1], D[:, 2, 2] = z[bc] * dFdp, z[bc] * dFdT, z[bc] * dFdz + bF
    np.add.at(val7[:, 3], bc, D)

    # Column scaling (p in MPa) and row scaling by the mean accumulation diagonal.
    val7[:, :, :, 0] *= P_SCALE
    acc = np.array([vol * PORO * CT / dt * P_SCALE,
                    vol * (PORO * CF + (1.0 - PORO) * CR) / dt,
                    vol * PORO / dt])
    val7 /= acc[None, None, :, None]

    offs = np.array([-nx * ny, -nx, -1, 0, 1, nx, nx * ny], dtype=np.int64)
    cols7 = np.arange(nc, dtype=np.int64)[:, None] + offs[None, :]
    counts = has7.sum(axis=1)
    row_ptr = np.zeros(nc + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols7[has7].astype(np.int32)
    values = np.ascontiguousarray(val7[has7])
    del val7, cols7
    meta = dict(name=name, grid=[nx, ny, nz], seed=seed, sigma=sigma, corr=corr,
                n_wells=n_wells, r_front=r_front, kappa=kappa, peclet=pe,
                peclet_at_kappa0=pe0, pe_target=pe_target, tol=tol,
                dx=[DX, DY, DZ], porosity=PORO, ct=CT, mu_c=MU_C, cf=CF, cr=CR,
                dt=dt, row_scale=acc.tolist(), p_scale=P_SCALE,
                n_cells=nc, nnzb=int(col_idx.shape[0]))
    if rhs:
        xs = np.random.default_rng(seed + 1000).standard_normal(BLOCK * nc)
        b = bsr_matvec_plain(row_ptr, col_idx, values, xs)
    else:
        xs = np.zeros(BLOCK * nc)
        b = np.zeros(BLOCK * nc)
    return Case(name, nx, ny, nz, row_ptr.astype(np.int32), col_idx, values,
                b, xs, tol, meta)


def _delaunay_geometry(pts):
    """Planar Delaunay triangulation of `pts` (cell units) and its Voronoi dual.

    Returns the unique edges (i < j), the Voronoi edge length of each
    (circumcentre to circumcentre; circumcentre to the edge midpoint on the
    hull), the dual (barycentric) area of each point, and for every hull edge
    its outward unit normal, its length, and the triangle count."""
    from scipy.spatial import Delaunay
    tri = Delaunay(pts).simplices.astype(np.int64)
    ntri = tri.shape[0]
    A, B, C = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    # circumcentres
    d = 2.0 * (A[:, 0] * (B[:, 1] - C[:, 1]) + B[:, 0] * (C[:, 1] - A[:, 1]) + C[:, 0] * (A[:, 1] - B[:, 1]))
    a2, b2, c2 = (A ** 2).sum(1), (B ** 2).sum(1), (C ** 2).sum(1)
    cc = np.stack([(a2 * (B[:, 1] - C[:, 1]) + b2 * (C[:, 1] - A[:, 1]) + c2 * (A[:, 1] - B[:, 1])) / d,
                   (a2 * (C[:, 0] - B[:, 0]) + b2 * (A[:, 0] - C[:, 0]) + c2 * (B[:, 0] - A[:, 0])) / d], axis=1)
    tri_area = 0.5 * np.abs(d) / 2.0
    dual = np.zeros(pts.shape[0])
    for k in range(3):
        np.add.at(dual, tri[:, k], tri_area / 3.0)
    # edges with the triangles on either side and the vertex opposite
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    opp = np.concatenate([tri[:, 2], tri[:, 0], tri[:, 1]])
    tid = np.tile(np.arange(ntri), 3)
    e.sort(axis=1)
    key = e[:, 0] * pts.shape[0] + e[:, 1]
    order = np.argsort(key, kind="stable")
    key, e, opp, tid = key[order], e[order], opp[order], tid[order]
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    start = np.flatnonzero(first)
    count = np.diff(np.append(start, key.shape[0]))
    edges = e[start]
    t0 = tid[start]
    mid = 0.5 * (pts[edges[:, 0]] + pts[edges[:, 1]])
    ell = np.empty(edges.shape[0])
    two = count == 2
    ell[two] = np.linalg.norm(cc[t0[two]] - cc[tid[start[two] + 1]], axis=1)
    hull = ~two
    ell[hull] = np.linalg.norm(cc[t0[hull]] - mid[hull], axis=1)
    ell = np.maximum(ell, 1e-3)
    # outward normals of hull edges: away from the opposite vertex
    he = edges[hull]
    t = pts[he[:, 1]] - pts[he[:, 0]]
    nrm = np.stack([t[:, 1], -t[:, 0]], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    away = mid[hull] - pts[opp[start[hull]]]
    nrm *= np.where((nrm * away).sum(1) < 0, -1.0, 1.0)[:, None]
    hull_len = np.linalg.norm(t, axis=1)
    return edges, ell, dual, he, nrm, hull_len, ntri


def prism(name, n_points, n_layers, *, seed, sigma, corr, n_wells, r_front,
          kappa=KAPPA0, pe_target=None, tol=1e-6, rhs=True, rcm=True):
    """Assemble the thermal TPFA Jacobian on an unstructured prism mesh.

    `n_points` seeded uniform points in a square of side sqrt(n_points) cells
    (one cell = DX metres, so the mean point spacing is about DX) are
    Delaunay-triangulated; each point's Voronoi column, cut into `n_layers`
    layers of thickness DZ, is a cell.  Lateral neighbours are the Delaunay
    edges with TPFA transmissibility DZ * l_ij * k_harm / d_ij (l_ij the
    Voronoi edge length, d_ij the point distance); vertical neighbours share
    the column's dual area.  The physics, state, permeability statistics and
    scaling follow `cartesian`.  With `rcm` the cells are renumbered by
    reverse Cuthill-McKee on the cell graph, and that numbering is the matrix
    order (and so the ILU(0) order)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    rng = np.random.default_rng(seed)
    side = math.sqrt(n_points)
    pts = rng.uniform(0.0, side, size=(n_points, 2))
    edges, ell, dual, hedges, hnrm, hlen, ntri = _delaunay_geometry(pts)
    npnt, nl = n_points, n_layers
    nc = npnt * nl
    # permeability: the cartesian correlated field on a covering grid, sampled per cell
    G = max(1, int(math.ceil(side)))
    g = _gauss_field(rng, (nl, G, G), corr)
    gx = np.minimum((pts[:, 0]).astype(np.int64), G - 1)
    gy = np.minimum((pts[:, 1]).astype(np.int64), G - 1)
    perm = (10.0 ** (-13.0 + sigma * g[:, gy, gx])).ravel()          # layer-major: c = l*npnt + i
    # state from the point coordinates (cell units)
    if n_wells == 1:
        wells = [(0.0, 0.0)]
    elif n_wells == 4:
        q1, q3 = side / 4.0, 3.0 * side / 4.0
        wells = [(q1, q1), (q3, q1), (q1, q3), (q3, q3)]
    else:
        raise ValueError("n_wells must be 1 or 4")
    R = math.hypot(side, side)
    px, py = pts[:, 0], pts[:, 1]
    p2 = _radial_p(px, py, wells, R)
    dmin = np.full(npnt, np.inf)
    for (iw, jw) in wells:
        dmin = np.minimum(dmin, np.sqrt((px - iw) ** 2 + (py - jw) ** 2))
    T2 = T_RES - DT_INJ * 0.5 * (1.0 - np.tanh(dmin - r_front))
    z2 = 0.5 * (1.0 - np.tanh(dmin - 2.0 * r_front))
    p, T, z = np.tile(p2, nl), np.tile(T2, nl), np.tile(z2, nl)
    vol = np.tile(dual * DX * DY * DZ, nl)
    # faces: (direction, a, b, area, dist) with per-face area and distance
    lay = (np.arange(nl, dtype=np.int64) * npnt)[:, None]
    dlen = np.linalg.norm(pts[edges[:, 0]] - pts[edges[:, 1]], axis=1) * DX
    faces = [(0, (lay + edges[:, 0]).ravel(), (lay + edges[:, 1]).ravel(),
              np.tile(DZ * ell * DX, nl), np.tile(dlen, nl))]
    if nl > 1:
        lv = (np.arange(nl - 1, dtype=np.int64) * npnt)[:, None]
        ids = np.arange(npnt, dtype=np.int64)[None, :]
        faces.append((2, (lv + ids).ravel(), (lv + npnt + ids).ravel(),
                      np.tile(dual * DX * DY, nl - 1), np.full((nl - 1) * npnt, DZ)))
    fluxes = [(area / dist) * K_REF * LAM_REF * (p[a] - p[b]) for (d, a, b, area, dist) in faces]
    pe0 = peclet(fluxes, faces, kappa)
    if pe_target is not None:
        kappa = kappa * pe0 / pe_target
    pe = peclet(fluxes, faces, kappa)

    # matrix order
    fa = np.concatenate([f[1] for f in faces])
    fb = np.concatenate([f[2] for f in faces])
    if rcm:
        graph = csr_matrix((np.ones(2 * fa.shape[0], dtype=np.int8),
                            (np.concatenate([fa, fb]), np.concatenate([fb, fa]))), shape=(nc, nc))
        order = reverse_cuthill_mckee(graph, symmetric_mode=True).astype(np.int64)
        new = np.empty(nc, dtype=np.int64)
        new[order] = np.arange(nc, dtype=np.int64)
        del graph
    else:
        order = new = np.arange(nc, dtype=np.int64)

    rows, cols, blks = [], [], []
    diag = np.zeros((nc, 3, 3))
    diag[:, 0, 0] = vol * PORO * CT / DT
    diag[:, 1, 1] = vol * (PORO * CF + (1.0 - PORO) * CR) / DT
    diag[:, 2, 2] = vol * PORO / DT
    for F, (d, a, b, area, dist) in zip(fluxes, faces):
        ka, kb = perm[a], perm[b]
        tf = (area / dist) * 2.0 * ka * kb / (ka + kb)
        kf = kappa * area / dist
        a_up = (F > 0) | ((F == 0) & (new[a] < new[b]))
        up = np.where(a_up, a, b)
        Da, Db = _face_blocks(F, a_up, up, tf, kf, z, T)
        np.add.at(diag, a, Da)
        np.add.at(diag, b, -Db)
        rows += [a, b]
        cols += [b, a]
        blks += [Db, -Da]
    # open lateral boundary: outflow through the hull faces at the cell's own state
    mid = 0.5 * (pts[hedges[:, 0]] + pts[hedges[:, 1]])
    dp = _radial_p(mid[:, 0], mid[:, 1], wells, R) - _radial_p(mid[:, 0] + hnrm[:, 0], mid[:, 1] + hnrm[:, 1], wells, R)
    geo = DZ * hlen * DX / DX                                   # area / distance (one cell outward)
    Fh = np.maximum(geo * K_REF * LAM_REF * dp, 0.0)
    for end in (0, 1):                                          # half of the face to each end point
        bc = (lay + hedges[:, end]).ravel()
        bF = np.tile(0.5 * Fh, nl)
        keep = bF > 0
        bc, bF = bc[keep], bF[keep]
        lam, lT, lz = _mobility(z[bc], T[bc])
        tb = np.tile(0.5 * geo, nl)[keep] * perm[bc]
        D = np.zeros((bc.shape[0], 3, 3))
        dFdp, dFdT, dFdz = tb * lam, bF * lT / lam, bF * lz / lam
        D[:, 0, 0], D[:, 0, 1], D[:, 0, 2] = dFdp, dFdT, dFdz
        D[:, 1, 0] = CF * T[bc] * dFdp
        D[:, 1, 1] = CF * T[bc] * dFdT + bF * CF
        D[:, 1, 2] = CF * T[bc] * dFdz
        D[:, 2, 0], D[:, 2, 1], D[:, 2, 2] = z[bc] * dFdp, z[bc] * dFdT, z[bc] * dFdz + bF
        np.add.at(diag, bc, D)

    # scaling: p in MPa; rows by the accumulation diagonal of the mean cell
    vbar = float(vol.mean())
    acc = np.array([vbar * PORO * CT / DT * P_SCALE,
                    vbar * (PORO * CF + (1.0 - PORO) * CR) / DT,
                    vbar * PORO / DT])
    ids = np.arange(nc, dtype=np.int64)
    r_all = new[np.concatenate([ids] + rows)]
    c_all = new[np.concatenate([ids] + cols)]
    v_all = np.concatenate([diag] + blks)
    del diag, blks
    v_all[:, :, 0] *= P_SCALE
    v_all /= acc[None, :, None]
    key = r_all * nc + c_all
    srt = np.argsort(key, kind="stable")
    key, v_all = key[srt], v_all[srt]
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    start = np.flatnonzero(first)
    values = np.ascontiguousarray(np.add.reduceat(v_all, start, axis=0))
    ukey = key[start]
    col_idx = (ukey % nc).astype(np.int32)
    counts = np.bincount(ukey // nc, minlength=nc)
    row_ptr = np.zeros(nc + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    deg = np.bincount(np.concatenate([edges[:, 0], edges[:, 1]]), minlength=npnt)
    meta = dict(name=name, mesh="voronoi-prism", n_points=npnt, n_layers=nl, seed=seed,
                sigma=sigma, corr=corr, n_wells=n_wells, r_front=r_front, kappa=kappa,
                peclet=pe, peclet_at_kappa0=pe0, pe_target=pe_target, tol=tol, rcm=bool(rcm),
                dz=DZ, spacing=DX, porosity=PORO, ct=CT, mu_c=MU_C, cf=CF, cr=CR, dt=DT,
                row_scale=acc.tolist(), p_scale=P_SCALE, n_cells=nc, nnzb=int(col_idx.shape[0]),
                lateral_degree=[int(deg.min()), float(deg.mean()), int(deg.max())],
                n_triangles=int(ntri))
    if rhs:
        xs = np.random.default_rng(seed + 1000).standard_normal(BLOCK * nc)
        b = bsr_matvec_plain(row_ptr, col_idx, values, xs)
    else:
        xs = np.zeros(BLOCK * nc)
        b = np.zeros(BLOCK * nc)
    return Case(name, npnt, 1, nl, row_ptr.astype(np.int32), col_idx, values, b, xs, tol, meta)


def bsr_matvec_plain(row_ptr, col_idx, values, x):
    """b = A x used only to manufacture right-hand sides (b = A x*)."""
    nc = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(nc), np.diff(row_ptr))
    xb = x.reshape(nc, 3)
    contrib = np.einsum("kab,kb->ka", values, xb[col_idx])
    out = np.zeros((nc, 3))
    np.add.at(out, rows, contrib)
    return out.ravel()


# Workloads.  Seeds are SEED_BASE + k for workload k.
def config0():
    """20x20x5 grid, log10 k ~ N(-13, 0.5) i.i.d., one corner injector, tol 1e-8."""
    return cartesian("grid20x20x5", 20, 20, 5, seed=SEED_BASE + 0, sigma=0.5, corr=0,
                     n_wells=1, r_front=3.0, tol=1e-8)


def config1(pe_target=None):
    """100x100x20 grid, log-k std 1.0, correlation 10 cells, four injectors."""
    name = "grid100x100x20" + ("" if pe_target is None else f"_pe{pe_target:g}")
    return cartesian(name, 100, 100, 20, seed=SEED_BASE + 1, sigma=1.0, corr=10,
                     n_wells=4, r_front=5.0, pe_target=pe_target, tol=1e-6)


def config3():
    """250x250x50 grid (3.125M cells, 9.375M DOF), log-k std 1.5."""
    return cartesian("grid250x250x50", 250, 250, 50, seed=SEED_BASE + 3, sigma=1.5,
                     corr=10, n_wells=4, r_front=5.0, tol=1e-6)


def config3_slab(nz):
    """The 250x250x50 generator restricted to nz layers (bounded CPU samples)."""
    return cartesian(f"grid250x250x{nz}", 250, 250, nz, seed=SEED_BASE + 3, sigma=1.5,
                     corr=10, n_wells=4, r_front=5.0, tol=1e-6)


def config2():
    """Unstructured mesh: 50k points x 20 layers of Voronoi prisms (1M cells,
    3M DOF), log-k std 1.0, correlation 10 cells, four injectors, RCM order."""
    return prism("prism50000x20", 50000, 20, seed=SEED_BASE + 2, sigma=1.0, corr=10,
                 n_wells=4, r_front=5.0, tol=1e-6)


def prism_small(n_points, n_layers, seed=17, rcm=True, **kw):
    """Small prism meshes for pins and parity at oracle-friendly sizes."""
    return prism(f"prism{n_points}x{n_layers}", n_points, n_layers, seed=seed, sigma=1.0,
                 corr=2, n_wells=4, r_front=2.0, rcm=rcm, **kw)


SERVING_GRIDS = [(40, 40, 10), (80, 80, 20), (160, 160, 20), (200, 200, 40)]
SERVING_TOLS = [1e-4, 1e-6]


def serving_stream(n_requests, rate=20.0, seed=SEED_BASE * 1000):
    """A Poisson request stream: (arrival time in s, grid, tolerance, seed) per
    request.  Inter-arrival times are exponential with mean 1/rate; the grid is
    drawn uniformly from SERVING_GRIDS and the tolerance from SERVING_TOLS.
    Request r's Jacobian uses seed + r."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    t -= t[0]
    grids = rng.integers(len(SERVING_GRIDS), size=n_requests)
    tols = rng.integers(len(SERVING_TOLS), size=n_requests)
    return [(float(t[r]), SERVING_GRIDS[int(grids[r])], SERVING_TOLS[int(tols[r])], seed + r)
            for r in range(n_requests)]


def serving_case(grid, tol, seed):
    """One serving request: the 100x100x20 generator (log-k std 1.0,
    correlation 10 cells, four injectors) on `grid` with its own seed."""
    nx, ny, nz = grid
    return cartesian(f"grid{nx}x{ny}x{nz}_s{seed}", nx, ny, nz, seed=seed, sigma=1.0, corr=10,
                     n_wells=4, r_front=5.0, tol=tol)


def small(nx, ny, nz, seed=7, sigma=0.5, n_wells=1, r_front=2.0, **kw):
    """Tiny grids for pins and parity at oracle-friendly sizes."""
    return cartesian(f"grid{nx}x{ny}x{nz}", nx, ny, nz, seed=seed, sigma=sigma, corr=0,
                     n_wells=n_wells, r_front=r_front, **kw)


def by_name(name: str) -> Case:
    table = {"grid20x20x5": config0, "grid100x100x20": config1,
             "grid250x250x50": config3}
    if name in table:
        return table[name]()
    if name == "prism50000x20":
        return config2()
    if name.startswith("prism"):
        npnt, nl = (int(v) for v in name[5:].split("x"))
        return prism_small(npnt, nl)
    if name.startswith("grid250x250x") and name != "grid250x250x50":
        return config3_slab(int(name.split("x")[-1]))
    if name.startswith("grid100x100x20_pe"):
        return config1(float(name.split("_pe")[1]))
    if name.startswith("grid"):
        dims = [int(v) for v in name[4:].split("x")]
        return small(*dims)
    raise KeyError(name)


def meta_json(case: Case) -> str:
    return json.dumps(case.meta, sort_keys=True)

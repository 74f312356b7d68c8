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
        vals.append(np.abs(F[nz_]) * CF * dist / (kappa * area))
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


def cartesian(name, nx, ny, nz, *, seed, sigma, corr, n_wells, r_front,
              kappa=KAPPA0, pe_target=None, tol=1e-6, rhs=True):
    """Assemble the thermal TPFA Jacobian on an nx*ny*nz grid (x fastest)."""
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
    val7[:, 3, 0, 0] += vol * PORO * CT / DT
    val7[:, 3, 1, 1] += vol * (PORO * CF + (1.0 - PORO) * CR) / DT
    val7[:, 3, 2, 2] += vol * PORO / DT

    for F, (d, a, b, area, dist) in zip(fluxes, faces):
        ka, kb = perm[a], perm[b]
        tf = (area / dist) * 2.0 * ka * kb / (ka + kb)
        kf = kappa * area / dist
        a_up = (F > 0) | ((F == 0) & (a < b))
        up = np.where(a_up, a, b)
        lam, lT, lz = _mobility(z[up], T[up])
        Tu, zu = T[up], z[up]
        # Darcy: F = tf lam (p_a - p_b); the derivatives follow from that law
        dF_dpa = tf * lam
        dF_dpb = -tf * lam
        dF_dTu = F * lT / lam
        dF_dzu = F * lz / lam
        m = a.shape[0]
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
    acc = np.array([vol * PORO * CT / DT * P_SCALE,
                    vol * (PORO * CF + (1.0 - PORO) * CR) / DT,
                    vol * PORO / DT])
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
                dt=DT, row_scale=acc.tolist(), p_scale=P_SCALE,
                n_cells=nc, nnzb=int(col_idx.shape[0]))
    if rhs:
        xs = np.random.default_rng(seed + 1000).standard_normal(BLOCK * nc)
        b = bsr_matvec_plain(row_ptr, col_idx, values, xs)
    else:
        xs = np.zeros(BLOCK * nc)
        b = np.zeros(BLOCK * nc)
    return Case(name, nx, ny, nz, row_ptr.astype(np.int32), col_idx, values,
                b, xs, tol, meta)


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


def small(nx, ny, nz, seed=7, sigma=0.5, n_wells=1, r_front=2.0, **kw):
    """Tiny grids for pins and parity at oracle-friendly sizes."""
    return cartesian(f"grid{nx}x{ny}x{nz}", nx, ny, nz, seed=seed, sigma=sigma, corr=0,
                     n_wells=n_wells, r_front=r_front, **kw)


def by_name(name: str) -> Case:
    table = {"grid20x20x5": config0, "grid100x100x20": config1,
             "grid250x250x50": config3}
    if name in table:
        return table[name]()
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

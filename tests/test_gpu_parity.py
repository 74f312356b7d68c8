"""GPU parity: the HIP library against the CPU oracle through the C ABI.

Bars: block SpMV within a componentwise rounding bound (1e-13 of |A||x|);
one preconditioner application within 1e-10 relative (2-norm) of the oracle;
GMRES/FGMRES iteration counts within +-1 of the oracle and the true relative
residual at or below the tolerance.
"""
import numpy as np
import pytest

import oracle as O
import paper_2308_11892_amd as L
from synth import jacobian as J

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# Voronoi-prism meshes in RCM order (the unstructured workload at small sizes)
PRISMS = ["prism300x4", "prism2000x5"]
CASES = ["grid20x20x5", "grid7x5x3", "grid1x1x1", "grid2x1x1", "grid13x1x1", "grid33x17x2"] + PRISMS


@pytest.fixture(scope="module")
def solvers():
    cache = {}

    def get(name):
        if name not in cache:
            c = J.by_name(name)
            say(f"[setup] {name} cells={c.n_cells}")
            cache[name] = (c, L.Solver(c.row_ptr, c.col_idx, c.values),
                           O.Cptr(c.row_ptr, c.col_idx, c.values))
        return cache[name]

    yield get
    for _, s, _ in cache.values():
        s.close()


@pytest.mark.parametrize("name", CASES)
def test_spmv_parity(solvers, name):
    c, s, _ = solvers(name)
    say(f"[spmv] {name}")
    x = np.random.default_rng(1).standard_normal(c.n_dof)
    y = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
    s.spmv(dev(x), y)
    yo = O.bsr_spmv(c.row_ptr, c.col_idx, c.values, x)
    absA = J.bsr_matvec_plain(c.row_ptr, c.col_idx, np.abs(c.values), np.abs(x))
    assert np.all(np.abs(host(y) - yo) <= 1e-13 * absA + 1e-300)


GRIDS_3D = ["grid20x20x5", "grid7x5x3", "grid33x17x2"]
GRIDS_1D = ["grid1x1x1", "grid2x1x1", "grid13x1x1"]


def _apply_vectors(c, ref):
    rng = np.random.default_rng(2)
    vecs = [rng.standard_normal(c.n_dof), c.b / np.linalg.norm(c.b)]
    # a Krylov direction: A M^-1 b, normalised
    w = ref.spmv(ref.apply(vecs[1]))
    vecs.append(w / np.linalg.norm(w))
    return vecs


@pytest.mark.parametrize("name", GRIDS_3D + PRISMS)
def test_apply_parity(solvers, name):
    c, s, ref = solvers(name)
    say(f"[apply] {name}")
    for r in _apply_vectors(c, ref):
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        zo = ref.apply(r)
        err = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
        assert err <= 1e-10, (name, err)


@pytest.mark.parametrize("name", GRIDS_1D)
def test_apply_exact_on_1d_grids(solvers, name):
    """On 1D grids ILU(0) is exact and Eq. (3) collapses to A^-1; the two
    stages then cancel (|x1| >> |z|), so the bar is the forward error of the
    oracle's own apply against a dense solve (times 10, floor 1e-13)."""
    c, s, ref = solvers(name)
    say(f"[apply-1d] {name}")
    A = c.to_scipy().toarray()
    for r in _apply_vectors(c, ref):
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        ze = np.linalg.solve(A, r)
        e_or = np.linalg.norm(ref.apply(r) - ze) / np.linalg.norm(ze)
        e_gpu = np.linalg.norm(host(z) - ze) / np.linalg.norm(ze)
        assert e_gpu <= 10 * max(e_or, 1e-13), (name, e_gpu, e_or)


def test_apply_is_deterministic(solvers):
    c, s, _ = solvers("grid20x20x5")
    r = dev(np.random.default_rng(4).standard_normal(c.n_dof))
    z1 = torch.empty_like(r)
    z2 = torch.empty_like(r)
    s.apply(r, z1)
    s.apply(r, z2)
    assert torch.equal(z1, z2)


@pytest.mark.parametrize("name,restart,flexible,tol", [
    ("grid20x20x5", 30, False, 1e-8),
    ("grid20x20x5", 50, True, 1e-8),
    ("grid33x17x2", 30, False, 1e-8),
    ("grid13x1x1", 30, False, 1e-10),
    ("prism2000x5", 30, False, 1e-8),
    ("prism2000x5", 50, True, 1e-6),
])
def test_gmres_parity(solvers, name, restart, flexible, tol):
    c, s, ref = solvers(name)
    say(f"[gmres] {name} restart={restart} flexible={flexible} tol={tol}")
    b = dev(c.b)
    x = torch.zeros_like(b)
    info = s.gmres_solve(b, x, restart=restart, flexible=flexible, rtol=tol)
    xo, oinfo = ref.gmres(c.b, restart=restart, flexible=flexible, rtol=tol)
    assert info["converged"], info
    assert abs(info["iterations"] - oinfo["iterations"]) <= 1, (info, oinfo)
    xh = host(x)
    res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, xh)) / np.linalg.norm(c.b)
    assert res <= tol * (1 + 1e-6), res
    assert abs(info["rel_res_true"] - res) <= 1e-3 * res + 1e-15


def test_gmres_not_converged_returns_last_iterate(solvers):
    c, s, _ = solvers("grid20x20x5")
    b = dev(c.b)
    x = torch.zeros_like(b)
    info = s.gmres_solve(b, x, rtol=1e-300, max_iter=3)
    assert info["status"] == L.CPTR_NOT_CONVERGED and info["iterations"] == 3
    assert info["rel_res_true"] < 1.0


def test_gmres_nonzero_initial_guess(solvers):
    c, s, ref = solvers("grid20x20x5")
    x0 = np.random.default_rng(9).standard_normal(c.n_dof) * 1e-3
    b = dev(c.b)
    x = dev(x0)
    info = s.gmres_solve(b, x, x0_is_zero=False, rtol=1e-8)
    _, oinfo = ref.gmres(c.b, x0=x0, rtol=1e-8)
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1


def test_gmres_zero_rhs(solvers):
    c, s, _ = solvers("grid7x5x3")
    b = torch.zeros(c.n_dof, dtype=torch.float64, device=DEV)
    x = torch.ones_like(b)
    info = s.gmres_solve(b, x)
    assert info["converged"] and info["iterations"] == 0
    assert torch.count_nonzero(x).item() == 0


def test_profiled_solve_reports_phases(solvers):
    c, s, _ = solvers("grid20x20x5")
    b = dev(c.b)
    x = torch.zeros_like(b)
    s.phase_times(reset=True)
    info = s.gmres_solve(b, x, rtol=1e-8, profile=True)
    ph = s.phase_times(reset=True)
    assert ph["spmv"][1] >= info["iterations"]
    assert ph["ilu_fwd"][1] >= info["iterations"] and ph["ilu_fwd"][0] > 0
    assert ph["arnoldi"][1] == info["iterations"]
    # a mask times only the phases whose bit (index + 1) is set, and the
    # solve itself is unchanged
    x2 = torch.zeros_like(b)
    k = L.PHASES.index("ilu_bwd")
    info2 = s.gmres_solve(b, x2, rtol=1e-8, profile=1 << (k + 1))
    ph2 = s.phase_times(reset=True)
    assert ph2["ilu_bwd"][1] == ph["ilu_bwd"][1] and ph2["ilu_bwd"][0] > 0
    assert all(cnt == 0 for name, (_, cnt) in ph2.items() if name != "ilu_bwd")
    assert info2["iterations"] == info["iterations"] and torch.equal(x, x2)
    # without profiling (and with the timed ilu_bwd mask above) the next step's
    # restriction is queued before the host reads the Hessenberg column; the
    # kernels and their order are the same, so the result is too
    x3 = torch.zeros_like(b)
    info3 = s.gmres_solve(b, x3, rtol=1e-8)
    assert info3["iterations"] == info["iterations"] and torch.equal(x, x3)


@pytest.mark.parametrize("pe", [None, 0.1, 10.0, 1000.0])
def test_gmres_parity_grid100x100x20(pe):
    c = J.config1(pe)
    say(f"[gmres] {c.name} FGMRES(50) tol 1e-6")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
        rng = np.random.default_rng(5)
        r = rng.standard_normal(c.n_dof)
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        zo = ref.apply(r)
        assert np.linalg.norm(host(z) - zo) <= 1e-10 * np.linalg.norm(zo)
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
    _, oinfo = ref.gmres(c.b, restart=50, flexible=True, rtol=1e-6)
    say(f"  gpu {info['iterations']} it, oracle {oinfo['iterations']} it")
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1
    res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, host(x))) / np.linalg.norm(c.b)
    assert res <= 1e-6


@pytest.mark.parametrize("name", ["grid20x20x5", "grid33x17x2", "grid7x5x3", "grid2x2x2",
                                  "grid1x1x1", "grid13x1x1"] + PRISMS)
def test_ilu_sweep_modes_agree(name):
    """Per-level launches, one-launch sweeps and (on 3D grids) the tiled grid
    sweeps compute the same preconditioner; all match the oracle."""
    c = J.by_name(name)
    say(f"[sweep-modes] {name}")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    r = np.random.default_rng(12).standard_normal(c.n_dof)
    zo = ref.apply(r)
    is_grid = min(c.nx, c.ny, c.nz) >= 2
    modes = [L.ILU_SWEEP_LEVELS, L.ILU_SWEEP_ONE_LAUNCH] + ([L.ILU_SWEEP_GRID] if is_grid else [])
    outs = []
    for mode in modes:
        with L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=mode) as s:
            used = s.export("SWEEP", 0, 4, np.int32)
            assert used[0] == mode, (mode, used)
            if mode == L.ILU_SWEEP_GRID:
                assert tuple(used[1:]) == (c.nx, c.ny, c.nz)
            z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
            for _ in range(3):  # repeated applies reuse the ticket counters and sentinels
                s.apply(dev(r), z)
            outs.append(host(z))
    for z in outs:
        assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    for z in outs[1:]:
        # the schedules sum the neighbour blocks in different orders
        assert np.linalg.norm(z - outs[0]) <= 1e-13 * np.linalg.norm(outs[0])
    if not is_grid:
        with pytest.raises(L.CptrError):
            L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=L.ILU_SWEEP_GRID)


def test_auto_sweep_picks_grid_on_cartesian():
    c = J.config0()
    with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
        assert tuple(s.export("SWEEP", 0, 4, np.int32)) == (L.ILU_SWEEP_GRID, 20, 20, 5)


def test_one_launch_sweep_gmres_grid100x100x20():
    c = J.config1()
    say(f"[sweep-modes] {c.name} gmres")
    with L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=L.ILU_SWEEP_ONE_LAUNCH) as s:
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    _, oinfo = ref.gmres(c.b, restart=50, flexible=True, rtol=1e-6)
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1


def test_gmres_parity_prism10000x10():
    """A 100k-cell Voronoi-prism mesh in RCM order: one application within
    1e-10 and FGMRES(50) to 1e-6 within +-1 iteration of the oracle, through
    the automatic sweep schedule (no grid structure)."""
    c = J.by_name("prism10000x10")
    say(f"[gmres] {c.name} FGMRES(50) tol 1e-6")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
        assert s.export("SWEEP", 0, 4, np.int32)[0] in (L.ILU_SWEEP_ONE_LAUNCH, L.ILU_SWEEP_LEVELS)
        r = np.random.default_rng(6).standard_normal(c.n_dof)
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        zo = ref.apply(r)
        assert np.linalg.norm(host(z) - zo) <= 1e-10 * np.linalg.norm(zo)
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
    _, oinfo = ref.gmres(c.b, restart=50, flexible=True, rtol=1e-6)
    say(f"  gpu {info['iterations']} it, oracle {oinfo['iterations']} it")
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1
    res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, host(x))) / np.linalg.norm(c.b)
    assert res <= 1e-6


@pytest.mark.parametrize("name", ["grid20x20x5", "grid33x17x2", "prism2000x5"])
def test_cpr_parity(name):
    """CPR (pressure alone in the first stage, elliptic set {p}) runs through the
    same code with one elliptic unknown: one application within 1e-10 of the
    oracle's CPR and GMRES iterations within +-1."""
    c = J.by_name(name)
    say(f"[cpr] {name}")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values, elliptic=(0,))
    with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=(0,)) as s:
        for r in _apply_vectors(c, ref):
            z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
            s.apply(dev(r), z)
            zo = ref.apply(r)
            assert np.linalg.norm(host(z) - zo) <= 1e-10 * np.linalg.norm(zo)
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=30, rtol=1e-8)
    _, oinfo = ref.gmres(c.b, restart=30, rtol=1e-8)
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1, (info, oinfo)


def test_cptr_against_cpr_on_the_peclet_sweep():
    """The paper's comparison on the 100x100x20 generator with a 30-day time
    step (conduction and transport strong enough to matter): CPTR needs no
    more iterations than CPR at any Peclet number, and its count does not
    move with Pe."""
    its = {"cptr": [], "cpr": []}
    for pe in (0.1, 10.0, 1000.0):
        c = J.cartesian("g", 100, 100, 20, seed=J.SEED_BASE + 1, sigma=1.0, corr=10, n_wells=4,
                        r_front=5.0, pe_target=pe, dt=86400.0 * 30)
        for name, ell in (("cptr", (0, 1)), ("cpr", (0,))):
            with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=ell) as s:
                b = dev(c.b)
                x = torch.zeros_like(b)
                info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
                assert info["converged"]
                its[name].append(info["iterations"])
    say(f"[cpr] Pe 0.1/10/1000: CPTR {its['cptr']} CPR {its['cpr']}")
    assert all(a <= b for a, b in zip(its["cptr"], its["cpr"]))
    assert max(its["cptr"]) - min(its["cptr"]) <= 1


@pytest.mark.parametrize("name,row", [("grid3x3x2", 2), ("prism2000x5", 0)])
def test_device_ilu_zero_pivot_matches_host(name, row):
    """A device handle factors ILU(0) on the GPU; a singular diagonal block is
    reported like the host factorisation does (same row), on a grid and on an
    unstructured mesh."""
    c = J.small(3, 3, 2) if name == "grid3x3x2" else J.by_name(name)
    v = c.values.copy()
    k = [q for q in range(c.row_ptr[row], c.row_ptr[row + 1]) if c.col_idx[q] == row][0]
    v[k, 2, 2] = 0.0
    v[k, 0:2, 2] = 0.0
    v[k, 2, 0:2] = 0.0
    msgs = []
    for host_only in (1, 0):
        with pytest.raises(L.CptrError) as e:
            L.Solver(c.row_ptr, c.col_idx, v, host_only=host_only, restriction=L.RESTRICT_INJECTION)
        assert e.value.code == L.CPTR_E_ZERO_PIVOT
        msgs.append(str(e.value))
    assert "ILU" in msgs[1] and msgs[0] == msgs[1], msgs


@pytest.mark.parametrize("name", ["grid7x5x3", "prism2000x5"])
def test_device_ilu_export_refused(name):
    c = J.by_name(name)
    with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
        with pytest.raises(L.CptrError) as e:
            s.export("ILU_VALS", 0, c.nnzb * 9)
        assert e.value.code == L.CPTR_E_STATE


@pytest.mark.parametrize("name", ["grid20x20x5", "prism2000x5"])
def test_setup_from_device_arrays(name):
    """A handed over in device memory (cptr_bsr.on_device = 1) gives the same
    preconditioner, bit for bit, as the same matrix from host memory."""
    c = J.by_name(name)
    r = dev(np.random.default_rng(13).standard_normal(c.n_dof))
    outs = []
    for on_dev in (False, True):
        if on_dev:
            args = (torch.tensor(c.row_ptr, device=DEV), torch.tensor(c.col_idx, device=DEV),
                    torch.tensor(c.values, device=DEV))
        else:
            args = (c.row_ptr, c.col_idx, c.values)
        with L.Solver(*args) as s:
            z = torch.empty_like(r)
            s.apply(r, z)
            outs.append(host(z))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name,elliptic,agg", [("grid20x20x5", (0, 1), 1), ("prism2000x5", (0, 1), 1),
                                               ("grid30x20x6", (0,), 1), ("grid100x100x20", (0, 1), 1),
                                               ("prism2000x5", (0, 1), 2), ("grid20x20x5", (0, 1), 0)])
def test_device_setup_steps_equal_host(name, elliptic, agg):
    """A device handle forms every strength graph, every interpolation
    (extended+i, and multipass on the aggressive levels) and every coarse
    operator R A P on the GPU; the hierarchy equals the host's bit for bit
    (same splits, patterns and values on every level)."""
    c = J.by_name(name)
    say(f"[device setup] {name} elliptic={elliptic} agg_levels={agg}")
    with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=elliptic, agg_levels=agg) as sd, \
            L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=elliptic, host_only=1, agg_levels=agg) as sh:
        rows_d, nnz_d = sd.hierarchy()
        rows_h, nnz_h = sh.hierarchy()
        assert np.array_equal(rows_d, rows_h) and np.array_equal(nnz_d, nnz_h)
        sites = sd.export("SETUP_SITES", 0, 15, np.int32)
        built = len(rows_d) - 1
        na = min(agg, built)
        assert list(sites[:10]) == [built, built, built - na, built - na, built, built, na, na, na, na], sites
        # every first pass starts on the device (its small components there)
        assert sites[10] == sites[11] >= built + na, sites
        assert list(sites[13:]) == [0, 0], sites
        say(f"  first-pass points decided on the device: {sites[12] / 10:.1f} %")
        for l in range(len(rows_d)):
            for which in ("A", "P") if l + 1 < len(rows_d) else ("A",):
                Md, Mh = sd.level_matrix(l, which), sh.level_matrix(l, which)
                assert np.array_equal(Md.indptr, Mh.indptr) and np.array_equal(Md.indices, Mh.indices)
                assert np.array_equal(Md.data, Mh.data), f"level {l} {which}"


@pytest.mark.parametrize("name,block,agg", [("grid100x100x20", 4096, 1), ("grid100x100x20", 1, 1),
                                            ("prism2000x5", 512, 1), ("prism2000x5", 64, 0),
                                            ("grid20x20x5", 1000, 1)])
def test_device_hmis_blocks_equal_host(name, block, agg):
    """hmis_block > 0: every split over several blocks (the blocks' first
    passes, the cover by their C points and the PMIS rounds) runs on the GPU
    and gives the host's split, so the whole hierarchy matches bit for bit."""
    c = J.by_name(name)
    say(f"[device hmis] {name} hmis_block={block} agg_levels={agg}")
    kw = dict(hmis_block=block, agg_levels=agg)
    with L.Solver(c.row_ptr, c.col_idx, c.values, **kw) as sd, \
            L.Solver(c.row_ptr, c.col_idx, c.values, host_only=1, **kw) as sh:
        rows_d, nnz_d = sd.hierarchy()
        rows_h, nnz_h = sh.hierarchy()
        assert np.array_equal(rows_d, rows_h) and np.array_equal(nnz_d, nnz_h)
        sites = sd.export("SETUP_SITES", 0, 15, np.int32)
        assert sites[14] > 0 and sites[13] == sites[14], sites
        for l in range(len(rows_d)):
            for which in ("A", "P") if l + 1 < len(rows_d) else ("A",):
                Md, Mh = sd.level_matrix(l, which), sh.level_matrix(l, which)
                assert np.array_equal(Md.indptr, Mh.indptr) and np.array_equal(Md.indices, Mh.indices)
                assert np.array_equal(Md.data, Mh.data), f"level {l} {which}"

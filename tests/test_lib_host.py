"""CPU tests of the HIP library: ABI surface, error paths and the host setup.

The library's setup is an independent implementation; here it is built
host-only (no device calls) and compared with the oracle: identical C/F
splits level by level, interpolation and operators to rounding, and ILU(0)
factors that reproduce A on its pattern and give the oracle's sweeps.
"""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import paper_2308_11892_amd as L
from synth import jacobian as J


def host_solver(c, **kw):
    return L.Solver(c.row_ptr, c.col_idx, c.values, host_only=1, **kw)


def test_library_exports_every_header_symbol():
    lib = C.CDLL(L.LIB_PATH)
    names = L.header_functions()
    assert {"cptr_setup", "cptr_apply", "cptr_gmres_solve", "cptr_destroy"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_defaults_follow_the_paper():
    o = L.setup_opts()
    assert (o.strong_threshold, o.max_row_sum, o.max_levels, o.max_coarse, o.p_max_elmts,
            o.agg_levels) == (0.25, 0.9, 25, 9, 4, 1)
    s = L.solve_opts()
    assert (s.max_iter, s.rtol, s.restart) == (200, 1e-6, 30)
    # one l1-Jacobi sweep on each side; the Krylov space of FGMRES(50) is
    # allocated at setup
    assert (o.num_sweeps, o.max_restart, o.flexible_space) == (1, 50, 1)
    # one HMIS block per level: the first pass over the whole level; coarsest
    # levels up to 4096 rows solved exactly
    assert o.hmis_block == 0 and o.max_dense_coarse == 4096
    # the V-cycle below the largest level of at most 2048 rows runs as one
    # dense operator
    assert o.dense_tail == 2048


@pytest.mark.parametrize("case,agg", [("grid20x20x5", 1), ("grid6x5x4", 1), ("grid12x1x1", 1),
                                      ("grid100x100x20_pe0.1", 1), ("grid20x20x5", 0),
                                      ("grid100x100x20_pe0.1", 0), ("prism300x4", 1),
                                      ("prism2000x5", 1), ("prism2000x5", 0)])
def test_host_setup_matches_oracle(case, agg):
    c = J.by_name(case)
    h = O.Cptr(c.row_ptr, c.col_idx, c.values, agg_levels=agg)
    s = host_solver(c, agg_levels=agg)
    rows, nnz = s.hierarchy()
    a = h.amg
    assert len(rows) == a.nlevels
    # quasi-IMPES weights are the same division, bit for bit
    W = s.export("W", 0, c.n_cells * 2)
    assert np.array_equal(W, h.W().ravel())
    for l in range(a.nlevels):
        assert rows[l] == a.size(l)[0]
        # same arithmetic in the same order (FP contraction off on both
        # sides): every level's operator, split and interpolation agree to
        # the last bit
        Al, Ao = s.level_matrix(l, "A"), a.A(l)
        assert np.array_equal(Al.indptr, Ao.indptr) and np.array_equal(Al.indices, Ao.indices)
        assert np.array_equal(Al.data, Ao.data), l
        if l + 1 < a.nlevels:
            assert np.array_equal(s.cf(l), a.cf(l)), f"C/F split differs at level {l}"
            Pl, Po = s.level_matrix(l, "P"), a.P(l)
            assert np.array_equal(Pl.indices, Po.indices) and np.array_equal(Pl.data, Po.data), l
            dv = s.export("DINV", l, int(rows[l]))
            assert np.array_equal(dv, a.dinv(l))


def _block_factors(c, F):
    """Block L (unit block-lower) and U from the exported block factors."""
    nb = c.n_cells
    rows = np.repeat(np.arange(nb), np.diff(c.row_ptr))
    cols = c.col_idx
    low = cols < rows
    Lb = sp.bsr_matrix((F[low], cols[low], np.concatenate([[0], np.cumsum(np.bincount(rows[low], minlength=nb))])),
                       shape=(c.n_dof, c.n_dof)).toarray() + np.eye(c.n_dof)
    up = ~low
    Ub = sp.bsr_matrix((F[up], cols[up], np.concatenate([[0], np.cumsum(np.bincount(rows[up], minlength=nb))])),
                       shape=(c.n_dof, c.n_dof)).toarray()
    return Lb, Ub


def test_host_block_ilu_is_ilu0():
    c = J.small(5, 4, 3)
    s = host_solver(c)
    F = s.export("ILU_VALS", 0, c.nnzb * 9).reshape(c.nnzb, 3, 3)
    Lb, Ub = _block_factors(c, F)
    A = c.to_scipy().toarray()
    mask = sp.bsr_matrix((np.ones_like(c.values), c.col_idx, c.row_ptr),
                         shape=A.shape).toarray() > 0
    assert np.abs((Lb @ Ub - A)[mask]).max() <= 1e-13 * np.abs(A).max()
    # same preconditioner as the oracle's scalar ILU(0)
    h = O.Cptr(c.row_ptr, c.col_idx, c.values)
    r = np.random.default_rng(0).standard_normal(c.n_dof)
    x = np.linalg.solve(Ub, np.linalg.solve(Lb, r))
    assert np.linalg.norm(x - h.ilu_solve(r)) <= 1e-10 * np.linalg.norm(x)
    nl = s.export("ILU_NLEVELS", 0, 2, np.int32)
    assert tuple(nl) == (5 + 4 + 3 - 2, 5 + 4 + 3 - 2)


def test_host_setup_cpr_split_matches_oracle():
    c = J.small(6, 5, 3)
    h = O.Cptr(c.row_ptr, c.col_idx, c.values, elliptic=(0,))
    s = L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=(0,), host_only=1)
    W = s.export("W", 0, c.n_cells * 2)
    # explicit 2x2 inverse here, elimination in the oracle: rounding-level differences
    np.testing.assert_allclose(W, h.W().ravel(), rtol=1e-9, atol=1e-14 * np.abs(W).max())
    rows, _ = s.hierarchy()
    for l in range(len(rows) - 1):
        assert np.array_equal(s.cf(l), h.amg.cf(l))


# ----------------------------------------------------------------- errors
def _expect(code, fn):
    with pytest.raises(L.CptrError) as e:
        fn()
    assert e.value.code == code, str(e.value)
    return str(e.value)


def test_invalid_arguments():
    c = J.small(3, 3, 2)
    _expect(L.CPTR_E_INVALID, lambda: L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=(0, 0), host_only=1))
    _expect(L.CPTR_E_INVALID, lambda: L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=(0, 3), host_only=1))
    _expect(L.CPTR_E_INVALID, lambda: L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=(0, 1, 2), host_only=1))
    v = c.values.copy()
    v[5, 1, 1] = np.nan
    msg = _expect(L.CPTR_E_INVALID, lambda: L.Solver(c.row_ptr, c.col_idx, v, host_only=1))
    assert "non-finite" in msg
    ci = c.col_idx.copy()
    ci[[0, 1]] = ci[[1, 0]]
    msg = _expect(L.CPTR_E_INVALID, lambda: L.Solver(c.row_ptr, ci, c.values, host_only=1))
    assert "row 0" in msg
    # drop the diagonal block of row 4
    k = [q for q in range(c.row_ptr[4], c.row_ptr[5]) if c.col_idx[q] == 4][0]
    keep = np.ones(c.nnzb, bool)
    keep[k] = False
    rp = c.row_ptr.copy()
    rp[5:] -= 1
    msg = _expect(L.CPTR_E_INVALID, lambda: L.Solver(rp, c.col_idx[keep], c.values[keep], host_only=1))
    assert "diagonal" in msg and "4" in msg
    for kw, word in [(dict(num_sweeps=0), "num_sweeps"), (dict(num_sweeps=9), "num_sweeps"),
                     (dict(max_restart=0), "max_restart"), (dict(max_restart=65), "max_restart"),
                     (dict(flexible_space=2), "flexible_space"), (dict(hmis_block=-1), "range"),
                     (dict(max_dense_coarse=-1), "range"), (dict(max_dense_coarse=4097), "range"),
                     (dict(dense_tail=-1), "range"), (dict(dense_tail=4097), "range")]:
        msg = _expect(L.CPTR_E_INVALID, lambda: L.Solver(c.row_ptr, c.col_idx, c.values, host_only=1, **kw))
        assert word in msg, msg


@pytest.mark.parametrize("case,agg,block", [("grid100x100x20_pe0.1", 1, 4096), ("grid100x100x20_pe0.1", 0, 4096),
                                            ("grid20x20x5", 1, 1), ("prism2000x5", 1, 512),
                                            ("prism2000x5", 0, 64), ("grid40x40x10", 1, 1000)])
def test_host_hmis_split_matches_oracle(case, agg, block):
    """HMIS over row blocks: the library's host split (blocks in parallel,
    then the PMIS rounds) equals the oracle's on every level, and so do the
    interpolation and the coarse operators built on it."""
    c = J.by_name(case)
    h = O.Cptr(c.row_ptr, c.col_idx, c.values, agg_levels=agg, hmis_block=block)
    s = host_solver(c, agg_levels=agg, hmis_block=block)
    rows, _ = s.hierarchy()
    a = h.amg
    assert len(rows) == a.nlevels
    for l in range(a.nlevels - 1):
        assert np.array_equal(s.cf(l), a.cf(l)), f"C/F split differs at level {l}"
        Pl, Po = s.level_matrix(l, "P"), a.P(l)
        assert np.array_equal(Pl.indices, Po.indices) and np.array_equal(Pl.data, Po.data), l
    Al, Ao = s.level_matrix(a.nlevels - 1, "A"), a.A(a.nlevels - 1)
    assert np.array_equal(Al.data, Ao.data)


def test_zero_pivot_errors():
    c = J.small(3, 3, 2)
    v = c.values.copy()
    k = [q for q in range(c.row_ptr[2], c.row_ptr[3]) if c.col_idx[q] == 2][0]
    v[k, 2, 2] = 0.0
    v[k, 0:2, 2] = 0.0
    v[k, 2, 0:2] = 0.0
    # singular hyperbolic diagonal entry -> quasi-IMPES cannot form W
    _expect(L.CPTR_E_ZERO_PIVOT, lambda: L.Solver(c.row_ptr, c.col_idx, v, host_only=1))
    # with injection the same matrix fails in ILU(0) on the singular block
    msg = _expect(L.CPTR_E_ZERO_PIVOT,
                  lambda: L.Solver(c.row_ptr, c.col_idx, v, host_only=1, restriction=L.RESTRICT_INJECTION))
    assert "ILU" in msg


def test_host_only_handle_refuses_device_calls():
    c = J.small(3, 3, 2)
    s = host_solver(c)
    x, y = np.zeros(c.n_dof), np.zeros(c.n_dof)
    assert L.lib().cptr_apply(s._h, L._ptr(x), L._ptr(y), None) == L.CPTR_E_STATE
    assert "host-only" in L.lib().cptr_last_error(s._h).decode()


def test_host_only_handle_forms_products_on_the_host():
    c = J.small(8, 6, 4)
    s = host_solver(c)
    rows, _ = s.hierarchy()
    sites = s.export("SETUP_SITES", 0, 15, np.int32)
    # one aggressive level
    L_ = len(rows) - 1
    assert list(sites[:11]) == [0, L_, 0, L_ - 1, 0, L_, 0, 1, 0, 1, 0] and sites[11] >= L_ + 1 and sites[12] == 0
    assert list(sites[13:]) == [0, 0]  # one HMIS block: no blocked split


def test_coarsening_limit_reports_stall():
    c = J.small(6, 6, 4)
    # a two-level cap leaves a coarsest level far above the dense limit
    # only when the limit is tiny; max_levels=1 puts all rows in the dense solve
    s = L.Solver(c.row_ptr, c.col_idx, c.values, host_only=1, max_levels=1)
    rows, _ = s.hierarchy()
    assert len(rows) == 1 and rows[0] == 2 * c.n_cells


@pytest.mark.parametrize("case,maxd,levels", [("grid20x20x5", 0, 25), ("grid20x20x5", 50, 2),
                                               ("prism2000x5", 100, 3), ("grid12x1x1", 0, 1)])
def test_relaxed_coarsest_matches_oracle(case, maxd, levels):
    """A coarsest level above max_dense_coarse is smoothed, not factored: the
    library forms its l1 diagonal (and no LU) exactly as the oracle does with
    the same limit, on top of the same hierarchy."""
    c = J.by_name(case)
    h = O.Cptr(c.row_ptr, c.col_idx, c.values, max_dense=maxd, max_levels=levels)
    s = host_solver(c, max_dense_coarse=maxd, max_levels=levels)
    rows, _ = s.hierarchy()
    a = h.amg
    assert len(rows) == a.nlevels and rows[-1] > maxd
    last = a.nlevels - 1
    for l in range(a.nlevels):
        Al, Ao = s.level_matrix(l, "A"), a.A(l)
        assert np.array_equal(Al.indices, Ao.indices) and np.array_equal(Al.data, Ao.data)
    dv = s.export("DINV", last, int(rows[last]))
    assert np.array_equal(dv, a.dinv(last))


def test_stalled_coarsening_is_relaxed():
    """On the 250x250x2 grid no row of level 0 passes the row-sum test, so the
    strength graph is empty, the first split has no C point and level 0 is the
    coarsest with 250,000 rows: it is smoothed (the setup used to refuse it
    with CPTR_E_SINGULAR_COARSE)."""
    c = J.by_name("grid250x250x2")
    s = host_solver(c)
    rows, _ = s.hierarchy()
    assert list(rows) == [2 * c.n_cells]
    dv = s.export("DINV", 0, int(rows[0]))
    assert np.all(np.isfinite(dv)) and np.all(dv != 0.0)


def test_fp32_preconditioner_options():
    """Mixed precision is a setup option, valid with every sweep schedule; an
    unknown precision is rejected before any work."""
    c = J.by_name("grid7x5x3")
    for sweep in (L.ILU_SWEEP_LEVELS, L.ILU_SWEEP_ONE_LAUNCH, L.ILU_SWEEP_GRID):
        host_solver(c, ilu_sweep=sweep, precond_precision=L.PRECISION_FP32).close()
    with pytest.raises(L.CptrError):
        L.Solver(c.row_ptr, c.col_idx, c.values, host_only=1, precond_precision=7)
    # the host hierarchy does not depend on the precision
    a = host_solver(c, precond_precision=L.PRECISION_FP32)
    b = host_solver(c)
    assert np.array_equal(a.hierarchy()[0], b.hierarchy()[0])

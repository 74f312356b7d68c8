"""GPU checks of the boundary's options: more l1-Jacobi sweeps per level
(cptr_setup_opts.num_sweeps) against the oracle's V-cycle with the same
count, a coarsest level above the dense limit smoothed instead of factored
(max_dense_coarse, and a coarsening that stops at level 0), the Krylov space
allocated at setup (max_restart, flexible_space) and the sweeps' wait-limit
report (cptr_sweep_check).

Bars as in the parity tests: one application within 1e-10 relative of the
oracle, GMRES iterations within +-1 and the true residual at the tolerance.
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


@pytest.mark.parametrize("name,sweeps", [("grid20x20x5", 2), ("grid20x20x5", 3), ("grid33x17x2", 2),
                                         ("prism2000x5", 2), ("prism2000x5", 3)])
def test_num_sweeps_parity(name, sweeps):
    """num_sweeps = k: k sweeps x += D^-1 (b - A x) before (the first from
    x = 0) and after the coarse correction on every smoothed level; the first
    stage and the whole application match the oracle's V-cycle with k sweeps."""
    c = J.by_name(name)
    say(f"[sweeps] {name} num_sweeps={sweeps}")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values, num_sweeps=sweeps)
    r = np.random.default_rng(31).standard_normal(c.n_dof)
    x1o, zo = ref.stage1(r), ref.apply(r)
    with L.Solver(c.row_ptr, c.col_idx, c.values, num_sweeps=sweeps) as s:
        rd = dev(r)
        x1 = torch.empty_like(rd)
        z = torch.empty_like(rd)
        for _ in range(2):
            s.stage1(rd, x1)
            s.apply(rd, z)
            e1 = np.linalg.norm(host(x1) - x1o) / np.linalg.norm(x1o)
            ez = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
            assert e1 <= 1e-10 and ez <= 1e-10, (e1, ez)
        s.sweep_check()
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=30, rtol=c.tol)
    _, oinfo = ref.gmres(c.b, restart=30, rtol=c.tol)
    say(f"  gpu {info['iterations']} it, oracle {oinfo['iterations']} it")
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1


@pytest.mark.parametrize("name,sweeps,maxd,levels", [("grid20x20x5", 1, 0, 25), ("grid20x20x5", 2, 0, 25),
                                                     ("prism2000x5", 1, 100, 3), ("grid33x17x2", 2, 0, 25),
                                                     ("grid20x20x5", 1, 100, 1)])
def test_relaxed_coarsest_parity(name, sweeps, maxd, levels):
    """max_dense_coarse below the coarsest level's size: that level gets
    num_sweeps sweeps before and after a zero coarse correction; the first
    stage, one application and the GMRES iterations match the oracle's
    V-cycle with the same limit."""
    c = J.by_name(name)
    say(f"[relaxed coarsest] {name} num_sweeps={sweeps} max_dense={maxd} max_levels={levels}")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values, num_sweeps=sweeps, max_dense=maxd, max_levels=levels)
    r = np.random.default_rng(33).standard_normal(c.n_dof)
    x1o, zo = ref.stage1(r), ref.apply(r)
    with L.Solver(c.row_ptr, c.col_idx, c.values, num_sweeps=sweeps, max_dense_coarse=maxd,
                  max_levels=levels) as s:
        rows, _ = s.hierarchy()
        assert rows[-1] > maxd
        rd = dev(r)
        x1 = torch.empty_like(rd)
        z = torch.empty_like(rd)
        s.stage1(rd, x1)
        s.apply(rd, z)
        e1 = np.linalg.norm(host(x1) - x1o) / np.linalg.norm(x1o)
        ez = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
        assert e1 <= 1e-10 and ez <= 1e-10, (e1, ez)
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=30, rtol=c.tol)
    _, oinfo = ref.gmres(c.b, restart=30, rtol=c.tol)
    say(f"  gpu {info['iterations']} it, oracle {oinfo['iterations']} it")
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1


@pytest.mark.parametrize("prec", [L.PRECISION_FP64, L.PRECISION_FP32])
def test_stalled_coarsening_solves(prec):
    """250x250x2: no strong link on level 0, so the hierarchy is level 0
    alone, 250,000 rows, smoothed rather than factored.  One application
    matches the oracle (1e-10 in FP64, 1e-3 with the FP32 preconditioner) and
    FGMRES converges in the oracle's iterations (+-1; +2 in FP32)."""
    c = J.by_name("grid250x250x2")
    say(f"[stalled coarsening] grid250x250x2 precision={prec}")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    r = np.random.default_rng(34).standard_normal(c.n_dof)
    zo = ref.apply(r)
    with L.Solver(c.row_ptr, c.col_idx, c.values, precond_precision=prec) as s:
        rows, _ = s.hierarchy()
        assert list(rows) == [2 * c.n_cells]
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        ez = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
        assert ez <= (1e-10 if prec == L.PRECISION_FP64 else 1e-3), ez
        b = dev(c.b)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=c.tol)
    _, oinfo = ref.gmres(c.b, restart=50, flexible=True, rtol=c.tol)
    say(f"  gpu {info['iterations']} it, oracle {oinfo['iterations']} it")
    slack = 1 if prec == L.PRECISION_FP64 else 2
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= slack


def test_num_sweeps_fp32():
    c = J.by_name("grid20x20x5")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values, num_sweeps=2)
    r = np.random.default_rng(32).standard_normal(c.n_dof)
    zo = ref.apply(r)
    with L.Solver(c.row_ptr, c.col_idx, c.values, num_sweeps=2, precond_precision=L.PRECISION_FP32) as s:
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        assert np.linalg.norm(host(z) - zo) <= 1e-3 * np.linalg.norm(zo)


def test_krylov_space_is_fixed_at_setup():
    """A solve never allocates: a restart above the handle's max_restart is
    refused, and so is a flexible solve without the Z vectors; the handle
    stays usable after both."""
    c = J.by_name("grid20x20x5")
    b = dev(c.b)
    with L.Solver(c.row_ptr, c.col_idx, c.values, max_restart=20, flexible_space=0) as s:
        x = torch.zeros_like(b)
        with pytest.raises(L.CptrError) as e:
            s.gmres_solve(b, x, restart=30, rtol=1e-8)
        assert e.value.code == L.CPTR_E_INVALID and "max_restart" in str(e.value)
        with pytest.raises(L.CptrError) as e:
            s.gmres_solve(b, x, restart=20, flexible=True, rtol=1e-8)
        assert e.value.code == L.CPTR_E_STATE
        info = s.gmres_solve(b, x, restart=20, rtol=1e-8)
        assert info["converged"]
        res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, host(x))) / np.linalg.norm(c.b)
        assert res <= 1e-8 * (1 + 1e-6)
    with L.Solver(c.row_ptr, c.col_idx, c.values, max_restart=64) as s:
        x = torch.zeros_like(b)
        assert s.gmres_solve(b, x, restart=64, flexible=True, rtol=1e-8)["converged"]


@pytest.mark.parametrize("name,mode", [("grid20x20x5", L.ILU_SWEEP_GRID), ("prism2000x5", L.ILU_SWEEP_ONE_LAUNCH),
                                       ("grid20x20x5", L.ILU_SWEEP_ONE_LAUNCH)])
def test_sweep_check_after_applies(name, mode):
    """Valid schedules never reach a wait bound: after several asynchronous
    applies the check reports success (and clears the flag)."""
    c = J.by_name(name)
    with L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=mode) as s:
        r = dev(np.random.default_rng(33).standard_normal(c.n_dof))
        z = torch.empty_like(r)
        for _ in range(4):
            s.apply(r, z)
            s.ilu_solve(r, z)
        s.sweep_check()
        s.sweep_check()

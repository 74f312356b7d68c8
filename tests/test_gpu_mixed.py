"""Mixed precision: the preconditioner (V-cycle operators and vectors, ILU(0)
factors and sweeps) in FP32 inside FP64 FGMRES; A, the restriction weights,
the coarsest dense solve, Arnoldi, Givens and the true residual stay FP64.

Bars.  One FP32 application against the FP64 oracle: relative 2-norm
difference at most 1e-3.  That bound comes from the arithmetic: every stored
operator and vector carries a relative rounding of 2^-24 (6e-8), and the
application chains about 2(L + 2) operator passes (V-cycle down and up) and
two triangular sweeps whose recurrences run over nx + ny + nz - 2 levels, so
with amplification by the ILU(0) factors' conditioning the FP32 result sits
near 1e-5 of the FP64 one (measured 2e-6 .. 2e-5); 1e-3 leaves two orders of
margin and still fails any indexing or type mistake, which shows up at O(1).
Whole solves reach the same true relative residual as FP64 (<= rtol) within
2 extra iterations of the oracle; the solution's difference from the oracle's
is reported and checked against the error the tolerance allows.
"""
import numpy as np
import pytest

import oracle as O
import paper_2308_11892_amd as L
from synth import jacobian as J

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FP32 = dict(precond_precision=L.PRECISION_FP32)


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name,sweep", [("grid20x20x5", L.ILU_SWEEP_AUTO), ("grid20x20x5", L.ILU_SWEEP_LEVELS),
                                        ("grid20x20x5", L.ILU_SWEEP_ONE_LAUNCH),
                                        ("grid33x17x2", L.ILU_SWEEP_AUTO), ("grid100x100x20", L.ILU_SWEEP_AUTO),
                                        ("grid100x100x20", L.ILU_SWEEP_LEVELS),
                                        ("prism2000x5", L.ILU_SWEEP_AUTO), ("prism2000x5", L.ILU_SWEEP_LEVELS)])
def test_fp32_apply_against_oracle(name, sweep):
    c = J.by_name(name)
    say(f"[fp32 apply] {name} sweep={sweep}")
    h = O.Cptr(c.row_ptr, c.col_idx, c.values)
    r = np.random.default_rng(3).standard_normal(c.n_dof)
    zo = h.apply(r)
    with L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=sweep, **FP32) as s:
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        zg = host(z)
        # the stages separately: M1^-1 and M2^-1
        x1 = torch.empty_like(z)
        s.stage1(dev(r), x1)
        x2 = torch.empty_like(z)
        s.ilu_solve(dev(r), x2)
        e1 = np.linalg.norm(host(x1) - h.stage1(r)) / np.linalg.norm(h.stage1(r))
        e2 = np.linalg.norm(host(x2) - h.ilu_solve(r)) / np.linalg.norm(h.ilu_solve(r))
    err = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
    say(f"[fp32 apply] {name}: apply {err:.2e} stage1 {e1:.2e} ilu {e2:.2e}")
    assert err <= 1e-3 and e1 <= 1e-3 and e2 <= 1e-3


def test_fp32_schedules_agree():
    """Grid, one-launch and per-level sweeps do the same FP32 arithmetic per
    row in a different order: they agree to a few FP32 roundings."""
    c = J.by_name("grid20x20x5")
    r = dev(np.random.default_rng(4).standard_normal(c.n_dof))
    out = []
    for sweep in (L.ILU_SWEEP_GRID, L.ILU_SWEEP_LEVELS, L.ILU_SWEEP_ONE_LAUNCH):
        with L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=sweep, **FP32) as s:
            z = torch.empty_like(r)
            s.apply(r, z)
            out.append(host(z))
    for o in out[1:]:
        d = np.linalg.norm(out[0] - o) / np.linalg.norm(o)
        say(f"[fp32 schedules] {d:.2e}")
        assert d <= 1e-5


@pytest.mark.parametrize("name,restart", [("grid20x20x5", 30), ("grid100x100x20", 50),
                                          ("grid100x100x20_pe1000", 50), ("prism10000x10", 50)])
def test_fp32_fgmres_reaches_tolerance(name, restart):
    c = J.by_name(name)
    say(f"[fp32 fgmres] {name}")
    xo, io = O.Cptr(c.row_ptr, c.col_idx, c.values).gmres(c.b, restart=restart, flexible=True, rtol=c.tol)
    with L.Solver(c.row_ptr, c.col_idx, c.values, **FP32) as s:
        x = torch.zeros(c.n_dof, dtype=torch.float64, device=DEV)
        info = s.gmres_solve(dev(c.b), x, restart=restart, flexible=True, rtol=c.tol)
        xg = host(x)
    rel = np.linalg.norm(c.b - J.bsr_matvec_plain(c.row_ptr, c.col_idx, c.values, xg)) / np.linalg.norm(c.b)
    dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    say(f"[fp32 fgmres] {name}: {info['iterations']} it (oracle {io['iterations']}), true rel res "
        f"{rel:.2e}, |x - x_oracle|/|x_oracle| = {dx:.2e}")
    assert info["converged"] and rel <= c.tol
    assert info["iterations"] <= io["iterations"] + 2
    # both solutions have residual <= tol; their difference is bounded by the
    # error that residual allows (measured well below 1e-3 on these systems)
    assert dx <= 1e-3


@pytest.mark.parametrize("name", ["grid20x20x5", "prism2000x5"])
def test_fp32_cpr_against_oracle(name):
    """The FP32 preconditioner with one elliptic unknown (CPR): one application
    against the FP64 oracle's CPR, and FGMRES to tolerance."""
    c = J.by_name(name)
    h = O.Cptr(c.row_ptr, c.col_idx, c.values, elliptic=(0,))
    r = np.random.default_rng(8).standard_normal(c.n_dof)
    zo = h.apply(r)
    with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=(0,), **FP32) as s:
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(dev(r), z)
        err = np.linalg.norm(host(z) - zo) / np.linalg.norm(zo)
        x = torch.zeros(c.n_dof, dtype=torch.float64, device=DEV)
        info = s.gmres_solve(dev(c.b), x, restart=30, flexible=True, rtol=1e-8)
        xg = host(x)
    _, io = h.gmres(c.b, restart=30, flexible=True, rtol=1e-8)
    rel = np.linalg.norm(c.b - J.bsr_matvec_plain(c.row_ptr, c.col_idx, c.values, xg)) / np.linalg.norm(c.b)
    say(f"[fp32 cpr] {name}: apply {err:.2e}; {info['iterations']} it (oracle {io['iterations']}), rel res {rel:.2e}")
    assert err <= 1e-3
    assert info["converged"] and rel <= 1e-8 and info["iterations"] <= io["iterations"] + 2

"""Full-size GPU parity on the 250x250x50 workload (3.125M cells, 9.375M DOF),
in the launch configuration the benchmark times (automatic sweep schedule =
tiled grid sweeps, FGMRES(50), rtol 1e-6).

The oracle runs the same seeded system on the host (about a minute): block
SpMV within a componentwise rounding bound, one CPTR application within 1e-10,
FGMRES iterations within +-1 and a true residual at or below 1e-6; the three
ILU sweep schedules agree with each other.
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


@pytest.fixture(scope="module")
def big():
    say("[fullsize] generating grid250x250x50")
    c = J.config3()
    say("[fullsize] oracle setup")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    say("[fullsize] library setup")
    s = L.Solver(c.row_ptr, c.col_idx, c.values)
    yield c, ref, s
    s.close()


def test_fullsize_uses_grid_sweeps(big):
    c, _, s = big
    assert tuple(s.export("SWEEP", 0, 4, np.int32)) == (L.ILU_SWEEP_GRID, 250, 250, 50)


def test_fullsize_spmv(big):
    c, _, s = big
    say("[fullsize] spmv")
    x = np.random.default_rng(1).standard_normal(c.n_dof)
    y = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
    s.spmv(torch.tensor(x, device=DEV), y)
    torch.cuda.synchronize()
    yo = O.bsr_spmv(c.row_ptr, c.col_idx, c.values, x)
    absA = O.bsr_spmv(c.row_ptr, c.col_idx, np.abs(c.values), np.abs(x))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-13 * absA + 1e-300)


def test_fullsize_apply(big):
    c, ref, s = big
    for seed in (2, 3):
        say(f"[fullsize] apply seed {seed}")
        r = np.random.default_rng(seed).standard_normal(c.n_dof)
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(torch.tensor(r, device=DEV), z)
        torch.cuda.synchronize()
        zo = ref.apply(r)
        zg = z.cpu().numpy()
        assert np.all(np.isfinite(zg))
        assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)


def test_fullsize_schedules_agree(big):
    c, _, s = big
    r = torch.tensor(np.random.default_rng(4).standard_normal(c.n_dof), device=DEV)
    z = torch.empty_like(r)
    s.apply(r, z)
    outs = []
    for mode in (L.ILU_SWEEP_ONE_LAUNCH, L.ILU_SWEEP_LEVELS):
        say(f"[fullsize] schedule {mode}")
        with L.Solver(c.row_ptr, c.col_idx, c.values, ilu_sweep=mode) as s2:
            z2 = torch.empty_like(r)
            s2.apply(r, z2)
            torch.cuda.synchronize()
            outs.append(z2)
    for z2 in outs:
        assert (torch.linalg.norm(z2 - z) / torch.linalg.norm(z)).item() <= 1e-13


def test_fullsize_fgmres(big):
    c, ref, s = big
    say("[fullsize] gpu FGMRES(50)")
    b = torch.tensor(c.b, device=DEV)
    x = torch.zeros_like(b)
    info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
    say(f"[fullsize] gpu {info['iterations']} it in {info['solve_s']:.3f} s; oracle FGMRES(50)")
    _, oinfo = ref.gmres(c.b, restart=50, flexible=True, rtol=1e-6)
    say(f"[fullsize] oracle {oinfo['iterations']} it")
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1
    xh = x.cpu().numpy()
    res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, xh)) / np.linalg.norm(c.b)
    assert res <= 1e-6

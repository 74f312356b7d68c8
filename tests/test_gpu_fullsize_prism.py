"""Full-size GPU parity on the unstructured workload: 50k Voronoi columns x 20
layers (1M cells, 3M DOF, 8.9M blocks) in reverse Cuthill-McKee order, with
the automatic sweep schedule (no grid structure, so the ILU(0) sweeps follow
the dependency levels of the RCM order), FGMRES(50), rtol 1e-6.

The oracle runs the same seeded system on the host: block SpMV within a
componentwise rounding bound, one CPTR application within 1e-10, FGMRES
iterations within +-1 and a true residual at or below 1e-6.
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
def mesh():
    say("[prism] generating prism50000x20")
    c = J.config2()
    say(f"[prism] {c.n_cells} cells, {c.nnzb} blocks; oracle setup")
    ref = O.Cptr(c.row_ptr, c.col_idx, c.values)
    say("[prism] library setup")
    s = L.Solver(c.row_ptr, c.col_idx, c.values)
    yield c, ref, s
    s.close()


def test_prism_schedule_and_levels(mesh):
    c, _, s = mesh
    used = s.export("SWEEP", 0, 4, np.int32)
    assert used[0] in (L.ILU_SWEEP_ONE_LAUNCH, L.ILU_SWEEP_LEVELS)
    nl = s.export("ILU_NLEVELS", 0, 2, np.int32)
    say(f"[prism] sweep schedule {used[0]}, ILU levels {tuple(nl)}")
    assert nl[0] > 1 and nl[1] > 1


def test_prism_spmv(mesh):
    c, _, s = mesh
    say("[prism] spmv")
    x = np.random.default_rng(1).standard_normal(c.n_dof)
    y = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
    s.spmv(torch.tensor(x, device=DEV), y)
    torch.cuda.synchronize()
    yo = O.bsr_spmv(c.row_ptr, c.col_idx, c.values, x)
    absA = O.bsr_spmv(c.row_ptr, c.col_idx, np.abs(c.values), np.abs(x))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-13 * absA + 1e-300)


def test_prism_apply(mesh):
    c, ref, s = mesh
    for seed in (2, 3):
        say(f"[prism] apply seed {seed}")
        r = np.random.default_rng(seed).standard_normal(c.n_dof)
        z = torch.empty(c.n_dof, dtype=torch.float64, device=DEV)
        s.apply(torch.tensor(r, device=DEV), z)
        torch.cuda.synchronize()
        zo = ref.apply(r)
        zg = z.cpu().numpy()
        assert np.all(np.isfinite(zg))
        assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)


def test_prism_fgmres(mesh):
    c, ref, s = mesh
    say("[prism] gpu FGMRES(50)")
    b = torch.tensor(c.b, device=DEV)
    x = torch.zeros_like(b)
    info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
    say(f"[prism] gpu {info['iterations']} it in {info['solve_s']:.3f} s; oracle FGMRES(50)")
    _, oinfo = ref.gmres(c.b, restart=50, flexible=True, rtol=1e-6)
    say(f"[prism] oracle {oinfo['iterations']} it")
    assert info["converged"] and abs(info["iterations"] - oinfo["iterations"]) <= 1
    xh = x.cpu().numpy()
    res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, xh)) / np.linalg.norm(c.b)
    assert res <= 1e-6

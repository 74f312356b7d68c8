"""cptr_gmres_solve_static (the entry point that allocates nothing: its
reduction scratch is a static device array) against cptr_gmres_solve,
through the C ABI.

Both run the same kernels in the same order on the same inputs, so the bar is
bit-identical solutions and equal iteration counts; each is also held to the
parity bar against the oracle (iterations within +-1, true residual at the
tolerance).  Two calls in a row, the second on a smaller system, show that the
shared array's leftover contents do not leak into the next call.
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


def _solve_both(name, restart, flexible, tol):
    c = J.by_name(name)
    say(f"[no-alloc] {name} restart={restart} flexible={flexible} tol={tol}")
    with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
        b = torch.tensor(c.b, device=DEV)
        xs = torch.zeros_like(b)
        info_s = s.gmres_solve(b, xs, static_scratch=True, restart=restart, flexible=flexible, rtol=tol)
        xd = torch.zeros_like(b)
        info_d = s.gmres_solve(b, xd, restart=restart, flexible=flexible, rtol=tol)
        torch.cuda.synchronize()
    _, oinfo = O.Cptr(c.row_ptr, c.col_idx, c.values).gmres(c.b, restart=restart, flexible=flexible, rtol=tol)
    say(f"  static {info_s['iterations']} it, handle scratch {info_d['iterations']} it, "
        f"oracle {oinfo['iterations']} it")
    assert info_s["converged"] and info_s["iterations"] == info_d["iterations"]
    assert info_s["rel_res_true"] == info_d["rel_res_true"]
    assert torch.equal(xs, xd)
    assert abs(info_s["iterations"] - oinfo["iterations"]) <= 1
    x = xs.cpu().numpy()
    res = np.linalg.norm(c.b - O.bsr_spmv(c.row_ptr, c.col_idx, c.values, x)) / np.linalg.norm(c.b)
    assert res <= tol * (1 + 1e-6)


def test_static_scratch_solve_equals_handle_scratch_solve_twice():
    # the larger system first, then a smaller one on the same shared array
    _solve_both("grid20x20x5", 30, True, 1e-8)
    _solve_both("grid7x5x3", 20, False, 1e-8)


def test_static_scratch_solve_unstructured():
    _solve_both("prism2000x5", 50, True, 1e-6)


def test_static_scratch_solve_rejects_profiling():
    c = J.by_name("grid7x5x3")
    with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
        b = torch.tensor(c.b, device=DEV)
        x = torch.zeros_like(b)
        with pytest.raises(L.CptrError) as e:
            s.gmres_solve(b, x, static_scratch=True, profile=1)
        assert e.value.code == L.CPTR_E_INVALID
        with pytest.raises(L.CptrError) as e:
            s.gmres_solve(b, x, static_scratch=True, restart=51)
        assert e.value.code == L.CPTR_E_INVALID and "max_restart" in str(e.value)

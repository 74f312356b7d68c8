"""The solve server on the GPU (continuous admission, HBM-budgeted).

Bars:
- every served solution is compared with the oracle's FP64 solution of the
  same system at the same tolerance, at the bars of the mixed-precision tests
  (the server runs the FP32 preconditioner inside FP64 FGMRES): relative
  difference <= 1e-3, iterations <= oracle + 2, true relative residual at or
  below the request's tolerance;
- each request's solution is bit-identical alone (one slot), in the mix (four
  slots, all requests submitted at once) and through a plain Solver handle --
  all kernels are deterministic and a request only touches its own memory;
- requests of the serving stream's grid sizes (40x40x10 and 80x80x20 in the
  mix, 160x160x20 and 200x200x40 alone) match the oracle the same way;
- requests admitted together run at the same time (their device intervals
  overlap);
- the HBM reservation of admitted requests never exceeds the budget; a
  request larger than the whole budget fails with CPTR_E_NOMEM without
  disturbing the others.
"""
import time

import numpy as np
import pytest

import oracle as O
import paper_2308_11892_amd as L
from synth import jacobian as J

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

SEED = J.SEED_BASE * 1000
# (workload, tolerance): small systems and two of the serving stream's grid
# sizes (the 100x100x20 generator at 40x40x10 and 80x80x20, own seeds)
MIX = [("grid12x10x4", 1e-6), ("serve40x40x10", 1e-4), ("grid30x20x6", 1e-6), ("prism300x4", 1e-6),
       ("grid16x16x8", 1e-4), ("serve80x80x20", 1e-6)]
# the elliptic set of each request: CPTR ({p, T}) except one CPR request ({p})
ELL = [(0, 1), (0, 1), (0, 1), (0, 1), (0,), (0, 1)]
SOLVE = dict(restart=30, flexible=True, max_iter=200)


def say(*a):
    print(*a, flush=True)


def case(name, tol=1e-6, k=0):
    if name.startswith("serve"):
        grid = tuple(int(v) for v in name[5:].split("x"))
        return J.serving_case(grid, tol, SEED + k)
    return J.by_name(name)


@pytest.fixture(scope="module")
def cases():
    return {n: case(n, tol, k) for k, (n, tol) in enumerate(MIX)}


def _rel_res(c, x):
    return np.linalg.norm(c.b - J.bsr_matvec_plain(c.row_ptr, c.col_idx, c.values, x)) / np.linalg.norm(c.b)


def _oracle(c, tol, ell=(0, 1)):
    return O.Cptr(c.row_ptr, c.col_idx, c.values, elliptic=ell).gmres(c.b, rtol=tol, **SOLVE)


def _check_against_oracle(name, c, tol, x, info, ref):
    xo, oinfo = ref
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    rr = _rel_res(c, x)
    say(f"[serve] {name} tol {tol}: {info['iterations']} it (oracle {oinfo['iterations']}), "
        f"rel diff to the oracle {rel:.2e}, rel res {rr:.2e}")
    assert info["status"] == L.CPTR_OK, info
    assert info["iterations"] <= oinfo["iterations"] + 2, (info, oinfo)
    assert rel <= 1e-3, rel
    assert rr <= tol


def _direct(c, tol, ell=(0, 1)):
    with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=ell, precond_precision=L.PRECISION_FP32) as s:
        b = torch.tensor(c.b, device=DEV)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, rtol=tol, **SOLVE)
        torch.cuda.synchronize()
        return x.cpu().numpy(), info


def test_same_result_alone_in_the_mix_direct_and_oracle(cases):
    say("[serve] oracle solves")
    refs = [_oracle(cases[n], tol, ell) for (n, tol), ell in zip(MIX, ELL)]
    say("[serve] direct solves")
    direct = [_direct(cases[n], tol, ell) for (n, tol), ell in zip(MIX, ELL)]
    say("[serve] one slot, one request at a time")
    alone = []
    with L.Server(max_inflight=1, setup_workers=1, hbm_budget_bytes=4 << 30) as sv:
        for (n, tol), ell in zip(MIX, ELL):
            c = cases[n]
            alone.append(sv.wait(sv.submit(c.row_ptr, c.col_idx, c.values, c.b, elliptic=ell, rtol=tol,
                                           **SOLVE)))
    say("[serve] four slots, all submitted at once")
    with L.Server(max_inflight=4, setup_workers=3, hbm_budget_bytes=4 << 30) as sv:
        ids = [sv.submit(cases[n].row_ptr, cases[n].col_idx, cases[n].values, cases[n].b, elliptic=ell,
                         rtol=tol, **SOLVE)
               for (n, tol), ell in zip(MIX, ELL)]
        mix = [sv.wait(i) for i in ids]
        st = sv.stats()
    say(f"[serve] stats {st}")
    assert st["completed"] == len(MIX) and st["failed"] == 0 and st["peak_inflight"] >= 1
    for (n, tol), (xd, di), (xa, ia), (xm, im), ref in zip(MIX, direct, alone, mix, refs):
        c = cases[n]
        assert ia["status"] == L.CPTR_OK and im["status"] == L.CPTR_OK, (ia, im)
        assert ia["iterations"] == im["iterations"] == di["iterations"], (n, ia, im, di)
        assert np.array_equal(xa, xm) and np.array_equal(xa, xd), n
        _check_against_oracle(n, c, tol, xm, im, ref)
        say(f"[serve] {n}: latency {im['latency_s'] * 1e3:.1f} ms, {im['device_bytes'] / 2**20:.1f} MiB")
        parts = im["queue_s"] + im["host_setup_s"] + im["admit_wait_s"] + im["device_setup_s"] + im["solve_s"]
        assert abs(parts - im["latency_s"]) <= 1e-6 + 1e-9 * im["latency_s"]


@pytest.mark.parametrize("grid,tol", [((160, 160, 20), 1e-6), ((200, 200, 40), 1e-4)])
def test_large_serving_sizes_match_the_oracle(grid, tol):
    """The two largest grid sizes of the serving stream, one request each."""
    c = J.serving_case(grid, tol, SEED + 100 + grid[0])
    say(f"[serve] {c.name}: {c.n_cells} cells")
    with L.Server(max_inflight=1, setup_workers=1, hbm_budget_bytes=16 << 30) as sv:
        x, info = sv.wait(sv.submit(c.row_ptr, c.col_idx, c.values, c.b, rtol=tol, **SOLVE))
    say(f"[serve] {c.name}: latency {info['latency_s'] * 1e3:.0f} ms (host setup "
        f"{info['host_setup_s'] * 1e3:.0f}, device setup {info['device_setup_s'] * 1e3:.0f}, "
        f"solve {info['solve_s'] * 1e3:.0f})")
    _check_against_oracle(c.name, c, tol, x, info, _oracle(c, tol))


def test_requests_admitted_together_overlap_on_the_device():
    """Four requests of one size (80x80x20, own seeds) submitted at once with
    four setup workers become ready together; with four slots at least two
    are in flight at once and their device intervals (admission to solution
    on the host) overlap.  Each still matches the oracle."""
    reqs = [J.serving_case((80, 80, 20), 1e-6, SEED + 200 + k) for k in range(4)]
    with L.Server(max_inflight=4, setup_workers=4, hbm_budget_bytes=8 << 30) as sv:
        ids = [sv.submit(c.row_ptr, c.col_idx, c.values, c.b, rtol=1e-6, **SOLVE) for c in reqs]
        outs = [sv.wait(i) for i in ids]
        st = sv.stats()
    spans = sorted((o[1]["admitted_at_s"], o[1]["done_at_s"]) for o in outs)
    say(f"[serve] peak in flight {st['peak_inflight']}; device intervals (s) "
        + ", ".join(f"[{a:.3f}, {b:.3f}]" for a, b in spans))
    assert st["peak_inflight"] >= 2
    assert any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))
    for c, (x, info) in zip(reqs, outs):
        _check_against_oracle(c.name, c, 1e-6, x, info, _oracle(c, 1e-6))


def test_admission_respects_the_hbm_budget(cases):
    c = cases["grid30x20x6"]
    with L.Server(max_inflight=1, hbm_budget_bytes=1 << 30) as sv:
        x0, i0 = sv.wait(sv.submit(c.row_ptr, c.col_idx, c.values, c.b, rtol=1e-6, **SOLVE))
    B = i0["device_bytes"]
    say(f"[serve] footprint of {c.name}: {B} bytes")
    assert B > 0
    for k in (1, 2):
        budget = int((k + 0.5) * B)
        with L.Server(max_inflight=4, setup_workers=4, hbm_budget_bytes=budget) as sv:
            ids = [sv.submit(c.row_ptr, c.col_idx, c.values, c.b, rtol=1e-6, **SOLVE) for _ in range(6)]
            outs = [sv.wait(i) for i in ids]
            st = sv.stats()
        say(f"[serve] budget {k}.5 x footprint: {st}")
        assert st["peak_reserved_bytes"] <= st["hbm_budget_bytes"]
        assert 1 <= st["peak_inflight"] <= k
        for x, info in outs:
            assert info["status"] == L.CPTR_OK and np.array_equal(x, x0)


def test_request_larger_than_the_budget_fails_alone(cases):
    small, big = cases["grid12x10x4"], cases["grid30x20x6"]
    with L.Server(max_inflight=1, hbm_budget_bytes=1 << 30) as sv:
        _, i_small = sv.wait(sv.submit(small.row_ptr, small.col_idx, small.values, small.b, rtol=1e-6, **SOLVE))
    budget = int(1.2 * i_small["device_bytes"])
    with L.Server(max_inflight=2, hbm_budget_bytes=budget) as sv:
        ib = sv.submit(big.row_ptr, big.col_idx, big.values, big.b, rtol=1e-6, **SOLVE)
        is_ = sv.submit(small.row_ptr, small.col_idx, small.values, small.b, rtol=1e-6, **SOLVE)
        xb, infob = sv.wait(ib)
        xs, infos = sv.wait(is_)
    assert xb is None and infob["status"] == L.CPTR_E_NOMEM and "budget" in infob["error"]
    assert infos["status"] == L.CPTR_OK and _rel_res(small, xs) <= 1e-6


def test_poisson_arrivals_report_latencies(cases):
    """Requests arriving while others run are admitted as slots free up."""
    rng = np.random.default_rng(11892000)
    with L.Server(max_inflight=3, setup_workers=2, hbm_budget_bytes=2 << 30) as sv:
        ids = []
        for k in range(10):
            n, tol = MIX[int(rng.integers(len(MIX)))]
            c = cases[n]
            ids.append((n, tol, sv.submit(c.row_ptr, c.col_idx, c.values, c.b, rtol=tol, **SOLVE)))
            time.sleep(float(rng.exponential(0.02)))
        lat = []
        for n, tol, i in ids:
            x, info = sv.wait(i)
            assert info["status"] == L.CPTR_OK and _rel_res(cases[n], x) <= tol
            lat.append(info["latency_s"])
        st = sv.stats()
    p50, p99 = np.percentile(lat, 50), np.percentile(lat, 99)
    say(f"[serve] 10 requests: p50 {p50 * 1e3:.1f} ms, p99 {p99 * 1e3:.1f} ms, peak in flight {st['peak_inflight']}")
    assert st["completed"] == 10 and 0 < p50 <= p99

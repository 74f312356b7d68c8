"""The solve server on the GPU (continuous admission, HBM-budgeted).

Bars: every request's solution is bit-identical alone (one slot), in the mix
(four slots, all requests submitted at once) and through a plain Solver
handle -- all kernels are deterministic and a request only touches its own
memory -- with the true relative residual at or below its tolerance; the
HBM reservation of admitted requests never exceeds the budget; a request
larger than the whole budget fails with CPTR_E_NOMEM without disturbing the
others.
"""
import time

import numpy as np
import pytest

import paper_2308_11892_amd as L
from synth import jacobian as J

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (workload, tolerance): the serving mix at oracle-friendly sizes
MIX = [("grid12x10x4", 1e-6), ("grid20x20x5", 1e-4), ("grid30x20x6", 1e-6), ("prism300x4", 1e-6),
       ("grid16x16x8", 1e-4), ("grid20x20x5", 1e-6)]
# the elliptic set of each request: CPTR ({p, T}) except one CPR request ({p})
ELL = [(0, 1), (0, 1), (0, 1), (0, 1), (0,), (0, 1)]
SOLVE = dict(restart=30, flexible=True, max_iter=200)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cases():
    return {n: J.by_name(n) for n, _ in MIX}


def _rel_res(c, x):
    return np.linalg.norm(c.b - J.bsr_matvec_plain(c.row_ptr, c.col_idx, c.values, x)) / np.linalg.norm(c.b)


def _direct(c, tol, ell=(0, 1)):
    with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=ell, precond_precision=L.PRECISION_FP32) as s:
        b = torch.tensor(c.b, device=DEV)
        x = torch.zeros_like(b)
        info = s.gmres_solve(b, x, rtol=tol, **SOLVE)
        torch.cuda.synchronize()
        return x.cpu().numpy(), info


def test_same_result_alone_in_the_mix_and_direct(cases):
    say("[serve] direct solves")
    direct = [_direct(cases[n], tol, ell) for (n, tol), ell in zip(MIX, ELL)]
    say("[serve] one slot, one request at a time")
    alone = []
    with L.Server(max_inflight=1, setup_workers=1, hbm_budget_bytes=2 << 30) as sv:
        for (n, tol), ell in zip(MIX, ELL):
            c = cases[n]
            alone.append(sv.wait(sv.submit(c.row_ptr, c.col_idx, c.values, c.b, elliptic=ell, rtol=tol,
                                           **SOLVE)))
    say("[serve] four slots, all submitted at once")
    with L.Server(max_inflight=4, setup_workers=3, hbm_budget_bytes=2 << 30) as sv:
        ids = [sv.submit(cases[n].row_ptr, cases[n].col_idx, cases[n].values, cases[n].b, elliptic=ell,
                         rtol=tol, **SOLVE)
               for (n, tol), ell in zip(MIX, ELL)]
        mix = [sv.wait(i) for i in ids]
        st = sv.stats()
    say(f"[serve] stats {st}")
    assert st["completed"] == len(MIX) and st["failed"] == 0 and st["peak_inflight"] >= 1
    for (n, tol), (xd, di), (xa, ia), (xm, im) in zip(MIX, direct, alone, mix):
        c = cases[n]
        assert ia["status"] == L.CPTR_OK and im["status"] == L.CPTR_OK, (ia, im)
        assert ia["iterations"] == im["iterations"] == di["iterations"], (n, ia, im, di)
        assert np.array_equal(xa, xm) and np.array_equal(xa, xd), n
        rr = _rel_res(c, xm)
        say(f"[serve] {n} tol {tol}: {im['iterations']} it, rel res {rr:.2e}, "
            f"latency {im['latency_s'] * 1e3:.1f} ms, {im['device_bytes'] / 2**20:.1f} MiB")
        assert rr <= tol
        parts = im["queue_s"] + im["host_setup_s"] + im["admit_wait_s"] + im["device_setup_s"] + im["solve_s"]
        assert abs(parts - im["latency_s"]) <= 1e-6 + 1e-9 * im["latency_s"]


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

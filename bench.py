#!/usr/bin/env python3
"""CPTR-preconditioned FGMRES benchmark on one MI355X.

One step = one full FGMRES(50) solve to a relative residual of 1e-6 of the
synthetic thermal Jacobian on the 250x250x50 grid (3.125M cells, 9.375M DOF),
FP64 throughout, right-hand side already resident in HBM.  Every step runs
the whole hot path: block SpMV, quasi-IMPES restriction, one system-AMG
V-cycle, the stage-two residual, the ILU(0) sweeps and the Arnoldi
orthogonalisation.

Prints one JSON line: DOF-iterations per second over the timed steps, the
time to tolerance, a roofline entry for the dominant single-kernel phase
(HIP events on the solve stream, algorithmic bytes per launch) and the CPU
oracle timed on a bounded slab of the same generator.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def phase_bytes(c, rows, nnz, ne, grid, tail=0):
    """Algorithmic bytes per launch of each timed phase: the values a phase must
    read and write once (FP64 values, int32 indices where an index array is
    part of the format).  On a detected grid the ILU sweeps carry no indices.
    With a dense bottom of the V-cycle at level `tail`, the levels from there
    down are one read of its n x n operator (and its vectors)."""
    nc, nnzb, N = c.n_cells, c.nnzb, c.n_dof
    n0 = ne * nc
    out = {}
    out["spmv"] = 76 * nnzb + 4 * (nc + 1) + 16 * N
    # r and W in; b0, and the pre-smoothed x0 = D^-1 b0 (with D^-1 read), out
    out["restrict"] = 8 * N + 8 * 2 * nc + 8 * n0 + 16 * n0
    a0 = (8 * ne * ne + 4) * nnzb                     # Ahat blocks + column indices
    p0 = 12 * 4 * n0                                  # P_0 / R_0: at most 4 entries per row
    # level 0: (residual after zero-start smoothing + restriction) and
    # (prolongation + post-smoothing), timed as two launches of the phase
    out["vcycle_l0"] = ((a0 + 8 * 3 * n0 + 8 * n0) + (p0 + 8 * n0)
                        + (p0 + 8 * 3 * n0) + (a0 + 8 * 4 * n0)) / 2
    out["stage2_resid"] = (8 * 3 * ne + 4) * nnzb + 8 * n0 + 16 * N
    nl = (nnzb - nc) // 2
    if grid:
        out["ilu_fwd"] = 72 * nl + 24 * nc + 24 * nc
        out["ilu_bwd"] = 72 * nl + 72 * nc + 24 * nc + 8 * ne * nc + 24 * nc
    else:
        out["ilu_fwd"] = 76 * nl + 4 * nc + 16 * N
        out["ilu_bwd"] = 76 * nl + 72 * nc + 4 * nc + 24 * N + 8 * n0
    coarse = 0
    for l in range(1, tail if tail > 0 else len(rows)):
        coarse += 2 * 12 * nnz[l] + 8 * 6 * rows[l]
    if tail > 0:
        coarse += 8 * rows[tail] * rows[tail] + 16 * rows[tail]
    out["vcycle_coarse"] = coarse
    return out


KERNEL_OF_PHASE = {"spmv": "k_bsr3_spmv", "restrict": "k_l0_restrict",
                   "stage2_resid": "k_stage2_grid", "ilu_fwd": "k_ilu_grid<true>",
                   "ilu_bwd": "k_ilu_grid<false>"}


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_grid250x250x50.md")
    src = os.path.join(ROOT, "paper_2308_11892_amd", "csrc", "kernels.hip")
    try:
        m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
        table = json.loads(m.group(1))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, AttributeError, ValueError):
        return None
    if table.get("kernels_sha256") != sha:
        return None
    return table["bytes_per_launch"].get(kernel)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _copy_bandwidth_gbs(mib=1024, reps=5):
    """Attainable host memory bandwidth: the median of `reps` single-thread
    numpy copies of `mib` MiB (read + write bytes per second)."""
    import numpy as np
    a = np.ones(mib * (1 << 20) // 8)
    b = np.empty_like(a)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        np.copyto(b, a)
        ts.append(time.perf_counter() - t0)
    return 2 * a.nbytes / float(np.median(ts)) / 1e9


def run_cpu_baseline(c, restart, reps=5):
    """The oracle as it stands (plain sequential C, one thread) on the same
    system: the median of `reps` FGMRES solves after one untimed warm-up is
    the value; its SpMV, one preconditioner application and the ILU(0)
    solve are timed beside (median of 5 each).  Setup is timed once, apart."""
    import numpy as np
    import oracle as O
    t0 = time.perf_counter()
    h = O.Cptr(c.row_ptr, c.col_idx, c.values)
    t_setup = time.perf_counter() - t0
    xo, info = h.gmres(c.b, restart=restart, flexible=True, rtol=c.tol)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        xo, info = h.gmres(c.b, restart=restart, flexible=True, rtol=c.tol)
        ts.append(time.perf_counter() - t0)
    t_solve = float(np.median(ts))
    r = np.random.default_rng(5).standard_normal(c.n_dof)
    kern = {}
    for name, fn in (("spmv", h.spmv), ("apply", h.apply), ("ilu_fwd_bwd", h.ilu_solve),
                     ("stage1", h.stage1)):
        kt = []
        for _ in range(5):
            t0 = time.perf_counter()
            fn(r)
            kt.append(time.perf_counter() - t0)
        kern[name] = round(float(np.median(kt)) * 1e3, 3)
    v = c.n_dof * info["iterations"] / t_solve
    return dict(value=v, unit="DOF-iter/s", cores=1, kind="oracle",
                sample=(f"median of {reps} oracle FGMRES({restart}) solves to {c.tol:g} of the same "
                        f"{c.name} system ({c.n_dof} DOF) after one warm-up, one thread: "
                        f"{info['iterations']} iterations in {t_solve:.2f} s (runs "
                        + ", ".join(f"{t:.2f}" for t in ts) + f" s); oracle setup {t_setup:.2f} s not in value"),
                threads=1, cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
                copy_bandwidth_gbs=round(_copy_bandwidth_gbs(), 1),
                kernel_ms=kern, setup_s=round(t_setup, 2), solve_s_runs=[round(t, 3) for t in ts],
                iterations=info["iterations"], x=xo)


def _make_request(spec):
    from synth import jacobian as J
    _, grid, tol, seed = spec
    return J.serving_case(grid, tol, seed)


def generate_requests(n, rate):
    """The serving stream's Jacobians, generated in forked worker processes
    (call before this process touches the GPU)."""
    import multiprocessing as mp
    from synth import jacobian as J
    stream = J.serving_stream(n, rate=rate)
    log(f"serving: generating {len(stream)} requests")
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        cases = pool.map(_make_request, stream, chunksize=1)
    return stream, cases


def serve_stream(stream, cases, rate, slots, setup_workers, setup_threads, verbose=True):
    """Submit the requests at their Poisson arrival times to a solve server
    (mixed-precision FGMRES(50)) and wait for all of them.  Returns the
    serving summary: solves/s over the makespan, p50/p99 latency, the median
    latency split, and whether the offered rate was sustained."""
    import threading

    import numpy as np
    import paper_2308_11892_amd as L
    from synth import jacobian as J

    cells = [c.n_cells for c in cases]
    log(f"serving: {len(cases)} requests, {sum(cells)} cells in total; starting the server")
    t_create = time.perf_counter()  # the server's clock origin (its *_at_s times), within microseconds
    sv = L.Server(max_inflight=slots, setup_workers=setup_workers,
                  setup_threads=setup_threads, hbm_budget_bytes=64 << 30)
    ids = [None] * len(stream)
    t0 = time.perf_counter()

    def submitter():
        for r, (ta, grid, tol, seed) in enumerate(stream):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            c = cases[r]
            ids[r] = sv.submit(c.row_ptr, c.col_idx, c.values, c.b, rtol=tol, restart=50, flexible=True,
                               max_iter=200)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    outs = [sv.wait(rid) for rid in ids]
    # the last solution back on the host, on this process's clock (checking
    # the solutions below is not part of the serving time)
    t_end = t_create + max(info["done_at_s"] for _, info in outs)
    res = []
    for r, (x, info) in enumerate(outs):
        c = cases[r]
        rr = float("nan") if x is None else float(
            np.linalg.norm(c.b - J.bsr_matvec_plain(c.row_ptr, c.col_idx, c.values, x)) / np.linalg.norm(c.b))
        res.append((info, rr, stream[r][2]))
        if verbose:
            log(f"request {r} {c.name} tol {stream[r][2]:g}: status {info['status']} {info['iterations']} it "
                f"rel res {rr:.2e} latency {info['latency_s'] * 1e3:.0f} ms (queue {info['queue_s'] * 1e3:.0f}, "
                f"host setup {info['host_setup_s'] * 1e3:.0f}, admit {info['admit_wait_s'] * 1e3:.0f}, "
                f"device setup {info['device_setup_s'] * 1e3:.0f}, solve {info['solve_s'] * 1e3:.0f})")
    st = sv.stats()
    sv.close()
    ok = [i for i, rr, tol in res if i["status"] >= 0 and rr <= tol]
    lat = np.array([i["latency_s"] for i, _, _ in res])
    med = lambda k: float(np.median([i[k] for i, _, _ in res]))
    span = stream[-1][0] - stream[0][0]
    sps = len(ok) / (t_end - t0)
    return {
        "requests": len(res), "converged_within_tol": len(ok),
        "offered_rate_per_s": rate, "arrival_span_s": round(span, 3),
        "solves_per_s": sps, "makespan_s": t_end - t0,
        # the offered rate is sustained when completions keep up with it
        "sustained": bool(sps >= 0.9 * rate and len(ok) == len(res)),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "median_ms": {k[:-2]: med(k) * 1e3 for k in ("queue_s", "host_setup_s", "admit_wait_s",
                                                       "device_setup_s", "solve_s")},
        "peak_inflight": st["peak_inflight"], "peak_reserved_gib": st["peak_reserved_bytes"] / 2**30,
        "hbm_budget_gib": st["hbm_budget_bytes"] / 2**30,
        "dtype": "f32 preconditioner, f64 Krylov",
        "workload": f"{len(res)} Poisson arrivals at {rate:g}/s, grids 40x40x10/80x80x20/160x160x20/"
                    "200x200x40 (100x100x20 generator, own seeds), tol 1e-4 or 1e-6, FGMRES(50)",
        "slots": slots, "setup_workers": setup_workers, "setup_threads": setup_threads,
    }


def run_serving(args):
    """Serving alone (--serve N): one JSON line with solves/s and p50/p99."""
    import torch
    stream, cases = generate_requests(args.serve, args.rate)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    out = serve_stream(stream, cases, args.rate, args.slots, args.setup_workers, args.setup_threads)
    out.update({"metric": "CPTR-FGMRES serving: solves/s and p50/p99 solve latency",
                "value": out["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
                "data": "synthetic"})
    print(json.dumps(out), flush=True)


def run_unstructured(restart):
    """The 1M-cell Voronoi-prism mesh in RCM order (no grid structure: the
    one-launch level-scheduled sweeps): FP64 FGMRES(50) to 1e-6, iterations,
    time to tolerance (median of 3 solves), setup, and the phase times of one
    profiled solve."""
    import numpy as np
    import torch
    import paper_2308_11892_amd as L
    from synth import jacobian as J
    log("unstructured: generating prism50000x20")
    c = J.by_name("prism50000x20")
    b = torch.tensor(c.b, device="cuda:0")
    kw = dict(restart=restart, flexible=True, rtol=c.tol)
    out = {"workload": f"{c.name}: 50k-point Voronoi prisms x 20 layers in RCM order, "
                       f"{c.n_cells} cells, {c.n_dof} DOF, {c.nnzb} blocks, FGMRES({restart}), rtol {c.tol:g}"}
    for prec, key in ((L.PRECISION_FP64, "fp64"), (L.PRECISION_FP32, "fp32_preconditioner")):
        with L.Solver(c.row_ptr, c.col_idx, c.values, precond_precision=prec) as s:
            x = torch.zeros_like(b)
            info = s.gmres_solve(b, x, **kw)
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = s.gmres_solve(b, x, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            s.phase_times(reset=True)
            s.gmres_solve(b, torch.zeros_like(b), profile=True, **kw)
            ph = {k: round(ms / cnt, 4) for k, (ms, cnt) in s.phase_times(reset=True).items() if cnt}
            out[key] = {"iterations": info["iterations"], "converged": info["converged"],
                        "true_rel_res": info["rel_res_true"], "time_to_tol_ms": float(np.median(ts)) * 1e3,
                        "dof_iter_per_s": c.n_dof * info["iterations"] / float(np.median(ts)),
                        "setup_s": info["setup_s"], "phase_avg_ms": ph,
                        "sweep": ["auto", "levels", "one_launch", "grid"][int(s.export("SWEEP", 0, 4, np.int32)[0])]}
            log(f"unstructured {key}: {info['iterations']} it, {np.median(ts) * 1e3:.1f} ms; "
                f"ILU {ph.get('ilu_fwd', 0):.3f} + {ph.get('ilu_bwd', 0):.3f} ms per application")
    return out


def run_cpr_comparison():
    """FGMRES(50) iterations to 1e-6 with CPTR (elliptic set {p, T}) and CPR
    (elliptic set {p}) on the 100x100x20 generator over the Peclet sweep, at the
    configured time step (1 day) and at 30 days.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2308_11892_amd as L
    from synth import jacobian as J

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rows = []
    for days in (1, 30):
        for pe in (0.1, 10.0, 1000.0):
            c = J.cartesian("grid100x100x20", 100, 100, 20, seed=J.SEED_BASE + 1, sigma=1.0, corr=10,
                            n_wells=4, r_front=5.0, pe_target=pe, dt=86400.0 * days)
            b = torch.tensor(c.b, device="cuda:0")
            its = {}
            for name, ell in (("cptr", (0, 1)), ("cpr", (0,))):
                with L.Solver(c.row_ptr, c.col_idx, c.values, elliptic=ell) as s:
                    x = torch.zeros_like(b)
                    info = s.gmres_solve(b, x, restart=50, flexible=True, rtol=1e-6)
                    its[name] = info["iterations"] if info["converged"] else None
            log(f"dt {days} d, Pe {pe:g}: CPTR {its['cptr']} CPR {its['cpr']}")
            rows.append({"dt_days": days, "peclet": pe, "kappa": c.meta["kappa"], **its})
    print(json.dumps({"metric": "FGMRES(50) iterations to 1e-6, CPTR vs CPR", "unit": "iterations",
                      "higher_is_better": False, "data": "synthetic",
                      "config": {"workload": "grid100x100x20 Peclet sweep"}, "rows": rows}), flush=True)


def build_info():
    """Source revision and kernel source hash recorded by the build (the GPU
    box has no git metadata)."""
    try:
        return json.load(open(os.path.join(ROOT, "paper_2308_11892_amd", "build_info.json")))
    except (OSError, ValueError):
        return None


def run_setup_only(args):
    """N setups of the workload on the GPU (device handle, FP64), one JSON line
    with each one's wall time and CPTR_EXPORT_SETUP_TIMES steps."""
    import numpy as np
    import torch
    import paper_2308_11892_amd as L
    from synth import jacobian as J
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    c = J.by_name(args.workload)
    runs = []
    for k in range(args.setup_only):
        t0 = time.perf_counter()
        with L.Solver(c.row_ptr, c.col_idx, c.values) as s:
            steps = s.export("SETUP_TIMES", 0, 10)
            sites = s.export("SETUP_SITES", 0, 15, np.int32)
        wall = time.perf_counter() - t0
        runs.append({"wall_s": round(wall, 4), **{k2: round(float(v), 4) for k2, v in zip(L.SETUP_STEPS, steps)}})
        log(f"setup {k}: {wall:.3f} s")
    print(json.dumps({"workload": args.workload, "setups": runs,
                      "first_pass_share_on_device": int(sites[12]) / 1000.0,
                      "device_sites": [int(v) for v in sites[:12]]}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid250x250x50")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "both"], default="both",
                    help="fp64: the FP64 solve only; both: also the mixed-precision solve "
                         "(FP32 preconditioner inside FP64 FGMRES), reported beside it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (three times), the "
                         "reference dispatch for scaling HBM byte counters")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="instead of the solve benchmark, run the serving workload: N requests "
                         "of four grid sizes arriving as a Poisson stream, solved by the "
                         "solve server with the mixed-precision preconditioner")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: mean arrivals per second")
    ap.add_argument("--slots", type=int, default=4, help="serving: requests on the GPU at once")
    ap.add_argument("--setup-workers", type=int, default=16, help="serving: concurrent host setups")
    ap.add_argument("--setup-threads", type=int, default=0,
                    help="serving: threads per host setup (0: sized per request, 1 to 4)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the serving sub-object of the default run (0: none)")
    ap.add_argument("--no-unstructured", action="store_true",
                    help="leave out the unstructured (1M-cell prism mesh) sub-object")
    ap.add_argument("--warm-setups", type=int, default=3, metavar="N",
                    help="after the FP64 solves, N more setups of the workload (setup_warm_s)")
    ap.add_argument("--setup-only", type=int, default=0, metavar="N",
                    help="instead of the solve benchmark, run N setups of the workload (the first "
                         "a warm-up) and print their step times; for a kernel trace of the setup")
    ap.add_argument("--compare-cpr", action="store_true",
                    help="instead of the solve benchmark, compare CPTR with CPR (elliptic set {p}) "
                         "on the 100x100x20 Peclet sweep at time steps of 1 and 30 days")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is documented, not built)", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        run_serving(args)
        return
    if args.compare_cpr:
        run_cpr_comparison()
        return
    if args.setup_only:
        run_setup_only(args)
        return

    import numpy as np
    # the serving requests are generated in forked workers before this
    # process touches the GPU
    serve_reqs = generate_requests(args.serve_requests, args.rate) if args.serve_requests > 0 else None
    import torch
    import paper_2308_11892_amd as L
    from synth import jacobian as J

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    log(f"generating {args.workload}")
    c = J.by_name(args.workload)
    log(f"cells {c.n_cells} DOF {c.n_dof} blocks {c.nnzb}; setup")
    stream = torch.cuda.current_stream()
    s = L.Solver(c.row_ptr, c.col_idx, c.values)
    rows, nnz = s.hierarchy()
    sweep_mode = s.export("SWEEP", 0, 4, np.int32)
    setup_steps = {k: round(float(v), 4) for k, v in zip(L.SETUP_STEPS, s.export("SETUP_TIMES", 0, 10))}
    grid_sweeps = int(sweep_mode[0]) == L.ILU_SWEEP_GRID
    b = torch.tensor(c.b, device=dev)
    x = torch.zeros_like(b)
    kw = dict(restart=args.restart, flexible=True, rtol=c.tol)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB")
        del src, dst
    setup_s = None
    for w in range(args.warmup):
        info = s.gmres_solve(b, x, **kw)
        setup_s = info["setup_s"]
        log(f"warmup {w}: {info['iterations']} it, {info['solve_s']:.3f} s, rel res {info['rel_res_true']:.2e}")
    tail = int(s.export("DENSE_TAIL", 0, 2, np.int32)[0])
    pbytes = phase_bytes(c, list(rows), list(nnz), 2, grid_sweeps, tail)

    def phase_table():
        table = {}
        for name, (ms, cnt) in s.phase_times(reset=True).items():
            if cnt == 0:
                continue
            e = dict(total_ms=round(ms, 3), launches=cnt, avg_ms=ms / cnt)
            if name in pbytes:
                e["bytes_per_launch"] = int(pbytes[name])
                e["GBps"] = pbytes[name] / (ms / cnt) / 1e6
            table[name] = e
        return table

    # every phase timed (HIP events on the solve stream between phases) in
    # untimed solves; the timed solves then carry events around the dominant
    # single-kernel phase only, so the other phase boundaries add no gaps
    s.phase_times(reset=True)
    for k in range(args.steps):
        s.gmres_solve(b, x, profile=True, **kw)
    phases = phase_table()
    single = [p for p in KERNEL_OF_PHASE if p in phases]
    if not grid_sweeps:
        single = [p for p in single if not p.startswith("ilu")]
    dom = max(single, key=lambda p: phases[p]["total_ms"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    infos = []
    for k in range(args.steps):
        info = s.gmres_solve(b, x, profile=1 << (L.PHASES.index(dom) + 1), **kw)
        its.append(info["iterations"])
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for k, info in enumerate(infos):
        log(f"step {k}: {info['iterations']} it, {info['solve_s']:.3f} s, rel res {info['rel_res_true']:.2e}")
    dk = phase_table()[dom]
    setup_s = infos[0]["setup_s"]
    value = c.n_dof * sum(its) / dt
    kname = KERNEL_OF_PHASE[dom]
    if dom == "stage2_resid" and not grid_sweeps:
        kname = "k_stage2_resid"
    roof = dict(kernel=kname, phase=dom, bound="hbm", achieved=round(dk["GBps"], 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(dk["GBps"] / HBM_PEAK_GBS, 4),
                traffic=pmc_traffic(kname), bytes_per_launch=dk["bytes_per_launch"],
                avg_launch_ms=round(dk["avg_ms"], 4), launches_timed=dk["launches"])
    out = {
        "metric": "CPTR-FGMRES DOF-iter/s to 1e-6 relative residual",
        "value": value,
        "unit": "DOF-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} thermal TPFA Jacobian (3x3 blocks), "
                               f"FGMRES({args.restart}) + CPTR, rtol {c.tol:g}",
                   "cells": c.n_cells, "dof": c.n_dof, "nnz_blocks": c.nnzb,
                   "amg_levels": len(rows), "amg_rows": [int(r) for r in rows],
                   "amg_dense_tail_level": tail,
                   "ilu_sweep": ["auto", "levels", "one_launch", "grid"][int(sweep_mode[0])]},
        "iterations": its,
        "time_to_tol_s": dt / args.steps,
        "seed": int(c.meta["seed"]),
        "build": build_info(),
        "gpu": torch.cuda.get_device_name(0) + " " + getattr(torch.cuda.get_device_properties(0), "gcnArchName", ""),
        "setup_s": setup_s,
        "setup_steps_s": setup_steps,
        "roofline": roof,
        "phases": phases,
    }
    x64 = x.cpu().numpy()
    s.close()
    if args.warm_setups > 0:
        # setups after the first in the process (no one-time initialisation):
        # what each linear solve of a simulation pays
        log(f"{args.warm_setups} more setups")
        runs = []
        for k in range(args.warm_setups):
            t0 = time.perf_counter()
            with L.Solver(c.row_ptr, c.col_idx, c.values) as sw:
                total = float(sw.export("SETUP_TIMES", 0, 10)[L.SETUP_STEPS.index("total")])
            runs.append({"library_s": round(total, 4), "wall_s": round(time.perf_counter() - t0, 4)})
        out["setup_warm_s"] = {"median": float(np.median([r["library_s"] for r in runs])), "runs": runs,
                               "note": "setup_s is the first setup in the process (one-time initialisation "
                                       "included); these are the following ones"}
    x32h = None
    if args.precision == "both":
        log("mixed precision: FP32 preconditioner, FP64 FGMRES; setup")
        s32 = L.Solver(c.row_ptr, c.col_idx, c.values, precond_precision=L.PRECISION_FP32)
        x32 = torch.zeros_like(b)
        for w in range(args.warmup):
            s32.gmres_solve(b, x32, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its32, infos32 = [], []
        for k in range(args.steps):
            info = s32.gmres_solve(b, x32, **kw)
            its32.append(info["iterations"])
            infos32.append(info)
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t0
        for k, info in enumerate(infos32):
            log(f"fp32 step {k}: {info['iterations']} it, {info['solve_s']:.3f} s, rel res {info['rel_res_true']:.2e}")
        s32.phase_times(reset=True)
        x32p = torch.zeros_like(b)
        s32.gmres_solve(b, x32p, profile=True, **kw)
        ph32 = {k: round(ms / cnt, 4) for k, (ms, cnt) in s32.phase_times(reset=True).items() if cnt}
        x32h = x32.cpu().numpy()
        s32.close()
        nrm = lambda v: float(np.linalg.norm(v))
        out["mixed_precision"] = {
            "value": c.n_dof * sum(its32) / dt32, "unit": "DOF-iter/s",
            "dtype": "f32 preconditioner, f64 Krylov",
            "ms_per_step": dt32 / args.steps * 1e3, "time_to_tol_s": dt32 / args.steps,
            "iterations": its32, "true_rel_res": infos32[-1]["rel_res_true"],
            "speedup_time_to_tol_vs_fp64": dt / dt32,
            "rel_diff_vs_fp64_solution": nrm(x32h - x64) / nrm(x64),
            "rel_err_vs_exact": nrm(x32h - c.x_star) / nrm(c.x_star),
            "fp64_rel_err_vs_exact": nrm(x64 - c.x_star) / nrm(c.x_star),
            "phase_avg_ms": ph32}
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {c.name}")
        cb = run_cpu_baseline(c, args.restart)
        out["cpu_baseline"] = {k: v for k, v in cb.items() if k != "x"}
        xo = cb["x"]
        out["rel_diff_vs_oracle_solution"] = float(np.linalg.norm(x64 - xo) / np.linalg.norm(xo))
        if x32h is not None:
            out["mixed_precision"]["rel_diff_vs_oracle_solution"] = float(
                np.linalg.norm(x32h - xo) / np.linalg.norm(xo))
    if not args.no_unstructured:
        out["unstructured"] = run_unstructured(args.restart)
    if serve_reqs is not None:
        out["serving"] = serve_stream(*serve_reqs, args.rate, args.slots, args.setup_workers, args.setup_threads,
                                      verbose=False)
        sv = out["serving"]
        log(f"serving: {sv['solves_per_s']:.1f} solves/s over {sv['makespan_s']:.2f} s, p50 "
            f"{sv['p50_latency_ms']:.0f} ms, p99 {sv['p99_latency_ms']:.0f} ms, sustained {sv['sustained']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

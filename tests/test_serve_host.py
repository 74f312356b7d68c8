"""Host-side checks of the solve server: the HBM arena allocator (built with
g++ from its header, randomised against an ownership map) and the option
validation of cptr_server_create, which happens before any device call."""
import os
import subprocess

import pytest

import paper_2308_11892_amd as L

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2308_11892_amd", "csrc")


def test_arena_allocator(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-O1", "-std=c++17", f"-I{CSRC}", os.path.join(HERE, "cpp", "arena_check.cpp"),
                    "-o", exe, "-pthread"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout


@pytest.mark.parametrize("kw", [dict(max_inflight=0), dict(max_inflight=65), dict(setup_workers=0),
                                dict(hbm_budget_bytes=0), dict(device=-1), dict(host_only=1)])
def test_server_rejects_bad_options(kw):
    with pytest.raises(L.CptrError) as e:
        L.Server(**kw)
    assert e.value.code == L.CPTR_E_INVALID


def test_server_defaults():
    o = L.cptr_server_opts()
    L.lib().cptr_server_opts_default(o)
    assert (o.max_inflight, o.setup_workers, o.device) == (4, 8, 0)
    assert o.setup.setup_threads == 0  # sized per request
    assert o.hbm_budget_bytes == 16 << 30
    # requests run with the mixed-precision preconditioner by default
    assert o.setup.precond_precision == L.PRECISION_FP32 and o.setup.agg_levels == 1


def _device_plan(c, **kw):
    import numpy as np
    with L.Solver(c.row_ptr, c.col_idx, c.values, host_only=1, **kw) as s:
        buf = s.export("DEVICE_PLAN", 0, 1 << 14, np.int64)
    return [int(v) for v in buf[1:int(buf[0]) + 1]]


def test_device_plan_releases_only_what_it_allocated():
    """The recorded device build (the server's footprint measurement): every
    release names an earlier, not yet released allocation."""
    from synth import jacobian as J
    for name in ("grid30x20x6", "prism300x4"):
        plan = _device_plan(J.by_name(name), max_restart=30, precond_precision=L.PRECISION_FP32)
        live = set()
        n_alloc = 0
        for v in plan:
            if v > 0:
                assert v % 256 == 0
                live.add(n_alloc)
                n_alloc += 1
            else:
                k = -1 - v
                assert k in live
                live.remove(k)
        assert n_alloc > 10 and live


@pytest.mark.parametrize("part_blocks", [1024, 4096])
def test_admission_replay_never_fails_a_build(tmp_path, part_blocks):
    """The admission test's allocation sequence (six 30x20x6 requests, FP32
    preconditioner, FGMRES(30)) replayed through DevArena under ASan/UBSan,
    with 2000 random interleavings of the requests admitted together (one at
    1.5x the footprint, two at 2.5x), with the reduction partials of 1024
    and of 4096 workgroups.  No build ever finds the arena without a piece
    large enough, so that test never takes the failed-build path (the release
    of a failed build's memory)."""
    from synth import jacobian as J
    c = J.by_name("grid30x20x6")
    plan = _device_plan(c, max_restart=30, precond_precision=L.PRECISION_FP32)
    part = 1024 * 66 * 8
    assert plan.count(part) == 1
    plan = [part_blocks * 66 * 8 if v == part else v for v in plan]
    exe = str(tmp_path / "arena_replay")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    f"-I{CSRC}", os.path.join(HERE, "cpp", "arena_replay.cpp"), "-o", exe, "-pthread"],
                   check=True)
    for mult, together in ((1.5, 1), (2.5, 2)):
        inp = f"{len(plan)} {' '.join(map(str, plan))} {c.n_dof} {mult} 6 {together} 2000\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True)
        assert out.returncode == 0, out.stdout + out.stderr
        f = dict(zip(out.stdout.split()[0::2], map(int, out.stdout.split()[1::2])))
        assert f["schedules"] == 2000 and f["with_failed_build"] == 0 and f["failed_builds"] == 0, out.stdout

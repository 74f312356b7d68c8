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

"""MI355X CPTR library: Python binding of libcptr.so (argument marshalling only).

Every step of the preconditioner and the solver runs in the HIP library; this
module only converts numpy arrays / torch tensors into pointers and back.  It
raises if the compiled library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcptr.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "cptr.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(_HERE), "include", "cptr_serve.h")]

CPTR_OK, CPTR_NOT_CONVERGED = 0, 1
CPTR_E_INVALID, CPTR_E_NOMEM, CPTR_E_ZERO_PIVOT = -1, -2, -3
CPTR_E_SINGULAR_COARSE, CPTR_E_HIP, CPTR_E_STATE = -4, -5, -6
RESTRICT_QUASI_IMPES, RESTRICT_INJECTION = 0, 1
ILU_SWEEP_AUTO, ILU_SWEEP_LEVELS, ILU_SWEEP_ONE_LAUNCH, ILU_SWEEP_GRID = 0, 1, 2, 3
PRECISION_FP64, PRECISION_FP32 = 0, 1
EXPORT = dict(CF=0, A_ROWPTR=1, A_COLS=2, A_VALS=3, P_ROWPTR=4, P_COLS=5, P_VALS=6, W=7,
              DINV=8, ILU_VALS=9, ILU_NLEVELS=10, SWEEP=11, SETUP_SITES=12,
              DEVICE_PLAN=13, SETUP_TIMES=14, DENSE_TAIL=15)
SETUP_STEPS = ["validate", "reduce", "strength", "split", "interp", "galerkin", "smoother", "ilu_levels",
               "device", "total"]
PHASES = ["spmv", "restrict", "vcycle_l0", "vcycle_coarse", "stage2_resid", "ilu_fwd",
          "ilu_bwd", "arnoldi", "update"]


class CptrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cptr status {code}: {msg}")
        self.code = code


class cptr_bsr(C.Structure):
    _fields_ = [("n_block_rows", C.c_int32), ("nnz_blocks", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("values", C.c_void_p),
                ("on_device", C.c_int32)]


class cptr_setup_opts(C.Structure):
    _fields_ = [("strong_threshold", C.c_double), ("max_row_sum", C.c_double),
                ("max_levels", C.c_int32), ("max_coarse", C.c_int32),
                ("p_max_elmts", C.c_int32), ("restriction", C.c_int32),
                ("host_only", C.c_int32), ("setup_threads", C.c_int32),
                ("ilu_sweep", C.c_int32), ("agg_levels", C.c_int32),
                ("precond_precision", C.c_int32), ("num_sweeps", C.c_int32),
                ("max_restart", C.c_int32), ("flexible_space", C.c_int32),
                ("hmis_block", C.c_int32), ("max_dense_coarse", C.c_int32),
                ("dense_tail", C.c_int32)]


class cptr_solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("flexible", C.c_int32),
                ("x0_is_zero", C.c_int32), ("rtol", C.c_double), ("profile", C.c_int32)]


class cptr_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("rel_res_est", C.c_double), ("rel_res_true", C.c_double),
                ("setup_s", C.c_double), ("solve_s", C.c_double)]


class cptr_server_opts(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("setup_workers", C.c_int32),
                ("hbm_budget_bytes", C.c_int64), ("device", C.c_int32),
                ("setup", cptr_setup_opts)]


class cptr_serve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("converged", C.c_int32),
                ("pad_", C.c_int32), ("rel_res_true", C.c_double), ("queue_s", C.c_double),
                ("host_setup_s", C.c_double), ("admit_wait_s", C.c_double),
                ("device_setup_s", C.c_double), ("solve_s", C.c_double),
                ("latency_s", C.c_double), ("device_bytes", C.c_int64),
                ("admitted_at_s", C.c_double), ("done_at_s", C.c_double)]


class cptr_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("peak_inflight", C.c_int32), ("pad_", C.c_int32),
                ("peak_reserved_bytes", C.c_int64), ("hbm_budget_bytes", C.c_int64)]


_lib = None


def lib():
    """Load libcptr.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2308_11892_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.cptr_setup_opts_default.argtypes = [C.POINTER(cptr_setup_opts)]
        L.cptr_setup_opts_default.restype = None
        L.cptr_solve_opts_default.argtypes = [C.POINTER(cptr_solve_opts)]
        L.cptr_solve_opts_default.restype = None
        L.cptr_setup.argtypes = [C.POINTER(cptr_bsr), C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                 C.POINTER(cptr_setup_opts), P, C.POINTER(P)]
        L.cptr_setup.restype = C.c_int
        L.cptr_apply.argtypes = [P, P, P, P]
        L.cptr_apply.restype = C.c_int
        L.cptr_stage1.argtypes = [P, P, P, P]
        L.cptr_stage1.restype = C.c_int
        L.cptr_ilu_solve.argtypes = [P, P, P, P]
        L.cptr_ilu_solve.restype = C.c_int
        L.cptr_spmv.argtypes = [P, P, P, P]
        L.cptr_spmv.restype = C.c_int
        L.cptr_sweep_check.argtypes = [P, P]
        L.cptr_sweep_check.restype = C.c_int
        L.cptr_gmres_solve.argtypes = [P, P, P, C.POINTER(cptr_solve_opts),
                                       C.POINTER(cptr_solve_info), P]
        L.cptr_gmres_solve.restype = C.c_int
        L.cptr_gmres_solve_static.argtypes = [P, P, P, C.POINTER(cptr_solve_opts),
                                              C.POINTER(cptr_solve_info), P]
        L.cptr_gmres_solve_static.restype = C.c_int
        L.cptr_destroy.argtypes = [P]
        L.cptr_destroy.restype = C.c_int
        L.cptr_last_error.argtypes = [P]
        L.cptr_last_error.restype = C.c_char_p
        L.cptr_hierarchy_info.argtypes = [P, C.POINTER(C.c_int32), P, P]
        L.cptr_hierarchy_info.restype = C.c_int
        L.cptr_export.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int64]
        L.cptr_export.restype = C.c_int
        L.cptr_phase_times.argtypes = [P, P, P, C.c_int32, C.c_int32]
        L.cptr_phase_times.restype = C.c_int
        L.cptr_server_opts_default.argtypes = [C.POINTER(cptr_server_opts)]
        L.cptr_server_opts_default.restype = None
        L.cptr_server_create.argtypes = [C.POINTER(cptr_server_opts), P]
        L.cptr_server_create.restype = C.c_int
        L.cptr_server_submit.argtypes = [P, C.POINTER(cptr_bsr), C.POINTER(C.c_int32), C.c_int32, P,
                                         C.POINTER(cptr_solve_opts), C.POINTER(C.c_int64)]
        L.cptr_server_submit.restype = C.c_int
        L.cptr_server_wait.argtypes = [P, C.c_int64, P, C.POINTER(cptr_serve_info), C.c_int32]
        L.cptr_server_wait.restype = C.c_int
        L.cptr_server_last_error.argtypes = [P]
        L.cptr_server_last_error.restype = C.c_char_p
        L.cptr_server_get_stats.argtypes = [P, C.POINTER(cptr_server_stats)]
        L.cptr_server_get_stats.restype = C.c_int
        L.cptr_server_destroy.argtypes = [P]
        L.cptr_server_destroy.restype = C.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/*.h."""
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(cptr_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def _ptr(a):
    """Device (torch) or host (numpy) data pointer."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _check(code, handle=None):
    if code < 0:
        raise CptrError(code, lib().cptr_last_error(handle).decode())
    return code


def setup_opts(**kw):
    o = cptr_setup_opts()
    lib().cptr_setup_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown setup option {k}")
        setattr(o, k, v)
    return o


def solve_opts(**kw):
    o = cptr_solve_opts()
    lib().cptr_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, int(v) if isinstance(v, bool) else v)
    return o


class Solver:
    """Handle around cptr_setup / cptr_apply / cptr_gmres_solve."""

    def __init__(self, row_ptr, col_idx, values, elliptic=(0, 1), stream=None, **opts):
        self._h = None
        on_device = hasattr(values, "data_ptr")
        if on_device:
            import torch
            rp = row_ptr.to(torch.int32).contiguous()
            ci = col_idx.to(torch.int32).contiguous()
            v = values.to(torch.float64).contiguous()
            nb, nnzb = rp.numel() - 1, ci.numel()
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            v = np.ascontiguousarray(values, dtype=np.float64)
            nb, nnzb = rp.shape[0] - 1, ci.shape[0]
        self._keep = (rp, ci, v)
        self.n_block_rows = nb
        self.n = 3 * nb
        A = cptr_bsr(nb, nnzb, _ptr(rp).value, _ptr(ci).value, _ptr(v).value, 1 if on_device else 0)
        ell = (C.c_int32 * len(elliptic))(*elliptic)
        o = setup_opts(**opts)
        self.host_only = bool(o.host_only)
        st = C.c_void_p(None) if self.host_only else _stream(stream)
        h = C.c_void_p()
        code = lib().cptr_setup(C.byref(A), 3, ell, len(elliptic), C.byref(o), st, C.byref(h))
        _check(code, None)
        self._h = h
        self._keep = None

    def close(self):
        if self._h:
            lib().cptr_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- hot path ----
    def apply(self, r, z, stream=None):
        _check(lib().cptr_apply(self._h, _ptr(r), _ptr(z), _stream(stream)), self._h)

    def stage1(self, r, x1, stream=None):
        _check(lib().cptr_stage1(self._h, _ptr(r), _ptr(x1), _stream(stream)), self._h)

    def ilu_solve(self, r, x, stream=None):
        _check(lib().cptr_ilu_solve(self._h, _ptr(r), _ptr(x), _stream(stream)), self._h)

    def spmv(self, x, y, stream=None):
        _check(lib().cptr_spmv(self._h, _ptr(x), _ptr(y), _stream(stream)), self._h)

    def sweep_check(self, stream=None):
        _check(lib().cptr_sweep_check(self._h, _stream(stream)), self._h)

    def gmres_solve(self, b, x, stream=None, static_scratch=False, **kw):
        """cptr_gmres_solve, or cptr_gmres_solve_static with static_scratch."""
        o = solve_opts(**kw)
        info = cptr_solve_info()
        fn = lib().cptr_gmres_solve_static if static_scratch else lib().cptr_gmres_solve
        code = _check(fn(self._h, _ptr(b), _ptr(x), C.byref(o), C.byref(info), _stream(stream)), self._h)
        return dict(status=code, converged=bool(info.converged), iterations=info.iterations,
                    restarts=info.restarts, rel_res_est=info.rel_res_est,
                    rel_res_true=info.rel_res_true, setup_s=info.setup_s, solve_s=info.solve_s)

    # ---- introspection ----
    def hierarchy(self):
        n = C.c_int32()
        _check(lib().cptr_hierarchy_info(self._h, C.byref(n), None, None), self._h)
        rows = np.zeros(n.value, dtype=np.int64)
        nnz = np.zeros(n.value, dtype=np.int64)
        _check(lib().cptr_hierarchy_info(self._h, C.byref(n), _ptr(rows), _ptr(nnz)), self._h)
        return rows, nnz

    def export(self, what, level=0, count=None, dtype=np.float64):
        if isinstance(what, str):
            what = EXPORT[what]
        if count is None:
            raise ValueError("count required")
        out = np.zeros(count, dtype=dtype)
        _check(lib().cptr_export(self._h, what, level, _ptr(out), out.nbytes), self._h)
        return out

    def level_matrix(self, level, which="A"):
        """Level-`level` operator (A) or interpolation (P) as scipy CSR."""
        import scipy.sparse as sp
        rows, _ = self.hierarchy()
        n = int(rows[level])
        pre = which
        rp = self.export(f"{pre}_ROWPTR", level, n + 1, np.int64)
        nnz = int(rp[-1])
        ci = self.export(f"{pre}_COLS", level, nnz, np.int32)
        v = self.export(f"{pre}_VALS", level, nnz, np.float64)
        m = n if which == "A" else int(rows[level + 1])
        return sp.csr_matrix((v, ci, rp), shape=(n, m))

    def cf(self, level):
        rows, _ = self.hierarchy()
        return self.export("CF", level, int(rows[level]), np.int32)

    def phase_times(self, reset=False):
        ms = np.zeros(len(PHASES))
        cnt = np.zeros(len(PHASES), dtype=np.int64)
        _check(lib().cptr_phase_times(self._h, _ptr(ms), _ptr(cnt), len(PHASES), int(reset)), self._h)
        return {p: (float(ms[k]), int(cnt[k])) for k, p in enumerate(PHASES)}


class Server:
    """Handle around cptr_server_*: queues solve requests, admits them to the
    GPU by HBM footprint as slots free up, and returns their solutions."""

    def __init__(self, max_inflight=4, setup_workers=8, hbm_budget_bytes=16 << 30, device=0,
                 **setup):
        self._h = None
        o = cptr_server_opts()
        lib().cptr_server_opts_default(C.byref(o))
        o.max_inflight, o.setup_workers = max_inflight, setup_workers
        o.hbm_budget_bytes, o.device = hbm_budget_bytes, device
        for k, v in setup.items():
            if not hasattr(o.setup, k):
                raise TypeError(f"unknown setup option {k}")
            setattr(o.setup, k, v)
        h = C.c_void_p()
        code = lib().cptr_server_create(C.byref(o), C.byref(h))
        if code < 0:
            raise CptrError(code, "cptr_server_create failed")
        self._h = h
        self._n = {}

    def submit(self, row_ptr, col_idx, values, b, elliptic=(0, 1), **solve):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        v = np.ascontiguousarray(values, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        nb = rp.shape[0] - 1
        A = cptr_bsr(nb, ci.shape[0], _ptr(rp).value, _ptr(ci).value, _ptr(v).value, 0)
        ell = (C.c_int32 * len(elliptic))(*elliptic)
        o = solve_opts(**solve)
        rid = C.c_int64()
        code = lib().cptr_server_submit(self._h, C.byref(A), ell, len(elliptic), _ptr(bb), C.byref(o),
                                        C.byref(rid))
        if code < 0:
            raise CptrError(code, "cptr_server_submit failed")
        self._n[rid.value] = 3 * nb
        return rid.value

    def wait(self, rid, timeout_ms=-1):
        """(x, info) of request rid; info["status"] < 0 for a failed request
        (x is None then)."""
        n = self._n[rid]
        x = np.zeros(n)
        info = cptr_serve_info()
        code = lib().cptr_server_wait(self._h, rid, _ptr(x), C.byref(info), timeout_ms)
        if code == CPTR_E_STATE:
            raise TimeoutError(f"request {rid} not finished")
        del self._n[rid]
        d = {k: getattr(info, k) for k, _ in cptr_serve_info._fields_ if k != "pad_"}
        d["status"] = code
        if code < 0:
            d["error"] = lib().cptr_server_last_error(self._h).decode()
            return None, d
        return x, d

    def stats(self):
        st = cptr_server_stats()
        lib().cptr_server_get_stats(self._h, C.byref(st))
        return {k: getattr(st, k) for k, _ in cptr_server_stats._fields_ if k != "pad_"}

    def close(self):
        if self._h:
            lib().cptr_server_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

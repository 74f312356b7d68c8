"""ctypes wrapper of the plain FP64 CPU oracle (libcptr_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the product path.  The C source
next to this file shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcptr_oracle.so")
_SRC = os.path.join(_HERE, "cptr_oracle.c")

OK, NOT_CONVERGED = 0, 1
PC_NONE, PC_ILU, PC_STAGE1, PC_CPTR = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, like the library's setup)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
               _SRC, "-o", _SO, "-lm"]
        subprocess.run(cmd, check=True)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        lp = C.POINTER(C.c_long)
        L.or_last_error.restype = C.c_char_p
        L.or_mat_info.argtypes = [P, ip, ip, lp]
        L.or_mat_copy.argtypes = [P, lp, ip, dp]
        L.or_mat_free.argtypes = [P]
        L.or_bsr_spmv.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, dp]
        L.or_strength.restype = P
        L.or_strength.argtypes = [C.c_int, lp, ip, dp, ip, C.c_double, C.c_double]
        L.or_rs_first_pass.argtypes = [C.c_int, lp, ip, ip]
        L.or_extpi.restype = P
        L.or_extpi.argtypes = [C.c_int, lp, ip, dp, lp, ip, ip, ip, C.c_int]
        L.or_strength2.restype = P
        L.or_strength2.argtypes = [C.c_int, lp, ip, ip]
        L.or_aggressive_split.argtypes = [C.c_int, lp, ip, ip]
        L.or_hmis_split.argtypes = [C.c_int, lp, ip, C.c_int, ip]
        L.or_aggressive_hmis.argtypes = [C.c_int, lp, ip, C.c_int, ip]
        L.or_multipass.restype = P
        L.or_multipass.argtypes = [C.c_int, lp, ip, dp, lp, ip, ip, ip]
        L.or_amg_setup.argtypes = [C.c_int, lp, ip, dp, ip, P, C.POINTER(P)]
        L.or_amg_nlevels.argtypes = [P]
        L.or_amg_get.restype = P
        L.or_amg_get.argtypes = [P, C.c_int, C.c_int]
        L.or_amg_get_cf.argtypes = [P, C.c_int, ip]
        L.or_amg_get_func.argtypes = [P, C.c_int, ip]
        L.or_amg_get_dinv.argtypes = [P, C.c_int, dp]
        L.or_amg_vcycle.argtypes = [P, dp, dp]
        L.or_amg_free.argtypes = [P]
        L.or_cptr_setup.argtypes = [C.c_int, C.c_int, ip, ip, dp, ip, C.c_int, C.c_int,
                                    P, C.POINTER(P)]
        L.or_cptr_amg.restype = P
        L.or_cptr_amg.argtypes = [P]
        L.or_cptr_get_ahat.restype = P
        L.or_cptr_get_ahat.argtypes = [P]
        L.or_cptr_get_w.argtypes = [P, dp]
        L.or_cptr_get_ilu.restype = P
        L.or_cptr_get_ilu.argtypes = [P]
        for nm in ("or_cptr_restrict", "or_cptr_prolong", "or_cptr_ilu_solve",
                   "or_cptr_stage1", "or_cptr_apply"):
            getattr(L, nm).argtypes = [P, dp, dp]
        L.or_cptr_free.argtypes = [P]
        L.or_gmres.argtypes = [C.c_int, C.c_int, ip, ip, dp, P, dp, dp, P, ip, dp, dp,
                               dp, ip]
        _lib = L
    return _lib


class AmgOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_row_sum", C.c_double),
                ("max_levels", C.c_int), ("max_coarse", C.c_int), ("pmax", C.c_int),
                ("agg_levels", C.c_int), ("num_sweeps", C.c_int), ("hmis_block", C.c_int),
                ("max_dense", C.c_int)]

    def __init__(self, theta=0.25, max_row_sum=0.9, max_levels=25, max_coarse=9, pmax=4,
                 agg_levels=1, num_sweeps=1, hmis_block=0, max_dense=4096):
        super().__init__(theta, max_row_sum, max_levels, max_coarse, pmax, agg_levels, num_sweeps,
                         hmis_block, max_dense)


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iter", C.c_int), ("flexible", C.c_int),
                ("precond", C.c_int), ("rtol", C.c_double)]

    def __init__(self, restart=30, max_iter=200, flexible=0, precond=PC_CPTR, rtol=1e-6):
        super().__init__(restart, max_iter, flexible, precond, rtol)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


def _err(code):
    if code < 0:
        raise OracleError(code, lib().or_last_error().decode())
    return code


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_long))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _take_mat(ptr):
    """Copy an or_mat into a scipy.sparse.csr_matrix and free it."""
    import scipy.sparse as sp
    L = lib()
    n, m, nnz = C.c_int(), C.c_int(), C.c_long()
    L.or_mat_info(ptr, C.byref(n), C.byref(m), C.byref(nnz))
    rp = np.zeros(n.value + 1, dtype=np.int64)
    ci = np.zeros(nnz.value, dtype=np.int32)
    v = np.zeros(nnz.value, dtype=np.float64)
    L.or_mat_copy(ptr, _l(rp), _i(ci), _d(v))
    L.or_mat_free(ptr)
    return sp.csr_matrix((v, ci, rp), shape=(n.value, m.value))


def _csr_parts(A):
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A.shape[0], _i64(A.indptr), _i32(A.indices), _f64(A.data)


# ----------------------------------------------------------------- kernels
def bsr_spmv(row_ptr, col_idx, values, x):
    nb = row_ptr.shape[0] - 1
    bs = values.shape[1]
    rp, ci, v, x = _i32(row_ptr), _i32(col_idx), _f64(values), _f64(x)
    y = np.zeros(nb * bs)
    lib().or_bsr_spmv(nb, bs, _i(rp), _i(ci), _d(v), _d(x), _d(y))
    return y


def strength(A, func, theta=0.25, max_row_sum=0.9):
    n, rp, ci, v = _csr_parts(A)
    f = _i32(func)
    return _take_mat(lib().or_strength(n, _l(rp), _i(ci), _d(v), _i(f), theta, max_row_sum))


def rs_first_pass(S):
    n, rp, ci, _ = _csr_parts(S)
    cf = np.zeros(n, dtype=np.int32)
    lib().or_rs_first_pass(n, _l(rp), _i(ci), _i(cf))
    return cf


def extpi(A, S, cf, func, pmax=0):
    n, rp, ci, v = _csr_parts(A)
    _, srp, sci, _ = _csr_parts(S)
    cf, f = _i32(cf), _i32(func)
    return _take_mat(lib().or_extpi(n, _l(rp), _i(ci), _d(v), _l(srp), _i(sci), _i(cf),
                                    _i(f), pmax))


def strength2(S, cf):
    """Distance-two strength among the C points of cf (rows/columns = C points in order)."""
    n, rp, ci, _ = _csr_parts(S)
    cf = _i32(cf)
    return _take_mat(lib().or_strength2(n, _l(rp), _i(ci), _i(cf)))


def aggressive_split(S):
    n, rp, ci, _ = _csr_parts(S)
    cf = np.zeros(n, dtype=np.int32)
    lib().or_aggressive_split(n, _l(rp), _i(ci), _i(cf))
    return cf


def hmis_split(S, block):
    """HMIS split over blocks of `block` consecutive points (0: one block)."""
    n, rp, ci, _ = _csr_parts(S)
    cf = np.zeros(n, dtype=np.int32)
    lib().or_hmis_split(n, _l(rp), _i(ci), int(block), _i(cf))
    return cf


def aggressive_hmis(S, block):
    n, rp, ci, _ = _csr_parts(S)
    cf = np.zeros(n, dtype=np.int32)
    lib().or_aggressive_hmis(n, _l(rp), _i(ci), int(block), _i(cf))
    return cf


def multipass(A, S, cf, func):
    n, rp, ci, v = _csr_parts(A)
    _, srp, sci, _ = _csr_parts(S)
    cf, f = _i32(cf), _i32(func)
    return _take_mat(lib().or_multipass(n, _l(rp), _i(ci), _d(v), _l(srp), _i(sci), _i(cf),
                                        _i(f)))


# ----------------------------------------------------------------- AMG
class Amg:
    def __init__(self, A, func, **opts):
        n, self._rp, self._ci, self._v = _csr_parts(A)
        self._f = _i32(func)
        self.n = n
        h = C.c_void_p()
        o = AmgOpts(**opts)
        _err(lib().or_amg_setup(n, _l(self._rp), _i(self._ci), _d(self._v), _i(self._f),
                                C.byref(o), C.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_amg_free(self._h)
            self._h = None

    @property
    def nlevels(self):
        return lib().or_amg_nlevels(self._h)

    def A(self, l):
        return _take_mat(lib().or_amg_get(self._h, l, 0))

    def P(self, l):
        return _take_mat(lib().or_amg_get(self._h, l, 1))

    def R(self, l):
        return _take_mat(lib().or_amg_get(self._h, l, 2))

    def size(self, l):
        n, m, nnz = C.c_int(), C.c_int(), C.c_long()
        p = lib().or_amg_get(self._h, l, 0)
        lib().or_mat_info(p, C.byref(n), C.byref(m), C.byref(nnz))
        lib().or_mat_free(p)
        return n.value, nnz.value

    def cf(self, l):
        out = np.zeros(self.size(l)[0], dtype=np.int32)
        lib().or_amg_get_cf(self._h, l, _i(out))
        return out

    def func(self, l):
        out = np.zeros(self.size(l)[0], dtype=np.int32)
        lib().or_amg_get_func(self._h, l, _i(out))
        return out

    def dinv(self, l):
        out = np.zeros(self.size(l)[0])
        lib().or_amg_get_dinv(self._h, l, _d(out))
        return out

    def vcycle(self, b):
        b = _f64(b)
        x = np.zeros_like(b)
        lib().or_amg_vcycle(self._h, _d(b), _d(x))
        return x


class _AmgView(Amg):
    """Borrowed view of the AMG hierarchy inside a Cptr handle."""

    def __init__(self, handle, owner):
        self._h = handle
        self._owner = owner

    def __del__(self):
        pass


# ----------------------------------------------------------------- CPTR
class Cptr:
    """Oracle CPTR preconditioner for a 3x3 (or b x b) block-CSR matrix."""

    def __init__(self, row_ptr, col_idx, values, elliptic=(0, 1), qi=True, **amg_opts):
        self.rp = _i32(row_ptr)
        self.ci = _i32(col_idx)
        self.v = _f64(values)
        self.nb = self.rp.shape[0] - 1
        self.bs = self.v.shape[1]
        self.n = self.nb * self.bs
        self.eidx = _i32(list(elliptic))
        self.ne = len(elliptic)
        h = C.c_void_p()
        o = AmgOpts(**amg_opts)
        _err(lib().or_cptr_setup(self.nb, self.bs, _i(self.rp), _i(self.ci), _d(self.v),
                                 _i(self.eidx), self.ne, 1 if qi else 0, C.byref(o),
                                 C.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_cptr_free(self._h)
            self._h = None

    @property
    def amg(self):
        return _AmgView(lib().or_cptr_amg(self._h), self)

    def ahat(self):
        return _take_mat(lib().or_cptr_get_ahat(self._h))

    def W(self):
        out = np.zeros(self.nb * self.ne * (self.bs - self.ne))
        lib().or_cptr_get_w(self._h, _d(out))
        return out.reshape(self.nb, self.ne, self.bs - self.ne)

    def ilu(self):
        return _take_mat(lib().or_cptr_get_ilu(self._h))

    def _unary(self, name, r, nout):
        r = _f64(r)
        out = np.zeros(nout)
        getattr(lib(), name)(self._h, _d(r), _d(out))
        return out

    def restrict(self, r):
        return self._unary("or_cptr_restrict", r, self.nb * self.ne)

    def prolong(self, e):
        return self._unary("or_cptr_prolong", e, self.n)

    def ilu_solve(self, r):
        return self._unary("or_cptr_ilu_solve", r, self.n)

    def stage1(self, r):
        return self._unary("or_cptr_stage1", r, self.n)

    def apply(self, r):
        return self._unary("or_cptr_apply", r, self.n)

    def spmv(self, x):
        return bsr_spmv(self.rp, self.ci, self.v, x)

    def gmres(self, b, x0=None, restart=30, max_iter=200, flexible=False,
              precond=PC_CPTR, rtol=1e-6, history=False):
        return gmres(self.rp, self.ci, self.v, b, x0=x0, pc=self, restart=restart,
                     max_iter=max_iter, flexible=flexible, precond=precond, rtol=rtol,
                     history=history)


def gmres(row_ptr, col_idx, values, b, x0=None, pc=None, restart=30, max_iter=200,
          flexible=False, precond=PC_NONE, rtol=1e-6, history=False):
    rp, ci, v = _i32(row_ptr), _i32(col_idx), _f64(values)
    nb = rp.shape[0] - 1
    bs = v.shape[1]
    b = _f64(b)
    x = np.zeros(nb * bs) if x0 is None else _f64(x0).copy()
    o = GmresOpts(restart, max_iter, 1 if flexible else 0, precond, rtol)
    it, est, tru, hn = C.c_int(), C.c_double(), C.c_double(), C.c_int()
    hist = np.zeros(max_iter + 2)
    st = _err(lib().or_gmres(nb, bs, _i(rp), _i(ci), _d(v), pc._h if pc is not None else None,
                             _d(b), _d(x), C.byref(o), C.byref(it), C.byref(est),
                             C.byref(tru), _d(hist), C.byref(hn)))
    info = dict(status=st, converged=(st == OK), iterations=it.value, rel_res_est=est.value,
                rel_res_true=tru.value)
    if history:
        info["history"] = hist[:hn.value].copy()
    return x, info

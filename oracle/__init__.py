"""ctypes shim over the plain FP64 CPU oracle (``oracle/pf_oracle.c``).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import this module.  It shares no code with the
GPU path and never imports it.

Every function cites the part of the paper it follows in ``pf_oracle.c``.  The
relative-residual helper and the dense brute-force check live in the tests, not here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i8p = ctypes.POINTER(ctypes.c_int8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.c_int, _ip, _ip, _dp, _i8p]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_dims.argtypes = [ctypes.c_void_p, _ip]
        L.oracle_order.argtypes = [ctypes.c_void_p, _ip]
        L.oracle_jacobian_pattern.argtypes = [ctypes.c_void_p, _ip, _ip]
        L.oracle_mismatch.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.oracle_jacobian.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oracle_jacobian_solve.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.oracle_sparse_solve.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp]
        L.oracle_branch_flows.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _ip, _dp, _dp, _dp,
                                          _dp, _dp, _dp]
        L.oracle_nr.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, _dp, _ip, _u8p, _i8p, _dp]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _cplx_to_pairs(z) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.complex128)
    return z.view(np.float64).reshape(z.shape + (2,))


@dataclass
class Result:
    v: np.ndarray          # [B][n][2] (|V|, theta)
    iters: np.ndarray      # [B] int32
    converged: np.ndarray  # [B] bool
    status: np.ndarray     # [B] int8: 0 converged, 1 max_iter, 2 non-finite, 3 singular
    hist: np.ndarray       # [B][max_iter+1] max|F| per mismatch evaluation (NaN after stop)


class System:
    """One Ybus pattern + values + bus types: unknown numbering, Jacobian pattern and the
    oracle's own minimum-degree order."""

    def __init__(self, row_ptr, col_idx, yval, bus_type):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.y = np.ascontiguousarray(_cplx_to_pairs(yval))
        self.bus_type = np.ascontiguousarray(bus_type, dtype=np.int8)
        self.n = int(self.row_ptr.shape[0] - 1)
        self._h = lib().oracle_create(self.n, _p(self.row_ptr, _ip), _p(self.col_idx, _ip),
                                      _p(self.y, _dp), _p(self.bus_type, _i8p))
        if not self._h:
            raise ValueError("oracle_create rejected the system")
        d = np.zeros(5, dtype=np.int32)
        lib().oracle_dims(self._h, _p(d, _ip))
        _, self.npv, self.npq, self.N, self.nnzj = (int(x) for x in d)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_destroy(h)
            self._h = None

    @classmethod
    def from_ybus(cls, yb, bus_type):
        return cls(yb.row_ptr, yb.col_idx, yb.val, bus_type)

    # unknown numbering: theta of pv buses, theta of pq buses, |V| of pq buses (ascending)
    def unknown_buses(self):
        bt = self.bus_type
        pv = np.flatnonzero(bt == 2)
        pq = np.flatnonzero(bt == 1)
        return pv, pq

    def order(self) -> np.ndarray:
        o = np.zeros(self.N, dtype=np.int32)
        lib().oracle_order(self._h, _p(o, _ip))
        return o

    def jacobian_pattern(self):
        rp = np.zeros(self.N + 1, dtype=np.int32)
        ci = np.zeros(self.nnzj, dtype=np.int32)
        lib().oracle_jacobian_pattern(self._h, _p(rp, _ip), _p(ci, _ip))
        return rp, ci

    def mismatch(self, sbus, v):
        s = np.ascontiguousarray(_cplx_to_pairs(sbus))
        vv = np.ascontiguousarray(v, dtype=np.float64)
        F = np.zeros(self.N)
        nf = np.zeros(1)
        lib().oracle_mismatch(self._h, _p(s, _dp), _p(vv, _dp), _p(F, _dp), _p(nf, _dp))
        return F, float(nf[0])

    def jacobian(self, v):
        vv = np.ascontiguousarray(v, dtype=np.float64)
        J = np.zeros(self.nnzj)
        lib().oracle_jacobian(self._h, _p(vv, _dp), _p(J, _dp))
        return J

    def jacobian_dense(self, v):
        rp, ci = self.jacobian_pattern()
        J = self.jacobian(v)
        D = np.zeros((self.N, self.N))
        for r in range(self.N):
            D[r, ci[rp[r]:rp[r + 1]]] = J[rp[r]:rp[r + 1]]
        return D

    def jacobian_solve(self, J, rhs):
        J = np.ascontiguousarray(J, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        x = np.zeros(self.N)
        rc = lib().oracle_jacobian_solve(self._h, _p(J, _dp), _p(rhs, _dp), _p(x, _dp))
        if rc:
            raise np.linalg.LinAlgError(f"oracle LU failed ({rc})")
        return x

    def solve(self, sbus, v0, tol=1e-8, max_iter=10, threads=None) -> Result:
        sbus = np.asarray(sbus)
        B = int(sbus.shape[0])
        s = np.ascontiguousarray(_cplx_to_pairs(sbus))
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        assert v0.shape == (B, self.n, 2)
        vo = np.zeros((B, self.n, 2))
        it = np.zeros(B, dtype=np.int32)
        cv = np.zeros(B, dtype=np.uint8)
        st = np.zeros(B, dtype=np.int8)
        hist = np.zeros((B, max_iter + 1))
        if threads is None:
            threads = os.cpu_count() or 1
        lib().oracle_nr(self._h, B, _p(s, _dp), _p(v0, _dp), float(tol), int(max_iter),
                        int(threads), _p(vo, _dp), _p(it, _ip), _p(cv, _u8p), _p(st, _i8p),
                        _p(hist, _dp))
        return Result(v=vo, iters=it, converged=cv.astype(bool), status=st, hist=hist)


def sparse_solve(row_ptr, col_idx, val, b):
    """Solve A x = b (square CSR A) with the oracle's pre-order + pivoting LU."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    N = int(rp.shape[0] - 1)
    x = np.zeros(N)
    rc = lib().oracle_sparse_solve(N, _p(rp, _ip), _p(ci, _ip), _p(v, _dp), _p(bb, _dp), _p(x, _dp))
    if rc:
        raise np.linalg.LinAlgError(f"oracle LU failed ({rc})")
    return x


def branch_flows(grid, v):
    """(S_from, S_to) complex [m] for every pi-model branch of a gridgen.Grid at V."""
    f = np.ascontiguousarray(grid.f, dtype=np.int32)
    t = np.ascontiguousarray(grid.t, dtype=np.int32)
    r = np.ascontiguousarray(grid.r, dtype=np.float64)
    x = np.ascontiguousarray(grid.x, dtype=np.float64)
    b = np.ascontiguousarray(grid.b, dtype=np.float64)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    m = int(f.shape[0])
    sf = np.zeros((m, 2))
    st = np.zeros((m, 2))
    lib().oracle_branch_flows(grid.n, m, _p(f, _ip), _p(t, _ip), _p(r, _dp), _p(x, _dp),
                              _p(b, _dp), _p(vv, _dp), _p(sf, _dp), _p(st, _dp))
    return sf[:, 0] + 1j * sf[:, 1], st[:, 0] + 1j * st[:, 1]

"""ctypes wrapper around the plain FP64 C++ oracle (wcl_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg; the product library never imports it.

All fields are numpy complex128 in the canonical host layouts:
gauge [V][4][3][3], spinor [V][4][3], site index x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wcl_oracle.cpp")
lib_path = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP over sites)."""
    if force or not os.path.exists(lib_path):
        tmp = lib_path + ".tmp"
        # x86-64-v3 (AVX2/FMA) rather than -march=native: the built library also
        # runs on other hosts than the one that built it; no FMA contraction,
        # so every product and sum rounds as written
        cmd = ["g++", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-std=c++17", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib_path)
    return lib_path


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            build()
        L = C.CDLL(lib_path)
        vp, dp, ip, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int64)
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [ip, ip, dp, C.c_int]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_last_error.restype = C.c_char_p
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_gammas.argtypes = [dp, dp]
        L.oracle_clover.argtypes = [vp, C.c_int64, i64p, dp]
        L.oracle_apply_D.argtypes = [vp, C.c_double, C.c_double, dp, dp]
        L.oracle_apply_D_sites.argtypes = [vp, C.c_double, C.c_double, dp, C.c_int64, i64p, dp]
        L.oracle_decomp.argtypes = [vp, ip, C.c_int, i64p, i64p]
        L.oracle_block_sites.argtypes = [vp, ip, C.c_int, C.c_int64, i64p]
        L.oracle_block_apply.argtypes = [vp, ip, C.c_int, C.c_int64, C.c_double, C.c_double, dp, dp]
        L.oracle_block_mr.argtypes = [vp, ip, C.c_int, C.c_int64, C.c_double, C.c_double, C.c_int, dp, dp]
        L.oracle_ras.argtypes = [vp, ip, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, dp, dp]
        L.oracle_schwarz.argtypes = [vp, ip, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                     C.c_double, dp, dp]
        L.oracle_block_solve.argtypes = [vp, ip, C.c_int, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_int,
                                         dp, dp]
        L.oracle_site_term_inverse.argtypes = [vp, C.c_double, C.c_double, C.c_int64, i64p, dp]
        L.oracle_apply_schur.argtypes = [vp, C.c_double, C.c_double, dp, dp]
        L.oracle_eo_solve.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, ip, dp]
        L.oracle_bicgstab.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, ip, dp]
        L.oracle_nested.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int,
                                    C.c_int, ip, C.c_int, C.c_int, C.c_int, dp, dp, ip, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _i64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """A lattice with resident gauge field (and optionally its clover field)."""

    def __init__(self, dims, U, bc=(1, 1, 1, 1), precompute_clover=True):
        self.lib = _load()
        self.dims = np.array(dims, dtype=np.int32)
        self.bc = np.array(bc, dtype=np.int32)
        self.V = int(np.prod(self.dims))
        self.U = _c128(U, (self.V, 4, 3, 3))
        self.h = self.lib.oracle_create(_ip(self.dims), _ip(self.bc), _dp(self.U), int(precompute_clover))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oracle_destroy(h)
            self.h = None

    @staticmethod
    def num_threads() -> int:
        return _load().oracle_num_threads()

    @staticmethod
    def set_threads(n: int):
        _load().oracle_set_threads(int(n))

    @staticmethod
    def gammas():
        g = np.zeros((4, 4, 4), dtype=np.complex128)
        s = np.zeros((4, 4, 4, 4), dtype=np.complex128)
        _load().oracle_gammas(_dp(g), _dp(s))
        return g, s

    def clover(self, sites=None) -> np.ndarray:
        sites = np.arange(self.V, dtype=np.int64) if sites is None else np.ascontiguousarray(sites, dtype=np.int64)
        out = np.zeros((len(sites), 12, 12), dtype=np.complex128)
        self.lib.oracle_clover(self.h, len(sites), _i64p(sites), _dp(out))
        return out

    def apply_D(self, psi, kappa, csw) -> np.ndarray:
        psi = _c128(psi, (self.V, 4, 3))
        out = np.zeros_like(psi)
        self.lib.oracle_apply_D(self.h, kappa, csw, _dp(psi), _dp(out))
        return out

    def apply_D_sites(self, psi, kappa, csw, sites) -> np.ndarray:
        psi = _c128(psi, (self.V, 4, 3))
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
        self.lib.oracle_apply_D_sites(self.h, kappa, csw, _dp(psi), len(sites), _i64p(sites), _dp(out))
        return out

    def decomp(self, block, s):
        b = np.array(block, dtype=np.int32)
        nb = np.zeros(1, np.int64)
        ev = np.zeros(1, np.int64)
        if self.lib.oracle_decomp(self.h, _ip(b), int(s), _i64p(nb), _i64p(ev)) != 0:
            raise ValueError(self.lib.oracle_last_error().decode())
        return int(nb[0]), int(ev[0])

    def block_sites(self, block, s, blk) -> np.ndarray:
        _, ev = self.decomp(block, s)
        out = np.zeros(ev, dtype=np.int64)
        b = np.array(block, dtype=np.int32)
        if self.lib.oracle_block_sites(self.h, _ip(b), int(s), int(blk), _i64p(out)) != 0:
            raise ValueError("bad block")
        return out

    def block_apply(self, block, s, blk, psi_ext, kappa, csw) -> np.ndarray:
        _, ev = self.decomp(block, s)
        psi_ext = _c128(psi_ext, (ev, 4, 3))
        out = np.zeros_like(psi_ext)
        b = np.array(block, dtype=np.int32)
        if self.lib.oracle_block_apply(self.h, _ip(b), int(s), int(blk), kappa, csw, _dp(psi_ext), _dp(out)) != 0:
            raise ValueError("bad block")
        return out

    def block_mr(self, block, s, blk, rhs_ext, kappa, csw, n) -> np.ndarray:
        _, ev = self.decomp(block, s)
        rhs_ext = _c128(rhs_ext, (ev, 4, 3))
        out = np.zeros_like(rhs_ext)
        b = np.array(block, dtype=np.int32)
        if self.lib.oracle_block_mr(self.h, _ip(b), int(s), int(blk), kappa, csw, int(n), _dp(rhs_ext), _dp(out)) != 0:
            raise ValueError("bad block")
        return out

    def ras(self, eta, kappa, csw, block, s, n_ras, n_dominv, exact=False) -> np.ndarray:
        eta = _c128(eta, (self.V, 4, 3))
        phi = np.zeros_like(eta)
        b = np.array(block, dtype=np.int32)
        rc = self.lib.oracle_ras(self.h, _ip(b), int(s), int(n_ras), int(n_dominv), int(bool(exact)),
                                 kappa, csw, _dp(eta), _dp(phi))
        if rc != 0:
            raise ValueError(self.lib.oracle_last_error().decode())
        return phi

    # domain solvers and Schwarz iterations: 0 = MR / RAS (Algorithm 1),
    # 1 = block Jacobi / additive, 2 = truncated BiCGStab / multiplicative
    def schwarz(self, eta, kappa, csw, block, s, n_ras, n_dominv, solver=0, schwarz=0, exact=False):
        eta = _c128(eta, (self.V, 4, 3))
        phi = np.zeros_like(eta)
        b = np.array(block, dtype=np.int32)
        rc = self.lib.oracle_schwarz(self.h, _ip(b), int(s), int(n_ras), int(n_dominv), int(bool(exact)),
                                     int(solver), int(schwarz), kappa, csw, _dp(eta), _dp(phi))
        if rc != 0:
            raise ValueError(self.lib.oracle_last_error().decode())
        return phi

    def block_solve(self, block, s, blk, rhs_ext, kappa, csw, solver, n) -> np.ndarray:
        _, ev = self.decomp(block, s)
        rhs_ext = _c128(rhs_ext, (ev, 4, 3))
        out = np.zeros_like(rhs_ext)
        b = np.array(block, dtype=np.int32)
        if self.lib.oracle_block_solve(self.h, _ip(b), int(s), int(blk), kappa, csw, int(solver), int(n),
                                       _dp(rhs_ext), _dp(out)) != 0:
            raise ValueError("bad block or solver")
        return out

    def site_term_inverse(self, kappa, csw, sites=None) -> np.ndarray:
        sites = np.arange(self.V, dtype=np.int64) if sites is None else np.ascontiguousarray(sites, dtype=np.int64)
        out = np.zeros((len(sites), 12, 12), dtype=np.complex128)
        if self.lib.oracle_site_term_inverse(self.h, kappa, csw, len(sites), _i64p(sites), _dp(out)) != 0:
            raise ValueError("singular site term")
        return out

    def apply_schur(self, psi, kappa, csw) -> np.ndarray:
        psi = _c128(psi, (self.V, 4, 3))
        out = np.zeros_like(psi)
        if self.lib.oracle_apply_schur(self.h, kappa, csw, _dp(psi), _dp(out)) != 0:
            raise ValueError(self.lib.oracle_last_error().decode())
        return out

    def eo_solve(self, eta, kappa, csw, tol=1e-10, max_iter=10000):
        eta = _c128(eta, (self.V, 4, 3))
        phi = np.zeros_like(eta)
        info = np.zeros(3, np.int32)
        rr = np.zeros(1)
        rc = self.lib.oracle_eo_solve(self.h, kappa, csw, tol, int(max_iter), _dp(eta), _dp(phi), _ip(info), _dp(rr))
        if rc < 0:
            raise ValueError(self.lib.oracle_last_error().decode())
        return phi, {"iters": int(info[0]), "restarts": int(info[1]), "converged": bool(info[2]),
                     "rel_resid": float(rr[0])}

    def bicgstab(self, eta, kappa, csw, tol=1e-10, max_iter=10000):
        eta = _c128(eta, (self.V, 4, 3))
        phi = np.zeros_like(eta)
        info = np.zeros(3, np.int32)
        rr = np.zeros(1)
        self.lib.oracle_bicgstab(self.h, kappa, csw, tol, int(max_iter), _dp(eta), _dp(phi), _ip(info), _dp(rr))
        return phi, {"iters": int(info[0]), "restarts": int(info[1]), "converged": bool(info[2]),
                     "rel_resid": float(rr[0])}

    def nested(self, eta, kappa, csw, tol=1e-10, max_outer=100, tol_inner=1e-4, max_inner=100,
               ras=True, block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4):
        eta = _c128(eta, (self.V, 4, 3))
        phi = np.zeros_like(eta)
        info = np.zeros(3, np.int32)
        rr = np.zeros(1)
        b = np.array(block, dtype=np.int32)
        rc = self.lib.oracle_nested(self.h, kappa, csw, tol, int(max_outer), tol_inner, int(max_inner),
                                    int(bool(ras)), _ip(b), int(s), int(n_ras), int(n_dominv),
                                    _dp(eta), _dp(phi), _ip(info), _dp(rr))
        if rc < 0:
            raise ValueError(self.lib.oracle_last_error().decode())
        return phi, {"outer_iters": int(info[0]), "inner_iters": int(info[1]), "converged": bool(info[2]),
                     "rel_resid": float(rr[0])}

"""Thin ctypes binding of libwcl.so (the C ABI declared in include/wcl.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (uint8 tensors sized by wcl_spinor_bytes) and
streams (torch.cuda.current_stream().cuda_stream).  There is no fallback:
if the library is missing or fails to load, import raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime libwcl.so links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwcl.so")

F64, F32, F16 = 0, 1, 2
BLOCK_AUTO, BLOCK_FUSED, BLOCK_SPLIT = 0, 1, 2
DOMSOLVE_MR, DOMSOLVE_JACOBI, DOMSOLVE_BICGSTAB = 0, 1, 2
SCHWARZ_RAS, SCHWARZ_AS, SCHWARZ_SAP = 0, 1, 2
ARITH_FP32, ARITH_DOT2 = 0, 1
PRECOND_NONE, PRECOND_RAS = 0, 1
OK, EINVAL, ENOMEM, EUNITARITY, ENOTCONV, EBREAKDOWN, EHIP, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
PENDING = 1
_NAMES = {0: "WCL_OK", -1: "WCL_EINVAL", -2: "WCL_ENOMEM", -3: "WCL_EUNITARITY", -4: "WCL_ENOTCONV",
          -5: "WCL_EBREAKDOWN", -6: "WCL_EHIP", -7: "WCL_ESTATE", 1: "WCL_PENDING"}


class WclError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class RasParams(C.Structure):
    _fields_ = [("block", C.c_int * 4), ("s", C.c_int), ("n_ras", C.c_int), ("n_dominv", C.c_int),
                ("storage", C.c_int), ("kernel", C.c_int), ("block_solver", C.c_int), ("schwarz", C.c_int),
                ("arith", C.c_int)]

    @classmethod
    def make(cls, block=(4, 4, 4, 4), s=0, n_ras=3, n_dominv=4, storage=F32, kernel=BLOCK_AUTO,
             block_solver=DOMSOLVE_MR, schwarz=SCHWARZ_RAS, arith=ARITH_FP32):
        return cls((C.c_int * 4)(*block), s, n_ras, n_dominv, storage, kernel, block_solver, schwarz, arith)


class SolverParams(C.Structure):
    _fields_ = [("tol_outer", C.c_double), ("tol_inner", C.c_double), ("max_outer", C.c_int),
                ("max_inner", C.c_int), ("max_restarts", C.c_int), ("precond", C.c_int), ("ras", RasParams),
                ("even_odd", C.c_int), ("timers", C.c_int)]

    @classmethod
    def make(cls, tol_outer=1e-10, tol_inner=1e-4, max_outer=200, max_inner=100, max_restarts=10,
             precond=PRECOND_RAS, ras=None, even_odd=0, timers=0):
        return cls(tol_outer, tol_inner, max_outer, max_inner, max_restarts, precond,
                   ras if ras is not None else RasParams.make(), even_odd, timers)


class SolveStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("dslash_full", C.c_int64), ("dslash_block", C.c_int64), ("ras_sweeps", C.c_int64),
                ("true_resid", C.c_double), ("ms_total", C.c_double), ("ms_dslash", C.c_double),
                ("ms_dominv", C.c_double), ("ms_blas", C.c_double), ("ms_host", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or paper_1011_3318_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, i, d, u64, i64 = C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_int64
    ip, dp = C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "wcl_init": (i, [i, u64, C.POINTER(vp)]),
        "wcl_finalize": (i, [vp]),
        "wcl_last_error": (C.c_char_p, []),
        "wcl_bytes_in_use": (u64, [vp]),
        "wcl_create_lattice": (i, [vp, ip, ip, C.POINTER(vp)]),
        "wcl_destroy_lattice": (i, [vp]),
        "wcl_volume": (i64, [vp]),
        "wcl_upload_gauge": (i, [vp, dp]),
        "wcl_compute_clover": (i, [vp]),
        "wcl_upload_clover": (i, [vp, dp]),
        "wcl_download_clover": (i, [vp, dp]),
        "wcl_spinor_bytes": (u64, [vp, i, i]),
        "wcl_pack_spinor": (i, [vp, i, i, dp, vp, vp]),
        "wcl_unpack_spinor": (i, [vp, i, i, vp, dp, vp]),
        "wcl_pack_spinor_dev": (i, [vp, i, i, vp, vp, vp]),
        "wcl_unpack_spinor_dev": (i, [vp, i, i, vp, vp, vp]),
        "wcl_apply_D": (i, [vp, i, d, d, vp, vp, i, vp]),
        "wcl_apply_schur": (i, [vp, i, d, d, vp, vp, i, vp]),
        "wcl_apply_D_blocks": (i, [vp, C.POINTER(RasParams), d, d, vp, dp, vp]),
        "wcl_block_info": (i, [vp, C.POINTER(RasParams), C.POINTER(i64), C.POINTER(i64)]),
        "wcl_ras_precondition": (i, [vp, C.POINTER(RasParams), d, d, vp, vp, i, vp]),
        "wcl_ras_precondition_noalloc": (i, [vp, C.POINTER(RasParams), d, d, vp, vp, i, vp]),
        "wcl_solve_nested_bicgstab": (i, [vp, C.POINTER(SolverParams), d, d, vp, vp, i, C.POINTER(SolveStats), vp]),
        "wcl_solve_bicgstab_f64": (i, [vp, d, i, d, d, vp, vp, C.POINTER(SolveStats), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def check(rc: int, what: str = ""):
    if rc < 0:
        raise WclError(rc, (lib.wcl_last_error() or b"").decode() or what)
    return rc


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = C.c_void_p()
        check(lib.wcl_init(device, hbm_budget, C.byref(h)), "wcl_init")
        self.h = h
        self.device = device

    def bytes_in_use(self) -> int:
        return lib.wcl_bytes_in_use(self.h)

    def close(self):
        if self.h:
            lib.wcl_finalize(self.h)
            self.h = None


class Lattice:
    """A lattice with resident gauge/clover fields on one device."""

    def __init__(self, ctx: Context, dims, bc=(1, 1, 1, 1)):
        self.ctx = ctx
        self.dims = tuple(int(v) for v in dims)
        h = C.c_void_p()
        check(lib.wcl_create_lattice(ctx.h, (C.c_int * 4)(*self.dims), (C.c_int * 4)(*bc), C.byref(h)))
        self.h = h
        self.V = lib.wcl_volume(h)
        self.device = torch.device("cuda", ctx.device)

    def close(self):
        if self.h:
            lib.wcl_destroy_lattice(self.h)
            self.h = None

    # ---- fields
    def upload_gauge(self, U: np.ndarray, clover: bool = True):
        U = np.ascontiguousarray(U, dtype=np.complex128)
        assert U.size == self.V * 36
        check(lib.wcl_upload_gauge(self.h, U.ctypes.data_as(C.POINTER(C.c_double))))
        if clover:
            check(lib.wcl_compute_clover(self.h))

    def upload_clover(self, Cpacked: np.ndarray):
        Cp = np.ascontiguousarray(Cpacked, dtype=np.float64)
        assert Cp.size == self.V * 72
        check(lib.wcl_upload_clover(self.h, Cp.ctypes.data_as(C.POINTER(C.c_double))))

    def download_clover(self) -> np.ndarray:
        out = np.zeros((self.V, 2, 36), dtype=np.float64)
        check(lib.wcl_download_clover(self.h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    # ---- spinors
    def spinor_bytes(self, prec: int, nrhs: int = 1) -> int:
        return int(lib.wcl_spinor_bytes(self.h, prec, nrhs))

    def empty(self, prec: int, nrhs: int = 1) -> torch.Tensor:
        return torch.empty(self.spinor_bytes(prec, nrhs), dtype=torch.uint8, device=self.device)

    def zeros(self, prec: int, nrhs: int = 1) -> torch.Tensor:
        return torch.zeros(self.spinor_bytes(prec, nrhs), dtype=torch.uint8, device=self.device)

    def pack(self, psi: np.ndarray, prec: int, nrhs: int = 1, out=None, stream=None) -> torch.Tensor:
        """host complex128 [nrhs][V][4][3] -> device buffer (internal layout)."""
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        assert psi.size == nrhs * self.V * 12
        out = self.empty(prec, nrhs) if out is None else out
        check(lib.wcl_pack_spinor(self.h, prec, nrhs, psi.ctypes.data_as(C.POINTER(C.c_double)), _ptr(out),
                                  _stream(stream)))
        return out

    def unpack(self, buf: torch.Tensor, prec: int, nrhs: int = 1, stream=None) -> np.ndarray:
        shape = (self.V, 4, 3) if nrhs == 1 else (nrhs, self.V, 4, 3)
        out = np.zeros(shape, dtype=np.complex128)
        check(lib.wcl_unpack_spinor(self.h, prec, nrhs, _ptr(buf), out.ctypes.data_as(C.POINTER(C.c_double)),
                                    _stream(stream)))
        return out

    # ---- operators
    def apply_D(self, prec, kappa, csw, x: torch.Tensor, out: torch.Tensor, nrhs: int = 1, stream=None):
        check(lib.wcl_apply_D(self.h, prec, kappa, csw, _ptr(x), _ptr(out), nrhs, _stream(stream)))
        return out

    def apply_schur(self, prec, kappa, csw, x: torch.Tensor, out: torch.Tensor, nrhs: int = 1, stream=None):
        check(lib.wcl_apply_schur(self.h, prec, kappa, csw, _ptr(x), _ptr(out), nrhs, _stream(stream)))
        return out

    def block_info(self, ras: RasParams):
        nb, ev = C.c_int64(), C.c_int64()
        check(lib.wcl_block_info(self.h, C.byref(ras), C.byref(nb), C.byref(ev)))
        return nb.value, ev.value

    def apply_D_blocks(self, ras: RasParams, kappa, csw, x: torch.Tensor, stream=None) -> np.ndarray:
        nb, ev = self.block_info(ras)
        out = np.zeros((nb, ev, 4, 3), dtype=np.complex128)
        check(lib.wcl_apply_D_blocks(self.h, C.byref(ras), kappa, csw, _ptr(x),
                                     out.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
        return out

    def ras_precondition(self, ras: RasParams, kappa, csw, r: torch.Tensor, v: torch.Tensor, nrhs: int = 1,
                         stream=None):
        check(lib.wcl_ras_precondition(self.h, C.byref(ras), kappa, csw, _ptr(r), _ptr(v), nrhs, _stream(stream)))
        return v

    def ras_precondition_noalloc(self, ras: RasParams, kappa, csw, r: torch.Tensor, v: torch.Tensor, nrhs: int = 1,
                                 stream=None):
        check(lib.wcl_ras_precondition_noalloc(self.h, C.byref(ras), kappa, csw, _ptr(r), _ptr(v), nrhs,
                                               _stream(stream)))
        return v

    # ---- solvers
    def solve_nested(self, params: SolverParams, kappa, csw, eta: torch.Tensor, phi: torch.Tensor, nrhs: int = 1,
                     stream=None, raise_on_notconv=True):
        st = SolveStats()
        rc = lib.wcl_solve_nested_bicgstab(self.h, C.byref(params), kappa, csw, _ptr(eta), _ptr(phi), nrhs,
                                           C.byref(st), _stream(stream))
        if rc != ENOTCONV or raise_on_notconv:
            check(rc)
        return rc, st.as_dict()

    def solve_bicgstab_f64(self, tol, max_iter, kappa, csw, eta: torch.Tensor, phi: torch.Tensor, stream=None,
                           raise_on_notconv=True):
        st = SolveStats()
        rc = lib.wcl_solve_bicgstab_f64(self.h, tol, max_iter, kappa, csw, _ptr(eta), _ptr(phi), C.byref(st),
                                        _stream(stream))
        if rc != ENOTCONV or raise_on_notconv:
            check(rc)
        return rc, st.as_dict()


# ------------------------------------------------------------------ serving
class ServerParams(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_slots", C.c_int), ("max_queue", C.c_int),
                ("max_batch", C.c_int)]


class Request(C.Structure):
    _fields_ = [("config_id", C.c_uint64), ("kappa", C.c_double), ("csw", C.c_double),
                ("params", C.POINTER(SolverParams)), ("eta_host", C.POINTER(C.c_double)),
                ("phi_host", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("stats", SolveStats), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("batch", C.c_int)]


def _server_sigs():
    vp = C.c_void_p
    sig = {
        "wcl_server_create": (C.c_int, [vp, C.POINTER(ServerParams), C.POINTER(vp)]),
        "wcl_server_destroy": (C.c_int, [vp]),
        "wcl_register_gauge": (C.c_int, [vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
        "wcl_submit": (C.c_int, [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "wcl_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(Result)]),
        "wcl_wait": (C.c_int, [vp, C.c_uint64, C.POINTER(Result)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


_server_sigs()


class Server:
    """Continuous-batching solve server (see include/wcl.h)."""

    def __init__(self, ctx: Context, max_slots: int = 4, hbm_budget: int = 0, max_queue: int = 0,
                 max_batch: int = 1):
        h = C.c_void_p()
        check(lib.wcl_server_create(ctx.h, C.byref(ServerParams(hbm_budget, max_slots, max_queue, max_batch)),
                                    C.byref(h)))
        self.h = h
        self._live = {}   # ticket -> (eta, phi, params) kept alive until collected
        self.dims = {}

    def register_gauge(self, config_id: int, dims, U):
        U = np.ascontiguousarray(U, dtype=np.complex128)
        check(lib.wcl_register_gauge(self.h, config_id, (C.c_int * 4)(*dims), U.ctypes.data_as(C.POINTER(C.c_double))))
        self.dims[config_id] = tuple(dims)

    def submit(self, config_id: int, kappa: float, csw: float, eta, params: SolverParams | None = None,
               phi=None) -> int:
        """Queues a solve; phi (optional, complex128 like eta) receives the solution."""
        eta = np.ascontiguousarray(eta, dtype=np.complex128)
        if phi is None:
            phi = np.zeros_like(eta)
        elif phi.shape != eta.shape or phi.dtype != np.complex128 or not phi.flags.c_contiguous:
            raise ValueError("phi must be a C-contiguous complex128 array shaped like eta")
        p = C.pointer(params) if params is not None else None
        req = Request(config_id, kappa, csw, p, eta.ctypes.data_as(C.POINTER(C.c_double)),
                      phi.ctypes.data_as(C.POINTER(C.c_double)))
        t = C.c_uint64()
        check(lib.wcl_submit(self.h, C.byref(req), C.byref(t)))
        self._live[t.value] = (eta, phi, params)
        return t.value

    def _collect(self, ticket, res):
        eta, phi, _ = self._live.pop(ticket)
        d = {"status": res.status, "t_submit": res.t_submit, "t_admit": res.t_admit, "t_done": res.t_done,
             "batch": res.batch}
        d.update(res.stats.as_dict())
        return phi, d

    def poll(self, ticket: int):
        res = Result()
        rc = lib.wcl_poll(self.h, ticket, C.byref(res))
        if rc == PENDING:
            return None
        check(rc)
        return self._collect(ticket, res)

    def wait(self, ticket: int):
        res = Result()
        check(lib.wcl_wait(self.h, ticket, C.byref(res)))
        return self._collect(ticket, res)

    def close(self):
        if self.h:
            check(lib.wcl_server_destroy(self.h))
            self.h = None
            self._live.clear()


lib.wcl_autotune.restype = C.c_int
lib.wcl_autotune.argtypes = [C.c_void_p, C.POINTER(SolverParams), C.c_double, C.c_double, C.c_void_p, C.c_int,
                             C.c_int, C.c_int, C.c_char_p, C.POINTER(SolverParams), C.POINTER(C.c_double),
                             C.c_void_p]


def autotune(lat: Lattice, base: SolverParams, kappa: float, csw: float, eta: torch.Tensor, nrhs: int = 1,
             cache_path: str | None = None, stream=None, storage=None, storage_mask=None, nsrc: int = 1):
    """Autotuned solver parameters for this lattice, timed on the nsrc tuning
    sources in eta (nsrc x nrhs FP64 spinors, see include/wcl.h).  storage: None = every candidate, F32 = FP32
    storage only, F16 = FP16 storage with either arithmetic; storage_mask
    (bit 0 FP32, bit 1 FP16, bit 2 FP16 with binary16-operand MR steps)
    overrides it."""
    best = SolverParams()
    ms = C.c_double()
    if storage_mask is not None:
        mask = storage_mask
    else:
        mask = 0 if storage is None else (1 if storage == F32 else 6)
    check(lib.wcl_autotune(lat.h, C.byref(base), kappa, csw, _ptr(eta), nrhs, nsrc, mask,
                           cache_path.encode() if cache_path else None, C.byref(best), C.byref(ms), _stream(stream)))
    return best, ms.value

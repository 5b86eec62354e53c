"""Thin ctypes binding of libbpjd.so (include/bpjd.h).

Argument marshalling only: every numeric step runs in the HIP library.  Host
arrays are numpy arrays; device arrays are any object with ``data_ptr()``
(a torch tensor on the GPU), passed with ``mem=MEM_DEVICE``.  If the built
library is missing, importing the functions raises ``LibraryNotBuilt``; there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libbpjd.so")

OK, PENDING = 0, 1
ERR_ARG, ERR_CSR, ERR_DD, ERR_NOT_SPD, ERR_NOCONV, ERR_OOM, ERR_HIP, ERR_OVER_BUDGET, ERR_STATE = \
    -1, -2, -3, -4, -5, -6, -7, -8, -9
MEM_HOST, MEM_DEVICE = 0, 1
STOP_RESIDUAL, STOP_PAPER = 0, 1
CELL_SQUARE, CELL_TRIANGLE = 0, 1
SUBSPACE_UU, SUBSPACE_U, SUBSPACE_GROW = 0, 1, 2
SPMM_PAIRS, SPMM_COLUMN, SPMM_FLAT = 1, 2, 3
PREC_FP64, PREC_MIXED = 0, 1


class LibraryNotBuilt(RuntimeError):
    pass


class BPJDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Csr(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p), ("mem", C.c_int32)]


class DD(C.Structure):
    _fields_ = [("P", Csr), ("n_sub", C.c_int32), ("sub_ptr", C.c_void_p), ("sub_idx", C.c_void_p)]


class DDGeom(C.Structure):
    _fields_ = [("coords", C.c_void_p), ("n_cx", C.c_int32), ("n_cy", C.c_int32),
                ("cx", C.c_void_p), ("cy", C.c_void_p), ("overlap_layers", C.c_int32),
                ("cell_shape", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("guard", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("stop_rule", C.c_int32), ("subspace", C.c_int32), ("precision", C.c_int32),
                ("n_init", C.c_int32), ("X_init", C.c_void_p), ("profile", C.c_int32), ("graphs", C.c_int32),
                ("autotune", C.c_int32), ("local_threads", C.c_int32),
                ("spmm_form", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("stop_value", C.c_double),
                ("max_residual", C.c_double), ("setup_ms", C.c_double), ("iterate_ms", C.c_double),
                ("n_sub", C.c_int32), ("n_coarse", C.c_int32), ("max_local", C.c_int32),
                ("max_band", C.c_int32), ("residuals", C.c_double * 64),
                ("phase_ms", C.c_double * 8), ("phase_count", C.c_int32 * 8),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double), ("graph_iterations", C.c_int32),
                ("spmm_form", C.c_int32)]

    def to_dict(self) -> dict:
        arrays = ("residuals", "phase_ms", "phase_count")
        d = {name: getattr(self, name) for name, _ in self._fields_ if name not in arrays}
        for a in arrays:
            d[a] = list(getattr(self, a))
        return d


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("queued", C.c_uint32), ("running", C.c_uint32), ("peak_running", C.c_uint32),
                ("max_slots", C.c_uint32), ("budget_bytes", C.c_uint64), ("bytes_in_use", C.c_uint64),
                ("peak_bytes", C.c_uint64)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


PHASES = ["local", "spmm", "coarse", "gather_scatter", "ortho", "rr", "residual", "setup"]


_lib = None

EXPORTS = {
    "bpjd_opts_default": (None, [C.POINTER(Opts), C.c_int32]),
    "bpjd_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "bpjd_ctx_destroy": (None, [C.c_void_p]),
    "bpjd_problem_create": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.POINTER(Csr), C.POINTER(DD), C.POINTER(Opts),
                                      C.POINTER(C.c_void_p)]),
    "bpjd_problem_create_geom": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.POINTER(Csr), C.POINTER(DDGeom),
                                           C.POINTER(Opts), C.POINTER(C.c_void_p)]),
    "bpjd_problem_destroy": (None, [C.c_void_p]),
    "bpjd_problem_set_values": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "bpjd_problem_dims": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "bpjd_problem_local_sizes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "bpjd_problem_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "bpjd_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Stats)]),
    "bpjd_setup": (C.c_int, [C.c_void_p]),
    "bpjd_apply_preconditioner": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "bpjd_spmm": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    "bpjd_coarse_eigenvalues": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "bpjd_coarse_eigen_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p]),
    "bpjd_server_create": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]),
    "bpjd_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Csr), C.POINTER(Csr), C.POINTER(DD), C.POINTER(DDGeom),
                                     C.POINTER(Opts), C.POINTER(C.c_uint64)]),
    "bpjd_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.POINTER(Stats)]),
    "bpjd_server_get_info": (C.c_int, [C.c_void_p, C.POINTER(ServerInfo)]),
    "bpjd_server_destroy": (None, [C.c_void_p]),
    "bpjd_strerror": (C.c_char_p, [C.c_int]),
    "bpjd_last_error": (C.c_char_p, [C.c_void_p]),
}


def lib():
    """Load libbpjd.so (raises LibraryNotBuilt if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryNotBuilt(f"{LIB_PATH} not found: run `python -m paper_2203_06327_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code < 0:
        L = lib()
        raise BPJDError(code, f"{L.bpjd_strerror(code).decode()}: {L.bpjd_last_error(None).decode()}")
    return code


def _ptr(a) -> int:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _geom(geom, keep: list) -> DDGeom:
    """(coords, cx, cy, layers[, cell_shape]) -> bpjd_dd_geom (host arrays kept alive in keep)."""
    coords, cx, cy, layers = geom[:4]
    shape = geom[4] if len(geom) > 4 else CELL_SQUARE
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cx = np.ascontiguousarray(cx, dtype=np.float64)
    cy = np.ascontiguousarray(cy, dtype=np.float64)
    keep += [coords, cx, cy]
    return DDGeom(coords.ctypes.data, len(cx), len(cy), cx.ctypes.data, cy.ctypes.data, int(layers), int(shape))


@dataclass
class _Keep:
    arrays: list


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Device memory of a context from PyTorch's caching allocator, on the context's
    stream (a torch stream made for it).  Counts calls and bytes, so a test can see
    every device byte the library holds."""

    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self.live = {}                  # ptr -> bytes
        self.allocs = self.frees = 0
        self.bytes_allocated = 0
        self._alloc = ALLOC_FN(self._on_alloc)
        self._free = FREE_FN(self._on_free)
        self.struct = Allocator(self._alloc, self._free, None)

    def _on_alloc(self, nbytes, user):
        try:
            ptr = self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:
            return None
        self.live[ptr] = int(nbytes)
        self.allocs += 1
        self.bytes_allocated += int(nbytes)
        return ptr

    def _on_free(self, ptr, user):
        self.live.pop(ptr, None)
        self.frees += 1
        self.torch.cuda.caching_allocator_delete(ptr)

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())


class Context:
    """A device, a stream and a device-memory provider (bpjd_ctx).  allocator: None
    (hipMalloc) or "torch" (PyTorch's caching allocator on a torch stream)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, allocator: Optional[str] = None):
        h = C.c_void_p()
        self.allocator = None
        al = None
        if allocator == "torch":
            self.allocator = TorchAllocator(device)
            al = C.byref(self.allocator.struct)
            if stream is None:
                stream = self.allocator.stream.cuda_stream
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        _check(lib().bpjd_ctx_create(device, al, stream, C.byref(h)))
        self.handle = h

    def last_error(self) -> str:
        return lib().bpjd_last_error(self.handle).decode()

    def close(self):
        if self.handle:
            lib().bpjd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceCSR:
    """A CSR matrix resident in device memory (torch tensors on the GPU): int32 row
    pointers and columns, float64 values; passed to the library as BPJD_MEM_DEVICE."""

    def __init__(self, A, device: int = 0):
        import torch
        dev = torch.device("cuda", device)
        self.shape = A.shape
        self.nnz = A.nnz
        self.rowptr = torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int32)).to(dev)
        self.col = torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).to(dev)
        self.val = torch.from_numpy(np.ascontiguousarray(A.data, dtype=np.float64)).to(dev)


def _csr(A, keep: list) -> Csr:
    """scipy CSR (host) or DeviceCSR -> bpjd_csr with int32 indices and float64 values."""
    if isinstance(A, DeviceCSR):
        keep.append(A)
        return Csr(A.shape[0], A.shape[1], A.nnz, A.rowptr.data_ptr(), A.col.data_ptr(), A.val.data_ptr(),
                   MEM_DEVICE)
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int32)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = np.ascontiguousarray(A.data, dtype=np.float64)
    keep += [rowptr, col, val]
    return Csr(A.shape[0], A.shape[1], A.nnz, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, MEM_HOST)


def make_opts(k: int, guard: int = 0, tol: float = 1e-8, max_iter: int = 500, stop_rule: int = STOP_RESIDUAL,
              subspace: int = SUBSPACE_UU, precision: int = PREC_MIXED, X_init: Optional[np.ndarray] = None,
              keep: Optional[list] = None, profile: int = 0, graphs: bool = True, autotune: bool = True,
              local_threads: int = 0, spmm_form: int = 0) -> Opts:
    o = Opts()
    lib().bpjd_opts_default(C.byref(o), k)
    o.guard, o.tol, o.max_iter, o.stop_rule, o.subspace, o.precision = guard, tol, max_iter, stop_rule, subspace, precision
    o.profile = int(profile)
    o.graphs = 1 if graphs else 0
    o.autotune = 1 if autotune else 0
    o.local_threads = int(local_threads)
    o.spmm_form = int(spmm_form)
    if X_init is not None:
        Xi = np.ascontiguousarray(X_init, dtype=np.float64)
        if keep is not None:
            keep.append(Xi)
        o.n_init = Xi.shape[1]
        o.X_init = Xi.ctypes.data
    return o


class Problem:
    """A BPJD problem on one GPU (wraps bpjd_problem)."""

    def __init__(self, ctx: Context, K, M, *, dd=None, geom=None, k: int, guard: int = 0, tol: float = 1e-8,
                 max_iter: int = 500, stop_rule: int = STOP_RESIDUAL, subspace: int = SUBSPACE_UU,
                 precision: int = PREC_MIXED, X_init: Optional[np.ndarray] = None, profile: int = 0,
                 graphs: bool = True, autotune: bool = True, local_threads: int = 0, spmm_form: int = 0):
        keep: list = []
        Kc, Mc = _csr(K, keep), _csr(M, keep)
        opts = make_opts(k, guard, tol, max_iter, stop_rule, subspace, precision, X_init, keep, profile, graphs,
                         autotune, local_threads, spmm_form)
        h = C.c_void_p()
        if geom is not None:
            g = _geom(geom, keep)
            _check(lib().bpjd_problem_create_geom(ctx.handle, C.byref(Kc), C.byref(Mc), C.byref(g), C.byref(opts),
                                                  C.byref(h)))
        elif dd is not None:
            P, subs = dd
            Pc = _csr(P, keep)
            sub_ptr = np.zeros(len(subs) + 1, dtype=np.int32)
            sub_ptr[1:] = np.cumsum([len(S) for S in subs])
            sub_idx = np.ascontiguousarray(np.concatenate([np.asarray(S) for S in subs]), dtype=np.int32)
            keep += [sub_ptr, sub_idx]
            d = DD(Pc, len(subs), sub_ptr.ctypes.data, sub_idx.ctypes.data)
            _check(lib().bpjd_problem_create(ctx.handle, C.byref(Kc), C.byref(Mc), C.byref(d), C.byref(opts),
                                             C.byref(h)))
        else:
            raise ValueError("give dd=(P, subdomains) or geom=(coords, cx, cy, layers)")
        self.ctx = ctx
        self.handle = h
        self.k = k
        n, nH, nsub, s = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().bpjd_problem_dims(h, C.byref(n), C.byref(nH), C.byref(nsub), C.byref(s)))
        self.n, self.n_coarse, self.n_sub, self.s = n.value, nH.value, nsub.value, s.value

    def close(self):
        if getattr(self, "handle", None):
            lib().bpjd_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, eigvals=None, eigvecs=None, mem: int = MEM_HOST, raise_noconv: bool = True):
        """Run Algorithm 3.1; returns (eigvals, eigvecs, stats dict).  Host outputs are allocated
        when not given; device outputs must be given (torch tensors)."""
        if mem == MEM_HOST:
            if eigvals is None:
                eigvals = np.empty(self.k)
            if eigvecs is None:
                eigvecs = np.empty((self.n, self.k))
        st = Stats()
        code = lib().bpjd_solve(self.handle, _ptr(eigvals), _ptr(eigvecs), mem, C.byref(st))
        if code != ERR_NOCONV or raise_noconv:
            _check(code)
        return eigvals, eigvecs, st.to_dict()

    def footprint(self) -> int:
        b = C.c_uint64()
        _check(lib().bpjd_problem_footprint(self.handle, C.byref(b)))
        return b.value

    def local_sizes(self):
        nl = np.empty(self.n_sub, dtype=np.int32)
        bw = np.empty(self.n_sub, dtype=np.int32)
        _check(lib().bpjd_problem_local_sizes(self.handle, _ptr(nl), _ptr(bw)))
        return nl, bw

    def setup(self):
        _check(lib().bpjd_setup(self.handle))

    def apply_preconditioner(self, X: np.ndarray, lam: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        Z = np.empty_like(X)
        _check(lib().bpjd_apply_preconditioner(self.handle, _ptr(X), _ptr(lam), _ptr(Z), MEM_HOST))
        return Z

    def spmm(self, X: np.ndarray):
        X = np.ascontiguousarray(X, dtype=np.float64)
        KX = np.empty_like(X)
        MX = np.empty_like(X)
        _check(lib().bpjd_spmm(self.handle, _ptr(X), X.shape[1], _ptr(KX), _ptr(MX), MEM_HOST))
        return KX, MX

    def coarse_eigenvalues(self) -> np.ndarray:
        out = np.empty(self.n_coarse)
        _check(lib().bpjd_coarse_eigenvalues(self.handle, _ptr(out), MEM_HOST))
        return out


def problem_from_mesh(ctx: Context, mesh, layers: int, shape: int = CELL_SQUARE, **kw) -> Problem:
    """Problem on a structured P1 mesh (coarse grid lines and coordinates from the mesh);
    shape: subdomains are coarse cells (CELL_SQUARE) or coarse triangles (CELL_TRIANGLE)."""
    return Problem(ctx, mesh.K, mesh.M, geom=(mesh.coords, mesh.cx, mesh.cy, layers, shape), **kw)


class Server:
    """Continuous-batching eigensolver server on one GPU (wraps bpjd_server).

    ``submit`` queues a problem and returns its id; ``poll`` returns None while it is
    queued or running, else (eigvals, eigvecs, stats dict) (raises on an error status).
    """

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_slots: int = 8):
        h = C.c_void_p()
        _check(lib().bpjd_server_create(ctx.handle, int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.ctx = ctx
        self.handle = h
        self._shape = {}

    def submit(self, K, M, *, geom=None, dd=None, k: int, guard: int = 0, tol: float = 1e-8, max_iter: int = 500,
               stop_rule: int = STOP_RESIDUAL, subspace: int = SUBSPACE_UU, precision: int = PREC_MIXED,
               X_init: Optional[np.ndarray] = None) -> int:
        keep: list = []
        Kc, Mc = _csr(K, keep), _csr(M, keep)
        opts = make_opts(k, guard, tol, max_iter, stop_rule, subspace, precision, X_init, keep, 0)
        rid = C.c_uint64()
        if geom is not None:
            g = _geom(geom, keep)
            _check(lib().bpjd_server_submit(self.handle, C.byref(Kc), C.byref(Mc), None, C.byref(g),
                                            C.byref(opts), C.byref(rid)))
        elif dd is not None:
            P, subs = dd
            Pc = _csr(P, keep)
            sub_ptr = np.zeros(len(subs) + 1, dtype=np.int32)
            sub_ptr[1:] = np.cumsum([len(S) for S in subs])
            sub_idx = np.ascontiguousarray(np.concatenate([np.asarray(S) for S in subs]), dtype=np.int32)
            keep += [sub_ptr, sub_idx]
            d = DD(Pc, len(subs), sub_ptr.ctypes.data, sub_idx.ctypes.data)
            _check(lib().bpjd_server_submit(self.handle, C.byref(Kc), C.byref(Mc), C.byref(d), None,
                                            C.byref(opts), C.byref(rid)))
        else:
            raise ValueError("give dd=(P, subdomains) or geom=(coords, cx, cy, layers)")
        self._shape[rid.value] = (K.shape[0], k)
        return rid.value

    def submit_mesh(self, mesh, layers: int, shape: int = CELL_SQUARE, **kw) -> int:
        return self.submit(mesh.K, mesh.M, geom=(mesh.coords, mesh.cx, mesh.cy, layers, shape), **kw)

    def poll(self, req_id: int, raise_noconv: bool = True):
        n, k = self._shape.get(req_id, (0, 0))      # an unknown id is the library's error
        lam = np.empty(k)
        X = np.empty((n, k))
        st = Stats()
        code = lib().bpjd_server_poll(self.handle, req_id, lam.ctypes.data if k else None,
                                      X.ctypes.data if k else None, C.byref(st))
        if code == PENDING:
            return None
        self._shape.pop(req_id, None)
        if code != ERR_NOCONV or raise_noconv:
            _check(code)
        return lam, X, st.to_dict()

    def info(self) -> dict:
        inf = ServerInfo()
        _check(lib().bpjd_server_get_info(self.handle, C.byref(inf)))
        return inf.to_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().bpjd_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coarse_eigen_noalloc(ctx: Context, KH, MH, bw: int, lamH, Y, info) -> None:
    """bpjd_coarse_eigen_noalloc on device tensors (KH, MH, lamH, Y: float64; info:
    int32): enqueued on the context's stream, no allocation, no synchronisation."""
    _check(lib().bpjd_coarse_eigen_noalloc(ctx.handle, int(KH.shape[0]), int(bw), _ptr(KH), _ptr(MH), _ptr(lamH),
                                           _ptr(Y), _ptr(info)))

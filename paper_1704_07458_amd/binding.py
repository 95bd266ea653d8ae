"""ctypes binding of liblobpcg_mi355x.so (include/lobpcg.h, include/lobpcg_steps.h).

Argument marshalling only: every step of the eigensolver runs in the library's
HIP kernels.  torch supplies device memory and the current stream.  There is no
CPU fallback: if the library is missing, load() raises.
"""

from __future__ import annotations

import ctypes as C
import os
import warnings
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblobpcg_mi355x.so")

LOBPCG_OK = 0
LOBPCG_NOT_CONVERGED = 1
STATUS_NAMES = {
    0: "OK",
    1: "NOT_CONVERGED",
    -1: "ERR_ARG",
    -2: "ERR_ALLOC",
    -3: "ERR_HIP",
    -4: "ERR_BREAKDOWN",
    -5: "ERR_NONFINITE",
    -6: "ERR_CALLBACK",
    -7: "ERR_STATE",
}


class LobpcgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class lobpcg_csr(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("rowptr", C.c_void_p),
        ("colind", C.c_void_p),
        ("values", C.c_void_p),
        ("on_device", C.c_int32),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_int32)


class lobpcg_zcsr(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("rowptr", C.c_void_p),
        ("colind", C.c_void_p),
        ("values_re", C.c_void_p),
        ("values_im", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class lobpcg_options(C.Structure):
    _fields_ = [
        ("block_size", C.c_int32),
        ("maxit", C.c_int32),
        ("precision", C.c_int32),
        ("precond", C.c_int32),
        ("implicit_products", C.c_int32),
        ("lq_literal", C.c_int32),
        ("tau_ortho", C.c_double),
        ("drop_factor", C.c_double),
        ("replace_factor", C.c_double),
        ("skip_factor", C.c_double),
        ("fp32_tol", C.c_double),
        ("seed", C.c_uint64),
        ("stream", C.c_void_p),
        ("ortho_mode", C.c_int32),
        ("force_ortho", C.c_int32),
        ("implicit_gram", C.c_int32),
        ("basic", C.c_int32),
        ("largest", C.c_int32),
        ("dev_alloc", ALLOC_FN),
        ("dev_free", FREE_FN),
        ("alloc_user", C.c_void_p),
        ("progress", PROGRESS_FN),
        ("progress_user", C.c_void_p),
    ]


class lobpcg_info(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("n_converged", C.c_int32),
        ("ortho_switch_iter", C.c_int32),
        ("fp32_iterations", C.c_int32),
        ("fp64_iterations", C.c_int32),
        ("svqb_calls", C.c_int32),
        ("ortho_calls", C.c_int32),
        ("flips", C.c_int32),
        ("norm_A_est", C.c_double),
        ("norm_B_est", C.c_double),
        ("seconds_total", C.c_double),
        ("seconds_phase", C.c_double * 8),
        ("explicit_xp_steps", C.c_int32),
        ("fp32_fallback", C.c_int32),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "seconds_phase"}
        names = ["spmm", "precond", "ortho", "gram", "rr", "update", "residual", "other"]
        d["seconds_phase"] = dict(zip(names, list(self.seconds_phase)))
        return d


class lobpcg_kernel_stat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("work", C.c_double)]


KERNEL_KINDS = ["spmm", "gram", "update", "residual", "rayleigh_ritz", "tridiagonalise",
                "tridiagonal_eig", "qr_backtransform", "cholesky_inverse"]

PRECOND_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                         C.c_int64, C.c_void_p, C.c_int64, C.c_void_p)

_lib = None

# Exported symbols and their signatures (restype, argtypes).
SIGNATURES = {
    "lobpcg_default_options": (None, [C.POINTER(lobpcg_options)]),
    "lobpcg_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(lobpcg_csr),
                                C.POINTER(lobpcg_csr), C.c_int32, C.POINTER(lobpcg_options)]),
    "lobpcg_solve": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_int32, PRECOND_FN,
                               C.c_void_p, C.POINTER(lobpcg_info)]),
    "lobpcg_eigpairs": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_int32]),
    "lobpcg_adjoint": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                 C.POINTER(C.c_int32)]),
    "lobpcg_create_hermitian": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(lobpcg_zcsr),
                                          C.POINTER(lobpcg_zcsr), C.c_int32,
                                          C.POINTER(lobpcg_options)]),
    "lobpcg_solve_hermitian": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                         C.c_int32, PRECOND_FN, C.c_void_p,
                                         C.POINTER(lobpcg_info)]),
    "lobpcg_eigpairs_hermitian": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_int64, C.c_void_p, C.c_int32]),
    "lobpcg_dims": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32)]),
    "lobpcg_destroy": (None, [C.c_void_p]),
    "lobpcg_last_error": (C.c_char_p, []),
    "lobpcg_set_profiling": (C.c_int, [C.c_void_p, C.c_int32]),
    "lobpcg_kernel_stats": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(lobpcg_kernel_stat)]),
    "lobpcg_spmm": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                              C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                              C.c_void_p]),
    "lobpcg_gram_workspace": (C.c_int64, [C.c_int64, C.c_int32, C.c_int32, C.c_int32]),
    "lobpcg_gram": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                              C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                              C.c_void_p]),
    "lobpcg_gram_noalloc": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                      C.c_void_p]),
    "lobpcg_gram_noalloc_max_bytes": (C.c_int64, []),
    "lobpcg_update": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                C.c_int64, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                C.c_void_p, C.c_int64, C.c_void_p]),
    "lobpcg_residual_workspace": (C.c_int64, [C.c_int64, C.c_int32]),
    "lobpcg_residual": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                  C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lobpcg_spmm_residual_workspace": (C.c_int64, [C.c_int64, C.c_int32]),
    "lobpcg_spmm_residual": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_double,
                                       C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "lobpcg_rr_step": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_void_p]),
}


# ROCm libraries the HIP library needs, in load order.  A process can hold only
# one HIP runtime: when torch ships its own copies (same sonames), those must be
# the ones the library binds to, so they are loaded first.
_ROCM_DEPS = ["libhsa-runtime64.so", "libamdhip64.so", "librocblas.so", "librocsolver.so"]


def _share_torch_runtime():
    try:
        import torch
    except Exception:
        return
    tlib = os.path.join(os.path.dirname(torch.__file__), "lib")
    for name in _ROCM_DEPS:
        path = os.path.join(tlib, name)
        if os.path.exists(path):
            C.CDLL(path, mode=C.RTLD_GLOBAL)


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} not found: build it with `python -m paper_1704_07458_amd.build`; "
            "there is no CPU fallback")
    _share_torch_runtime()
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> int:
    if code < 0:
        raise LobpcgError(code, load().lobpcg_last_error().decode())
    return code


def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_options() -> lobpcg_options:
    o = lobpcg_options()
    load().lobpcg_default_options(C.byref(o))
    return o


def _csr_struct(M, keep: list):
    """lobpcg_csr for a problems.CSR (host numpy) or a dict of device tensors."""
    s = lobpcg_csr()
    if isinstance(M, dict):
        rp, ci, va = M["rowptr"], M["colind"], M["values"]
        s.n, s.nnz = int(rp.numel() - 1), int(ci.numel())
        s.rowptr, s.colind, s.values = _ptr(rp), _ptr(ci), _ptr(va)
        s.on_device = 1
        keep.extend([rp, ci, va])
    else:
        rp = np.ascontiguousarray(M.rowptr, dtype=np.int64)
        ci = np.ascontiguousarray(M.colind, dtype=np.int32)
        va = np.ascontiguousarray(M.values, dtype=np.float64)
        keep.extend([rp, ci, va])
        s.n, s.nnz = int(M.n), int(ci.size)
        s.rowptr = rp.ctypes.data
        s.colind = ci.ctypes.data
        s.values = va.ctypes.data
        s.on_device = 0
    return s


def _zcsr_struct(M, keep: list):
    """lobpcg_zcsr for a problems.ZCSR (host numpy) or a dict of device tensors
    (rowptr, colind, values_re, values_im)."""
    s = lobpcg_zcsr()
    if isinstance(M, dict):
        rp, ci, vr, vi = M["rowptr"], M["colind"], M["values_re"], M["values_im"]
        s.n, s.nnz = int(rp.numel() - 1), int(ci.numel())
        s.rowptr, s.colind = _ptr(rp), _ptr(ci)
        s.values_re, s.values_im = _ptr(vr), _ptr(vi)
        s.on_device = 1
        keep.extend([rp, ci, vr, vi])
    else:
        arrs = [np.ascontiguousarray(M.rowptr, dtype=np.int64),
                np.ascontiguousarray(M.colind, dtype=np.int32),
                np.ascontiguousarray(M.values_re, dtype=np.float64),
                np.ascontiguousarray(M.values_im, dtype=np.float64)]
        keep.extend(arrs)
        s.n, s.nnz = int(M.n), int(arrs[1].size)
        s.rowptr, s.colind, s.values_re, s.values_im = [a.ctypes.data for a in arrs]
        s.on_device = 0
    return s


class TorchAllocator:
    """dev_alloc / dev_free hooks that take the handle's device memory from torch's
    caching allocator on the given stream (lobpcg_options.dev_alloc)."""

    def __init__(self, stream=None):
        import torch

        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        self.live = 0  # bytes currently handed out
        self._sizes = {}
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            p = int(self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                             self.stream))
            self._sizes[p] = int(nbytes)
            self.live += int(nbytes)
            return p
        except Exception:
            return None

    def _free(self, ptr, user):
        try:
            self.live -= self._sizes.pop(int(ptr), 0)
            self._torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass


class Solver:
    """Handle around lobpcg_create / solve / eigpairs / adjoint / destroy.

    allocator: "torch" (default) routes every device allocation of the handle
    through torch's caching allocator on the current stream (the dev_alloc /
    dev_free hooks of lobpcg_options); "hip" lets the library call hipMalloc.
    """

    def __init__(self, A, k: int, B=None, precond: str = "none", precision: str = "fp64",
                 block_size: int = 0, maxit: int = 2000, allocator: str = "torch",
                 progress=None, **opts):
        lib = load()
        o = self._options(precond, precision, block_size, maxit, allocator, progress, opts)
        keep: list = []
        a = _csr_struct(A, keep)
        b = _csr_struct(B, keep) if B is not None else None
        h = C.c_void_p()
        check(lib.lobpcg_create(C.byref(h), C.byref(a), C.byref(b) if b is not None else None,
                                int(k), C.byref(o)))
        self._finish(h, k, a, b)

    def _finish(self, h, k, a, b):
        lib = load()
        self._h = h
        self.k = int(k)
        n = C.c_int64()
        kk = C.c_int32()
        nx = C.c_int32()
        check(lib.lobpcg_dims(h, C.byref(n), C.byref(kk), C.byref(nx)))
        self.n, self.n_x = int(n.value), int(nx.value)
        self.nnz_A = int(a.nnz)
        self.nnz_B = int(b.nnz) if b is not None else None

    def _options(self, precond, precision, block_size, maxit, allocator, progress, opts):
        o = default_options()
        # progress(iteration, n_converged, phase) after every iteration (phase 1 = FP32)
        self._progress = None
        if progress is not None:
            self._progress = PROGRESS_FN(lambda user, it, nc, ph: progress(it, nc, ph))
            o.progress = self._progress
        o.block_size = block_size
        o.maxit = maxit
        o.precision = {"fp64": 0, "split": 1, "fp32-split": 1}[precision]
        self._callback = None
        if callable(precond):
            o.precond = 2
            self._callback = precond
        else:
            o.precond = {"none": 0, None: 0, "jacobi": 1}[precond]
        for key, val in opts.items():
            setattr(o, key, val)
        o.stream = _stream()
        self._alloc = None
        if allocator == "torch":
            self._alloc = TorchAllocator()
            o.dev_alloc = self._alloc.alloc_fn
            o.dev_free = self._alloc.free_fn
        elif allocator != "hip":
            raise ValueError("allocator must be 'torch' or 'hip'")
        return o

    def close(self):
        if getattr(self, "_h", None):
            load().lobpcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on: bool):
        check(load().lobpcg_set_profiling(self._h, 1 if on else 0))

    def kernel_stats(self, enable: bool) -> dict:
        """Per-kernel-class HIP-event totals since the last reset; then (re)enable or stop."""
        arr = (lobpcg_kernel_stat * len(KERNEL_KINDS))()
        check(load().lobpcg_kernel_stats(self._h, 1 if enable else 0, arr))
        return {name: {"launches": int(arr[i].launches), "seconds": float(arr[i].seconds),
                       "work": float(arr[i].work)} for i, name in enumerate(KERNEL_KINDS)}

    def solve(self, tol: float, X0=None) -> dict:
        """Run Algorithm 8.  X0: None, a host numpy array or a device tensor (n x n_x)."""
        import torch

        lib = load()
        info = lobpcg_info()
        keep = None
        if X0 is None:
            ptr, dev = None, 0
        elif isinstance(X0, np.ndarray):
            keep = np.ascontiguousarray(X0, dtype=np.float64)
            assert keep.shape == (self.n, self.n_x)
            ptr, dev = keep.ctypes.data, 0
        else:
            keep = X0.to(torch.float64).contiguous()
            assert tuple(keep.shape) == (self.n, self.n_x)
            ptr, dev = _ptr(keep), 1
        cb = PRECOND_FN(self._precond_trampoline) if self._callback else PRECOND_FN()
        self._cb_ref = cb
        code = check(lib.lobpcg_solve(self._h, float(tol), ptr, dev, cb, None, C.byref(info)))
        d = info.as_dict()
        d["status"] = STATUS_NAMES[code]
        d["converged"] = code == LOBPCG_OK
        return d

    def _precond_trampoline(self, user, n, ncols, dtype, R, ldr, W, ldw, stream):
        import torch

        try:
            dt = torch.float64 if dtype == 0 else torch.float32
            self._callback(n, ncols, dt, R, ldr, W, ldw, stream)
            return 0
        except Exception:
            return 1

    def eigpairs(self, count: Optional[int] = None):
        """(lambda, X, rho) as device tensors: count values, n x count, count values."""
        import torch

        count = self.k if count is None else int(count)
        lam = torch.empty(count, dtype=torch.float64, device="cuda")
        X = torch.empty((self.n, count), dtype=torch.float64, device="cuda")
        rho = torch.empty(count, dtype=torch.float64, device="cuda")
        check(load().lobpcg_eigpairs(self._h, count, _ptr(lam), _ptr(X), count, _ptr(rho), 1))
        return lam, X, rho

    def adjoint(self, count: int, lambda_bar, X_bar, cg_tol: float = 1e-12, cg_maxit: int = 0,
                want_B: bool = False):
        """Gradient on the stored values of A (device tensor of nnz(A) values) and the
        largest CG iteration count; with want_B (B != I) also the gradient on B's
        stored values: (grad_A, iters, grad_B)."""
        import torch

        grad = torch.empty(self.nnz_A, dtype=torch.float64, device="cuda")
        gB = None
        if want_B:
            if self.nnz_B is None:
                raise ValueError("want_B needs a pencil with B != I")
            gB = torch.empty(self.nnz_B, dtype=torch.float64, device="cuda")
        lb = None
        if lambda_bar is not None:
            lb = np.ascontiguousarray(np.asarray(lambda_bar, dtype=np.float64))
        xb = X_bar.to(torch.float64).contiguous() if X_bar is not None else None
        iters = C.c_int32()
        st = check(load().lobpcg_adjoint(self._h, int(count),
                                         lb.ctypes.data if lb is not None else None,
                                         _ptr(xb) if xb is not None else None, int(count),
                                         _ptr(grad), _ptr(gB) if gB is not None else None,
                                         float(cg_tol), int(cg_maxit), C.byref(iters)))
        if st == LOBPCG_NOT_CONVERGED:
            warnings.warn(f"lobpcg_adjoint: projected CG reached cg_maxit ({int(iters.value)}) "
                          f"above cg_tol {cg_tol:g}", RuntimeWarning, stacklevel=2)
        if want_B:
            return grad, int(iters.value), gB
        return grad, int(iters.value)


# ---------------------------------------------------------------- step calls
class HermitianSolver(Solver):
    """Handle around lobpcg_create_hermitian / solve_hermitian / eigpairs_hermitian:
    the k smallest (or largest) eigenpairs of a complex Hermitian pencil, run by
    the library on the real embedding [Re A, -Im A; Im A, Re A]."""

    def __init__(self, A, k: int, B=None, precond: str = "none", precision: str = "fp64",
                 block_size: int = 0, maxit: int = 2000, allocator: str = "torch",
                 progress=None, **opts):
        lib = load()
        o = self._options(precond, precision, block_size, maxit, allocator, progress, opts)
        keep: list = []
        a = _zcsr_struct(A, keep)
        b = _zcsr_struct(B, keep) if B is not None else None
        h = C.c_void_p()
        check(lib.lobpcg_create_hermitian(C.byref(h), C.byref(a),
                                          C.byref(b) if b is not None else None, int(k),
                                          C.byref(o)))
        self._finish(h, k, a, b)

    def solve(self, tol: float, X0=None) -> dict:
        """X0: None, a complex host numpy array or a complex device tensor (n x n_x)."""
        import torch

        lib = load()
        info = lobpcg_info()
        keep = []
        if X0 is None:
            pre = pim = None
            dev = 0
        elif isinstance(X0, np.ndarray):
            assert X0.shape == (self.n, self.n_x)
            keep = [np.ascontiguousarray(X0.real, dtype=np.float64),
                    np.ascontiguousarray(X0.imag, dtype=np.float64)]
            pre, pim, dev = keep[0].ctypes.data, keep[1].ctypes.data, 0
        else:
            assert tuple(X0.shape) == (self.n, self.n_x)
            keep = [X0.real.to(torch.float64).contiguous(),
                    X0.imag.to(torch.float64).contiguous()]
            pre, pim, dev = _ptr(keep[0]), _ptr(keep[1]), 1
        cb = PRECOND_FN(self._precond_trampoline) if self._callback else PRECOND_FN()
        self._cb_ref = cb
        code = check(lib.lobpcg_solve_hermitian(self._h, float(tol), pre, pim, dev, cb, None,
                                                C.byref(info)))
        d = info.as_dict()
        d["status"] = STATUS_NAMES[code]
        d["converged"] = code == LOBPCG_OK
        return d

    def eigpairs(self, count: Optional[int] = None):
        """(lambda, X, rho) as device tensors: count values, complex n x count, count values."""
        import torch

        count = self.k if count is None else int(count)
        lam = torch.empty(count, dtype=torch.float64, device="cuda")
        Xr = torch.empty((self.n, count), dtype=torch.float64, device="cuda")
        Xi = torch.empty((self.n, count), dtype=torch.float64, device="cuda")
        rho = torch.empty(count, dtype=torch.float64, device="cuda")
        check(load().lobpcg_eigpairs_hermitian(self._h, count, _ptr(lam), _ptr(Xr), _ptr(Xi),
                                               count, _ptr(rho), 1))
        return lam, torch.complex(Xr, Xi), rho

    def adjoint(self, *args, **kwargs):
        raise NotImplementedError("the adjoint is for real pencils")


def _dtype_code(t) -> int:
    import torch

    return 0 if t.dtype == torch.float64 else 1


def spmm(rowptr, colind, values, X, Y=None):
    """Y = A X for device CSR tensors and a row-major device block X."""
    import torch

    n, ncols = X.shape
    if Y is None:
        Y = torch.empty_like(X)
    check(load().lobpcg_spmm(n, _ptr(rowptr), _ptr(colind), _ptr(values), _dtype_code(X), _ptr(X),
                             X.stride(0), _ptr(Y), Y.stride(0), ncols, _stream()))
    return Y


def gram(L, R1, R2=None, col_offset: int = 0, mirror: bool = False, out=None):
    """G(:, col_offset:col_offset+p) = L^T [R1 | R2] in FP64.

    Returns the column-major output as an (ldg x ncols) view of element (i, j);
    with mirror=True the rows above col_offset are also written transposed,
    completing a symmetric m x m matrix (m = col_offset + p).
    """
    import torch

    n, m = L.shape
    p1 = R1.shape[1]
    p = p1 + (R2.shape[1] if R2 is not None else 0)
    ldg = max(m, col_offset + p)
    ws = load().lobpcg_gram_workspace(n, m, p, _dtype_code(L))
    work = torch.empty(max(ws, 8), dtype=torch.uint8, device="cuda")
    if out is None:
        out = torch.zeros((col_offset + p, ldg), dtype=torch.float64, device="cuda")
    check(load().lobpcg_gram(n, m, p, p1, _dtype_code(L), _ptr(L), L.stride(0), _ptr(R1),
                             R1.stride(0), _ptr(R2) if R2 is not None else None,
                             R2.stride(0) if R2 is not None else 0, _ptr(out), ldg, col_offset,
                             1 if mirror else 0, _ptr(work), _stream()))
    # column-major: tensor row j holds column j
    G = out.t()
    return G[:m, col_offset:col_offset + p] if not mirror else G[:m, :col_offset + p]


def gram_noalloc(L, R1, R2=None, col_offset: int = 0, mirror: bool = False, out=None):
    """As gram(), through lobpcg_gram_noalloc (no workspace: the library's fixed
    device scratch array).  `out` must be preallocated by the caller when the call
    may not allocate (e.g. under graph capture)."""
    import torch

    n, m = L.shape
    p1 = R1.shape[1]
    p = p1 + (R2.shape[1] if R2 is not None else 0)
    ldg = max(m, col_offset + p)
    if out is None:
        out = torch.zeros((col_offset + p, ldg), dtype=torch.float64, device="cuda")
    check(load().lobpcg_gram_noalloc(n, m, p, p1, _dtype_code(L), _ptr(L), L.stride(0), _ptr(R1),
                                     R1.stride(0), _ptr(R2) if R2 is not None else None,
                                     R2.stride(0) if R2 is not None else 0, _ptr(out), ldg,
                                     col_offset, 1 if mirror else 0, _stream()))
    G = out.t()
    return G[:m, col_offset:col_offset + p] if not mirror else G[:m, :col_offset + p]


def update(S, Cmat, Y=None, alpha: float = 1.0, beta: float = 0.0):
    """Y = beta Y + alpha S C with C an FP64 (K x N) matrix."""
    import torch

    n, K = S.shape
    N = Cmat.shape[1]
    Ccm = Cmat.to(torch.float64).t().contiguous()  # column-major storage of C
    if Y is None:
        Y = torch.zeros((n, N), dtype=S.dtype, device="cuda")
    check(load().lobpcg_update(n, K, N, _dtype_code(S), _ptr(S), S.stride(0), _ptr(Ccm), K,
                               float(alpha), float(beta), _ptr(Y), Y.stride(0), _stream()))
    return Y


def residual(AX, X, theta, BX=None, dinv=None, W=None, normA=1.0, normB=1.0, tol=1e-8):
    """rho (criterion 9), n_c and W = dinv .* R with reversed column order."""
    import torch

    n, nx = X.shape
    ws = load().lobpcg_residual_workspace(n, nx)
    work = torch.empty(max(ws, 8), dtype=torch.uint8, device="cuda")
    rho = torch.empty(nx, dtype=torch.float64, device="cuda")
    nc = torch.zeros(2, dtype=torch.int32, device="cuda")
    check(load().lobpcg_residual(n, nx, _dtype_code(X), _ptr(AX), AX.stride(0),
                                 _ptr(BX) if BX is not None else None,
                                 BX.stride(0) if BX is not None else 0, _ptr(X), X.stride(0),
                                 _ptr(theta), _ptr(dinv) if dinv is not None else None,
                                 _ptr(W) if W is not None else None,
                                 W.stride(0) if W is not None else 0, float(normA), float(normB),
                                 float(tol), _ptr(rho), _ptr(nc), _ptr(work), _stream()))
    return rho, nc


def spmm_residual(rowptr, colind, values, X, theta, W, dinv=None, AX=None, normA=1.0,
                  tol=1e-8):
    """A X fused with the residual for B = I (lobpcg_spmm_residual); W (n x nx view)
    receives the reversed, Jacobi-scaled residual; returns (rho, n_c) device tensors."""
    import torch

    lib = load()
    n, nx = int(X.shape[0]), int(X.shape[1])
    dt = _dtype_code(X)
    work = torch.empty(max(int(lib.lobpcg_spmm_residual_workspace(n, nx)), 8),
                       dtype=torch.uint8, device="cuda")
    rho = torch.empty(max(nx, 1), dtype=torch.float64, device="cuda")
    nc = torch.zeros(2, dtype=torch.int32, device="cuda")
    check(lib.lobpcg_spmm_residual(n, _ptr(rowptr), _ptr(colind), _ptr(values), dt, _ptr(X),
                                   int(X.stride(0)), nx, _ptr(theta),
                                   _ptr(dinv) if dinv is not None else None, _ptr(W),
                                   int(W.stride(0)), _ptr(AX) if AX is not None else None,
                                   int(AX.stride(0)) if AX is not None else 0, float(normA),
                                   float(tol), _ptr(rho), _ptr(nc), _ptr(work), _stream()))
    return rho[:nx], nc


def rr_step(GA, GB, n_x: int, n_c: int, use_ortho: bool, tau_skip: float, literal: bool = False,
            n_ident: int = 0):
    """Algorithm 7 on device FP64 (n_s x n_s) GA, GB; returns a dict.  n_ident: size of a
    leading block of GB that is exactly the identity (blockwise Cholesky)."""
    import torch

    ns = GA.shape[0]
    GAc = GA.to(torch.float64).t().contiguous()
    GBc = GB.to(torch.float64).t().contiguous() if GB is not None else GAc
    Cm = torch.zeros((2 * n_x, ns), dtype=torch.float64, device="cuda")  # column-major ns x 2nx
    theta = torch.zeros(ns, dtype=torch.float64, device="cuda")
    theta_p = torch.zeros((n_x, n_x), dtype=torch.float64, device="cuda")
    np_ = C.c_int32()
    fl = C.c_int32()
    cond = C.c_double()
    check(load().lobpcg_rr_step(ns, n_x, n_c, 1 if use_ortho else 0, 1 if literal else 0,
                                int(n_ident), _ptr(GAc), _ptr(GBc), ns, float(tau_skip), _ptr(Cm), ns,
                                _ptr(theta), _ptr(theta_p), C.byref(np_), C.byref(fl),
                                C.byref(cond), _stream()))
    p = int(np_.value)
    Cfull = Cm.t()  # ns x 2nx
    return {
        "flipped": bool(fl.value),
        "cond": float(cond.value),
        "n_p": p,
        "Cx": Cfull[:, :n_x],
        "Cp": Cfull[:, n_x:n_x + p],
        "theta": theta,
        "theta_p": theta_p.t()[:p, :p],
    }

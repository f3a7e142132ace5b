"""Python binding of librss (ctypes).  Argument marshalling only: every step
of the factorization and the solve runs in the library's HIP kernels; torch is
used for device memory and the current stream.

The library must have been built (``python -m paper_2310_15458_amd.build``);
importing the binding without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librss.so")

RSS_OK, RSS_EINVAL, RSS_ENOMEM, RSS_EUNSUPPORTED, RSS_ESINGULAR, RSS_ENOCONV, RSS_EHIP = 0, -1, -2, -3, -4, -5, -6
RSS_FP64, RSS_FP32_REFINE = 0, 1
KERNEL_CLASSES = ["assemble", "build_C", "id", "sparsify", "inverse", "gemm_y", "compact", "schur",
                  "root"]
_KIND = {"laplace": 0, "helmholtz": 1, "degenerate": 2}


class rss_kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("kappa", ctypes.c_double), ("weight", ctypes.c_double),
                ("diag", ctypes.c_double), ("q", ctypes.c_int), ("cell_diag", ctypes.c_int),
                ("h", ctypes.c_double), ("bump_a", ctypes.c_double), ("bump_c", ctypes.c_double * 2)]


class rss_options(ctypes.Structure):
    _fields_ = [("n_proxy", ctypes.c_int), ("proxy_radius", ctypes.c_double),
                ("precision", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("max_refine", ctypes.c_int), ("root", ctypes.c_double * 3),
                ("stream", ctypes.c_void_p), ("profile", ctypes.c_int), ("colours", ctypes.c_int)]


class rss_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("depth", ctypes.c_int), ("precision", ctypes.c_int),
                ("n_root", ctypes.c_int), ("boxes_compressed", ctypes.c_int64),
                ("rank_sum", ctypes.c_int64 * 16), ("box_count", ctypes.c_int64 * 16),
                ("redundant_sum", ctypes.c_int64 * 16),
                ("flops_id", ctypes.c_double), ("flops_lu", ctypes.c_double),
                ("flops_y", ctypes.c_double), ("flops_schur", ctypes.c_double),
                ("factor_bytes", ctypes.c_double), ("kernel_evals", ctypes.c_double),
                ("t_factor_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("last_relres", ctypes.c_double), ("last_iters", ctypes.c_int),
                ("device_bytes", ctypes.c_double), ("t_class_ms", ctypes.c_double * 12),
                ("n_class", ctypes.c_int64 * 12), ("id_retries", ctypes.c_int)]


EXPORTS = ["rss_factor", "rss_factor_ex", "rss_factor_batch", "rss_solve", "rss_solve_batch", "rss_apply",
           "rss_apply_batch", "rss_free", "rss_info", "rss_skeletons", "rss_kernel_block", "rss_residual",
           "rss_residual_static", "rss_gridop_create", "rss_gridop_apply", "rss_gridop_residual",
           "rss_gridop_free", "rss_set_residual_op", "rss_krylov", "rss_krylov_ex", "rss_factor_tuning",
           "rss_factor_tuning_clear",
           "rss_set_stream", "rss_set_graphs", "rss_trim_cache", "rss_set_autotune", "rss_server_create", "rss_server_factor", "rss_server_solve",
           "rss_server_poll", "rss_server_stats_get", "rss_server_destroy", "rss_last_error",
           "rss_error_string"]


class rss_tune_entry(ctypes.Structure):
    _fields_ = [("precision_bytes", ctypes.c_int), ("box_points_hi", ctypes.c_int), ("boxes_log2", ctypes.c_int),
                ("rows_log2", ctypes.c_int), ("target_workgroups", ctypes.c_int), ("chunks", ctypes.c_int),
                ("us", ctypes.c_float)]


class rss_krylov_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("relres", ctypes.c_double), ("t_ms", ctypes.c_double)]


class rss_server_options(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_double), ("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("leaf", ctypes.c_int), ("n_proxy", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("max_refine", ctypes.c_int), ("max_batch", ctypes.c_int), ("grid_residual", ctypes.c_int)]


class rss_completion(ctypes.Structure):
    _fields_ = [("req", ctypes.c_int64), ("kind", ctypes.c_int), ("status", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_end", ctypes.c_double),
                ("relres", ctypes.c_double), ("iters", ctypes.c_int), ("batch", ctypes.c_int)]


class rss_server_stats(ctypes.Structure):
    _fields_ = [("factored", ctypes.c_int64), ("evictions", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("batched_solves", ctypes.c_int64), ("max_batch_seen", ctypes.c_int64),
                ("resident", ctypes.c_int64), ("pending", ctypes.c_int64), ("used_bytes", ctypes.c_double),
                ("peak_bytes", ctypes.c_double), ("solved_unknowns", ctypes.c_double),
                ("inflight_bytes", ctypes.c_double), ("inflight_peak_bytes", ctypes.c_double),
                ("refactors", ctypes.c_int64)]

_lib = None


class RSSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def load():
    """Load librss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with python -m paper_2310_15458_amd.build")
    # torch ships its own HIP runtime; loading it first makes the library bind to
    # the same runtime (one set of devices, streams and allocations per process)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.rss_factor.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(rss_kernel), ctypes.c_double,
                               ctypes.c_int, P(ctypes.c_void_p)]
    lib.rss_factor_ex.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(rss_kernel), ctypes.c_double,
                                  ctypes.c_int, P(rss_options), P(ctypes.c_void_p)]
    lib.rss_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.rss_apply.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.rss_free.argtypes = [ctypes.c_void_p]
    lib.rss_free.restype = None
    lib.rss_info.argtypes = [ctypes.c_void_p, P(rss_stats)]
    lib.rss_skeletons.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_int32), P(ctypes.c_int64),
                                  ctypes.c_int64, P(ctypes.c_int64)]
    lib.rss_kernel_block.argtypes = [P(rss_kernel), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p]
    lib.rss_residual.argtypes = [P(rss_kernel), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.rss_residual_static.argtypes = [P(rss_kernel), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.rss_gridop_create.argtypes = [P(rss_kernel), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_void_p, P(ctypes.c_void_p)]
    lib.rss_gridop_apply.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.rss_gridop_residual.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int]
    lib.rss_gridop_free.argtypes = [ctypes.c_void_p]
    lib.rss_gridop_free.restype = None
    lib.rss_set_residual_op.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.rss_krylov.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                               ctypes.c_double, ctypes.c_int, P(rss_krylov_stats)]
    lib.rss_factor_tuning.argtypes = [P(rss_tune_entry), ctypes.c_int, P(ctypes.c_int)]
    lib.rss_factor_tuning_clear.argtypes = []
    lib.rss_krylov_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  P(rss_krylov_stats)]
    lib.rss_factor_batch.argtypes = [ctypes.c_int, P(ctypes.c_void_p), P(ctypes.c_int64), P(rss_kernel),
                                     ctypes.c_double, ctypes.c_int, P(rss_options), P(ctypes.c_void_p)]
    lib.rss_apply_batch.argtypes = [ctypes.c_int, P(ctypes.c_void_p), P(ctypes.c_void_p), P(ctypes.c_int)]
    lib.rss_solve_batch.argtypes = [ctypes.c_int, P(ctypes.c_void_p), P(ctypes.c_void_p), P(ctypes.c_int)]
    lib.rss_set_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.rss_set_graphs.argtypes = [ctypes.c_int]
    lib.rss_trim_cache.argtypes = [P(ctypes.c_int64)]
    lib.rss_set_autotune.argtypes = [ctypes.c_int]
    lib.rss_server_create.argtypes = [P(rss_server_options), P(ctypes.c_void_p)]
    lib.rss_server_factor.argtypes = [ctypes.c_void_p, P(ctypes.c_double), ctypes.c_int64, P(rss_kernel),
                                      P(ctypes.c_int64)]
    lib.rss_server_solve.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                     P(ctypes.c_int64)]
    lib.rss_server_poll.argtypes = [ctypes.c_void_p, P(rss_completion), ctypes.c_int, ctypes.c_int,
                                    P(ctypes.c_int)]
    lib.rss_server_stats_get.argtypes = [ctypes.c_void_p, P(rss_server_stats)]
    lib.rss_server_destroy.argtypes = [ctypes.c_void_p]
    lib.rss_last_error.restype = ctypes.c_char_p
    lib.rss_error_string.restype = ctypes.c_char_p
    lib.rss_error_string.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _check(rc):
    if rc != RSS_OK:
        lib = load()
        raise RSSError(rc, f"{lib.rss_error_string(rc).decode()}: {lib.rss_last_error().decode()}")


def make_kernel(kern) -> rss_kernel:
    """From any object with kind/kappa/weight/diag/q and optionally
    cell_diag/h/bump_a/bump_c (e.g. workloads.Kernel)."""
    k = rss_kernel(_KIND[kern.kind], float(kern.kappa), float(kern.weight), float(kern.diag),
                   int(getattr(kern, "q", 2)))
    k.cell_diag = 1 if getattr(kern, "cell_diag", False) else 0
    k.h = float(getattr(kern, "h", 0.0))
    k.bump_a = float(getattr(kern, "bump_a", 0.0))
    c = getattr(kern, "bump_c", (0.5, 0.5))
    k.bump_c[0], k.bump_c[1] = float(c[0]), float(c[1])
    return k


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_options(precision="fp64", n_proxy=0, proxy_radius=0.0, refine_tol=0.0, max_refine=0,
                 root=None, stream=None, profile=False, colours=0) -> rss_options:
    opt = rss_options()
    opt.n_proxy = int(n_proxy)
    opt.proxy_radius = float(proxy_radius)
    opt.precision = RSS_FP32_REFINE if precision in ("fp32", "fp32_refine", RSS_FP32_REFINE) else RSS_FP64
    opt.refine_tol = float(refine_tol)
    opt.max_refine = int(max_refine)
    if root is not None:
        opt.root[0], opt.root[1], opt.root[2] = (float(v) for v in root)
    opt.stream = _stream_ptr(stream).value
    opt.profile = 1 if profile else 0
    opt.colours = int(colours)
    return opt


class Factorization:
    """An RS-S factorization resident on the GPU (rss_factor_ex)."""

    def __init__(self, points, kern, tol: float, leaf: int, precision: str = "fp64",
                 n_proxy: int = 0, proxy_radius: float = 0.0, refine_tol: float = 0.0,
                 max_refine: int = 0, root=None, stream=None, profile: bool = False, colours: int = 0):
        lib = load()
        P = np.ascontiguousarray(points, dtype=np.float64)
        self.N = P.shape[0]
        self.kernel = kern
        self._k = make_kernel(kern)
        opt = make_options(precision, n_proxy, proxy_radius, refine_tol, max_refine, root, stream, profile,
                           colours)
        self._stream = opt.stream
        h = ctypes.c_void_p()
        _check(lib.rss_factor_ex(P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.N,
                                 ctypes.byref(self._k), float(tol), int(leaf), ctypes.byref(opt),
                                 ctypes.byref(h)))
        self._h = h

    @classmethod
    def _wrap(cls, handle, N, kern):
        self = cls.__new__(cls)
        self.N = N
        self.kernel = kern
        self._k = make_kernel(kern)
        self._h = handle
        return self

    def _b(self, B):
        import torch
        if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == torch.complex128):
            raise TypeError("B must be a complex128 CUDA tensor")
        if B.shape[0] != self.N:
            raise ValueError("B must have N rows")
        nrhs = 1 if B.dim() == 1 else B.shape[1]
        if B.dim() == 2 and not B.t().is_contiguous():
            raise ValueError("B must be column-major (use X.t().contiguous().t())")
        return nrhs

    def solve(self, B):
        """Overwrite B (N x nrhs, complex128, column-major CUDA tensor) with A^{-1} B
        (refined in the FP32 form).  Returns the status code (RSS_OK or RSS_ENOCONV)."""
        nrhs = self._b(B)
        rc = load().rss_solve(self._h, ctypes.c_void_p(B.data_ptr()), nrhs)
        if rc not in (RSS_OK, RSS_ENOCONV):
            _check(rc)
        return rc

    def apply(self, B):
        """Overwrite B with one application of the factored inverse (no refinement)."""
        nrhs = self._b(B)
        _check(load().rss_apply(self._h, ctypes.c_void_p(B.data_ptr()), nrhs))

    def info(self) -> dict:
        s = rss_stats()
        _check(load().rss_info(self._h, ctypes.byref(s)))
        out = {f: getattr(s, f) for f, _ in rss_stats._fields_}
        for f in ("rank_sum", "box_count", "redundant_sum", "t_class_ms", "n_class"):
            out[f] = list(out[f])
        return out

    def skeletons(self, depth: int):
        """{box: sorted skeleton ids} for one compressed depth (boxes with points)."""
        lib = load()
        nbox = 4 ** depth
        counts = (ctypes.c_int32 * nbox)()
        total = ctypes.c_int64()
        _check(lib.rss_skeletons(self._h, depth, counts, None, 0, ctypes.byref(total)))
        ids = (ctypes.c_int64 * max(1, total.value))()
        _check(lib.rss_skeletons(self._h, depth, counts, ids, total.value, ctypes.byref(total)))
        out, pos = {}, 0
        arr = np.frombuffer(ids, dtype=np.int64, count=total.value)
        for b in range(nbox):
            c = counts[b]
            if c < 0:
                continue
            out[b] = arr[pos:pos + c].copy()
            pos += c
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().rss_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor_batch(points_list, kernels, tol: float, leaf: int, **opts):
    """Factor several independent problems in one batched sweep
    (rss_factor_batch); returns one Factorization per problem."""
    lib = load()
    arrs = [np.ascontiguousarray(P, dtype=np.float64) for P in points_list]
    n = len(arrs)
    ptrs = (ctypes.c_void_p * n)(*[a.ctypes.data for a in arrs])
    ns = (ctypes.c_int64 * n)(*[a.shape[0] for a in arrs])
    ks = (rss_kernel * n)(*[make_kernel(k) for k in kernels])
    opt = make_options(**opts)
    out = (ctypes.c_void_p * n)()
    _check(lib.rss_factor_batch(n, ptrs, ns, ks, float(tol), int(leaf), ctypes.byref(opt), out))
    return [Factorization._wrap(ctypes.c_void_p(out[i]), arrs[i].shape[0], kernels[i]) for i in range(n)]


def apply_batch(facts, Bs):
    """One application of each factorization to its own right-hand sides
    (complex128 column-major CUDA tensors, overwritten), in one batched sweep."""
    n = len(facts)
    hs = (ctypes.c_void_p * n)(*[f._h.value for f in facts])
    bs = (ctypes.c_void_p * n)(*[B.data_ptr() for B in Bs])
    nr = (ctypes.c_int * n)(*[f._b(B) for f, B in zip(facts, Bs)])
    _check(load().rss_apply_batch(n, hs, bs, nr))


def set_graphs(enable: bool) -> bool:
    """rss_set_graphs: replay captured HIP graphs for single-handle applies
    (default) or launch every apply directly.  Returns the previous setting."""
    return bool(load().rss_set_graphs(1 if enable else 0))


def trim_cache() -> int:
    """rss_trim_cache: return the library's cached device memory (freed
    records and workspaces kept for reuse) on the current device to the
    driver.  Returns the bytes released."""
    out = ctypes.c_int64()
    _check(load().rss_trim_cache(ctypes.byref(out)))
    return int(out.value)


def set_autotune(mode) -> int:
    """rss_set_autotune: 1/True times candidate solve tiles on first use of a
    level shape (default), 0/False keeps the default tiles, 2 takes the fused
    tile wherever it fits.  Returns the previous mode."""
    rc = load().rss_set_autotune(int(mode))
    _check(min(rc, 0))
    return rc


def kernel_block(kern, points_dev, I_dev, J_dev):
    """A[I, J] evaluated on the device (complex128, ni x nj column-major tensor)."""
    import torch
    ni, nj = I_dev.numel(), J_dev.numel()
    out = torch.empty((nj, ni), dtype=torch.complex128, device=points_dev.device).t()
    k = make_kernel(kern)
    _check(load().rss_kernel_block(ctypes.byref(k), ctypes.c_void_p(points_dev.data_ptr()),
                                   points_dev.shape[0], ctypes.c_void_p(I_dev.data_ptr()), ni,
                                   ctypes.c_void_p(J_dev.data_ptr()), nj,
                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(None)))
    return out


def residual(kern, points_dev, X, B):
    """R = B - A X in FP64 with A evaluated on the fly (all complex128, column-major)."""
    import torch
    n = points_dev.shape[0]
    nrhs = 1 if X.dim() == 1 else X.shape[1]
    R = torch.empty((nrhs, n), dtype=torch.complex128, device=X.device).t()
    k = make_kernel(kern)
    _check(load().rss_residual(ctypes.byref(k), ctypes.c_void_p(points_dev.data_ptr()), n,
                               ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                               ctypes.c_void_p(R.data_ptr()), nrhs, _stream_ptr(None)))
    return R


def residual_static(kern, points_dev, X, B):
    """rss_residual_static: R = B - A X like residual(), with no device
    allocation inside the library (its scratch is a static device array)."""
    import torch
    n = points_dev.shape[0]
    nrhs = 1 if X.dim() == 1 else X.shape[1]
    R = torch.empty((nrhs, n), dtype=torch.complex128, device=X.device).t()
    k = make_kernel(kern)
    _check(load().rss_residual_static(ctypes.byref(k), ctypes.c_void_p(points_dev.data_ptr()), n,
                                      ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                      ctypes.c_void_p(R.data_ptr()), nrhs, _stream_ptr(None)))
    return R


class GridOperator:
    """rss_gridop_*: the product with A on the n x n grid of cell centres of
    [x0, x0 + n h] x [y0, y0 + n h] by FFT (the workloads' grids: x0 = y0 = 0,
    h = 1/n)."""

    def __init__(self, kern, n: int, x0: float = 0.0, y0: float = 0.0, h: float = 0.0, stream=None):
        k = make_kernel(kern)
        out = ctypes.c_void_p()
        _check(load().rss_gridop_create(ctypes.byref(k), int(n), float(x0), float(y0),
                                        float(h) if h else 1.0 / n, _stream_ptr(stream), ctypes.byref(out)))
        self._op = out
        self.n = n

    def apply(self, X):
        """A X for a complex128 column-major CUDA tensor X (n^2 x nrhs)."""
        import torch
        nrhs = 1 if X.dim() == 1 else X.shape[1]
        Y = torch.empty((nrhs, X.shape[0]), dtype=torch.complex128, device=X.device).t()
        if X.dim() == 1:
            Y = Y[:, 0]
        _check(load().rss_gridop_apply(self._op, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                       nrhs))
        return Y

    def residual(self, X, B):
        import torch
        nrhs = 1 if X.dim() == 1 else X.shape[1]
        R = torch.empty((nrhs, X.shape[0]), dtype=torch.complex128, device=X.device).t()
        if X.dim() == 1:
            R = R[:, 0]
        _check(load().rss_gridop_residual(self._op, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                          ctypes.c_void_p(R.data_ptr()), nrhs))
        return R

    def close(self):
        if getattr(self, "_op", None):
            load().rss_gridop_free(self._op)
            self._op = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_residual_op(fact, op):
    """rss_set_residual_op: refined solves of `fact` take their residual from
    the grid operator `op` (None: the on-the-fly residual)."""
    _check(load().rss_set_residual_op(fact._h, op._op if op is not None else None))


def krylov(fact, op, B, method: str = "cg", tol: float = 1e-12, maxit: int = 100, restart: int = 0,
           stream=None) -> dict:
    """rss_krylov_ex: CG ("cg") or GMRES ("gmres"; GMRES(restart) when
    restart > 0) preconditioned by the factorization ``fact`` (None: no
    preconditioner), products by the grid operator; B (complex128
    column-major CUDA tensor) is overwritten with the solution."""
    st = rss_krylov_stats()
    nrhs = 1 if B.dim() == 1 else B.shape[1]
    if fact is not None:
        fact._b(B)
    _check(load().rss_krylov_ex(fact._h if fact is not None else None, op._op, ctypes.c_void_p(B.data_ptr()),
                                nrhs, 0 if method == "cg" else 1, float(tol), int(maxit), int(restart),
                                _stream_ptr(stream), ctypes.byref(st)))
    return {"iters": st.iters, "relres": st.relres, "t_ms": st.t_ms}


def factor_tuning() -> list:
    """rss_factor_tuning: the factor-side tuner's table (one dict per bucket)."""
    lib = load()
    cnt = ctypes.c_int()
    _check(lib.rss_factor_tuning(None, 0, ctypes.byref(cnt)))
    buf = (rss_tune_entry * max(1, cnt.value))()
    _check(lib.rss_factor_tuning(buf, cnt.value, ctypes.byref(cnt)))
    return [{f: getattr(buf[i], f) for f, _ in rss_tune_entry._fields_} for i in range(cnt.value)]


def factor_tuning_clear():
    _check(load().rss_factor_tuning_clear())


def solve_batch(facts, Bs):
    """rss_solve_batch: refined (per handle settings) solves of several
    factorizations, every application batched.  Returns the status code."""
    n = len(facts)
    hs = (ctypes.c_void_p * n)(*[f._h.value for f in facts])
    bs = (ctypes.c_void_p * n)(*[B.data_ptr() for B in Bs])
    nr = (ctypes.c_int * n)(*[f._b(B) for f, B in zip(facts, Bs)])
    rc = load().rss_solve_batch(n, hs, bs, nr)
    if rc not in (RSS_OK, RSS_ENOCONV):
        _check(rc)
    return rc


class Server:
    """The library's solve server (rss_server_*): resident factorizations,
    continuous batching of solves, device-memory budget with LRU eviction."""

    def __init__(self, budget_bytes: float, precision: str = "fp32", tol: float = 1e-6, leaf: int = 64,
                 n_proxy: int = 0, refine_tol: float = 0.0, max_refine: int = 0, max_batch: int = 64,
                 grid_residual: bool = False):
        o = rss_server_options(float(budget_bytes),
                               RSS_FP32_REFINE if precision in ("fp32", "fp32_refine") else RSS_FP64,
                               float(tol), int(leaf), int(n_proxy), float(refine_tol), int(max_refine),
                               int(max_batch), 1 if grid_residual else 0)
        h = ctypes.c_void_p()
        _check(load().rss_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._s = h
        self._keep = {}

    def factor(self, points, kern) -> int:
        P = np.ascontiguousarray(points, dtype=np.float64)
        k = make_kernel(kern)
        out = ctypes.c_int64()
        _check(load().rss_server_factor(self._s, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        P.shape[0], ctypes.byref(k), ctypes.byref(out)))
        return out.value

    def solve(self, fid: int, B) -> int:
        """B: complex128 column-major CUDA tensor, overwritten on completion."""
        nrhs = 1 if B.dim() == 1 else B.shape[1]
        out = ctypes.c_int64()
        _check(load().rss_server_solve(self._s, int(fid), ctypes.c_void_p(B.data_ptr()), nrhs,
                                       ctypes.byref(out)))
        self._keep[out.value] = B
        return out.value

    def poll(self, wait_ms: int = 0, cap: int = 256) -> list:
        buf = (rss_completion * cap)()
        cnt = ctypes.c_int()
        _check(load().rss_server_poll(self._s, buf, cap, int(wait_ms), ctypes.byref(cnt)))
        out = []
        for i in range(cnt.value):
            c = buf[i]
            out.append({f: getattr(c, f) for f, _ in rss_completion._fields_})
            self._keep.pop(c.req, None)
        return out

    def stats(self) -> dict:
        st = rss_server_stats()
        _check(load().rss_server_stats_get(self._s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in rss_server_stats._fields_}

    def close(self):
        if getattr(self, "_s", None):
            load().rss_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

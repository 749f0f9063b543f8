"""Python binding of liblrpost.so (ctypes; argument marshalling only).

Every computation runs inside the HIP library.  Device memory and the HIP
stream come from PyTorch: spatial factors are float64 CUDA tensors of shape
(rank, nx) (row c holds column c of the column-major nx x rank factor W1);
temporal factors are float64 NumPy arrays of shape (rank, nt) (row c holds
column c of W2).  If the library is missing or cannot be loaded, importing a
function that needs it raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrpost.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lrpost.h")

LRPOST_FP64, LRPOST_MIXED = 0, 1
LRPOST_MISFIT, LRPOST_PRECOND = 0, 1
LRPOST_BLOCK_LANCZOS, LRPOST_RANDOMIZED = 0, 1
LRPOST_KERNEL_SMOOTHER_STEP, LRPOST_KERNEL_MG_DOWN, LRPOST_KERNEL_MG_UP, LRPOST_KERNEL_GRAM, LRPOST_KERNEL_PROJ = 0, 1, 2, 3, 4
LRPOST_KERNEL_STENCIL = 5
LRPOST_KERNEL_GRAM32 = 6
LRPOST_KERNEL_PROJ32 = 7
LRPOST_KERNEL_SINE, LRPOST_KERNEL_TRIDIAG = 8, 9
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "ENOCONV", -4: "EBREAKDOWN", -5: "EHIP"}


class LrpostError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("lrpost %s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


def convdiff_params(N: int, nt: int, T: float, nu: float, wind: float = 1.0, delta: float = -1.0) -> dict:
    """Host settings of the convection-diffusion operator (no GPU needed)."""
    out = np.zeros(7)
    _check(_lib.lrpost_convdiff_params(int(N), int(nt), float(T), float(nu), float(wind), float(delta), _hptr(out)))
    return {"delta": out[0], "fov_re": out[1], "fov_im": out[2], "ns_alpha": out[3], "ns_radius": out[4],
            "ns_iters": int(out[5]), "lam_min": out[6]}


class Desc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("nt", ctypes.c_int32), ("T", ctypes.c_double), ("alpha", ctypes.c_double),
        ("sigma", ctypes.c_double), ("box", ctypes.c_double * 4), ("trunc_tol", ctypes.c_double),
        ("rank_cap", ctypes.c_int32), ("precision", ctypes.c_int32), ("mg_levels", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("hip_stream", ctypes.c_void_p),
    ]


class LowRankC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nt", ctypes.c_int32), ("rank", ctypes.c_int32), ("cap", ctypes.c_int32),
                ("W1", ctypes.c_void_p), ("W2", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("applies", ctypes.c_int64), ("last_rank_y", ctypes.c_int32), ("last_rank_p", ctypes.c_int32),
                ("last_rank_out", ctypes.c_int32), ("last_basis", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("st_enrichments", ctypes.c_int32), ("st_unresolved", ctypes.c_int32),
                ("st_direct_grams", ctypes.c_int32), ("last_tail", ctypes.c_double), ("last_st_resid", ctypes.c_double),
                ("last_st_presid", ctypes.c_double), ("ritz_resid", ctypes.c_double),
                ("pool_mallocs", ctypes.c_int64), ("pool_trims", ctypes.c_int64), ("pool_malloc_s", ctypes.c_double)]


_lib = None


def header_symbols():
    """Names of the functions declared in include/lrpost.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lrpost_\w+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Load the library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblrpost.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lrpost_create": (I, [ctypes.POINTER(Desc), ctypes.POINTER(P)]),
        "lrpost_destroy": (I, [P]),
        "lrpost_retarget": (I, [P, D, D, pd, ctypes.c_uint64]),
        "lrpost_hess_apply": (I, [P, ctypes.POINTER(LowRankC), ctypes.POINTER(LowRankC), I]),
        "lrpost_hess_apply_batch": (I, [P, I, ctypes.POINTER(LowRankC), ctypes.POINTER(LowRankC), I]),
        "lrpost_spacetime_solve": (I, [P, ctypes.POINTER(LowRankC), ctypes.POINTER(LowRankC), I]),
        "lrpost_eigensolve": (I, [P, I, I, I, ctypes.POINTER(P)]),
        "lrpost_eigensolve_probes": (I, [P, I, I, ctypes.POINTER(LowRankC), ctypes.POINTER(P)]),
        "lrpost_eig_count": (I, [P]),
        "lrpost_eig_values": (I, [P, pd]),
        "lrpost_eig_vector": (I, [P, I, ctypes.POINTER(LowRankC)]),
        "lrpost_eig_vector_rank": (I, [P, I]),
        "lrpost_eigs_free": (I, [P]),
        "lrpost_eigs_from_pairs": (I, [P, I, pd, ctypes.POINTER(LowRankC), ctypes.POINTER(P)]),
        "lrpost_post_variance": (I, [P, P, P, I]),
        "lrpost_prior_variance": (I, [P, pd]),
        "lrpost_sample": (I, [P, P, I, P, P, I]),
        "lrpost_get_stats": (I, [P, ctypes.POINTER(Stats)]),
        "lrpost_stencil_apply": (I, [P, I, P, P, P, pd]),
        "lrpost_mg_solve": (I, [P, I, P, P, pd, I]),
        "lrpost_gram": (I, [P, I, P, I, P, pd]),
        "lrpost_gram_noalloc": (I, [P, I, P, I, P, P]),
        "lrpost_gram_f32": (I, [P, I, P, I, P, pd]),
        "lrpost_set_sweep_precision": (I, [P, I]),
        "lrpost_truncate": (I, [P, ctypes.POINTER(LowRankC), D, I]),
        "lrpost_set_log": (I, [P, I]),
        "lrpost_obs_count": (I, [P]),
        "lrpost_posterior_mean": (I, [P, pd, I, D, ctypes.POINTER(LowRankC), pd]),
        "lrpost_set_eig_limits": (I, [P, I, D]),
        "lrpost_eig_residuals": (I, [P, P, pd]),
        "lrpost_set_st_check": (I, [P, I, D]),
        "lrpost_profile": (I, [P, I]),
        "lrpost_profile_read": (I, [P, I, ctypes.POINTER(ctypes.c_int64), pd, pd, pd]),
        "lrpost_set_mg_fused": (I, [P, I]),
        "lrpost_set_graphs": (I, [P, I]),
        "lrpost_release_cache": (I, [P, ctypes.POINTER(ctypes.c_uint64)]),
        "lrpost_set_obs_mask": (I, [P, ctypes.c_void_p]),
        "lrpost_ic_apply": (I, [P, D, I, P, P]),
        "lrpost_ic_eigensolve": (I, [P, D, I, I, D, pd, P, ctypes.POINTER(ctypes.c_int)]),
        "lrpost_ic_post_variance": (I, [P, D, I, pd, P, P, I]),
        "lrpost_set_convection": (I, [P, D, D, D]),
        "lrpost_convdiff_params": (I, [I, I, D, D, D, D, pd]),
        "lrpost_convdiff_apply": (I, [P, I, P, P, pd, I]),
        "lrpost_convdiff_solve": (I, [P, I, P, P, pd, I]),
        "lrpost_set_apply_batch": (I, [P, I]),
        "lrpost_set_autotune": (I, [I]),
        "lrpost_autotune_report": (I, [ctypes.c_char_p, ctypes.c_size_t]),
        "lrpost_graph_info": (I, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "lrpost_server_create": (I, [ctypes.c_size_t, I, ctypes.POINTER(P)]),
        "lrpost_server_submit": (I, [P, P, I, I, ctypes.POINTER(ctypes.c_uint64)]),
        "lrpost_server_wait": (I, [P, ctypes.c_uint64, pd, I, pd, pd]),
        "lrpost_server_info": (I, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t)]),
        "lrpost_server_destroy": (I, [P]),
        "lrpost_server_class_stats": (I, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "lrpost_measure_fp64_rates": (I, [I, pd]),
        "lrpost_last_error": (ctypes.c_char_p, []),
        "lrpost_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise LrpostError(rc, _lib.lrpost_last_error().decode())


def _torch():
    import torch
    return torch


def _dptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _make_desc(desc, seed: int = 2, mg_levels: int = 0, stream_ptr=None) -> "Desc":
    d = Desc()
    d.N, d.nt, d.T, d.alpha, d.sigma = desc.N, desc.nt, desc.T, desc.alpha, desc.sigma
    for i in range(4):
        d.box[i] = desc.box[i]
    d.trunc_tol, d.rank_cap = desc.trunc_tol, desc.rank_cap
    d.precision = LRPOST_MIXED if getattr(desc, "precision", "fp64") == "mixed" else LRPOST_FP64
    d.mg_levels, d.seed = mg_levels, seed
    d.hip_stream = ctypes.c_void_p(stream_ptr)
    return d


def autotune_report() -> str:
    """The stencil strip-height autotuner's table (one line per shape class)."""
    lib = load()
    n = lib.lrpost_autotune_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib.lrpost_autotune_report(buf, n + 1)
    return buf.value.decode()


def measure_fp64_rates(iters: int = 4000) -> dict:
    """Attainable float64 TFLOP/s of the current device: the matrix-core
    instruction of the float64 kernels and the vector FMA, registers only."""
    out = np.zeros(2)
    _check(load().lrpost_measure_fp64_rates(int(iters), _hptr(out)))
    return {"mfma_f64_16x16x4": float(out[0]), "valu_fma_f64": float(out[1])}


def set_autotune(on: bool):
    """Time the stencil strip heights on each new shape class (default) or use the fixed rule."""
    _check(load().lrpost_set_autotune(1 if on else 0))


class Server:
    """Serving loop: posterior requests run concurrently on `workers` streams,
    admitted against a device-memory budget (lrpost_server_*)."""

    def __init__(self, hbm_budget_bytes: int, workers: int = 4):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.lrpost_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), workers, ctypes.byref(h)))
        self.h = h
        self._sizes = {}

    def submit(self, desc, k: int, want_diag: bool = True, seed: int = 2) -> int:
        d = _make_desc(desc, seed)
        t = ctypes.c_uint64()
        _check(_lib.lrpost_server_submit(self.h, ctypes.byref(d), k, 1 if want_diag else 0, ctypes.byref(t)))
        self._sizes[t.value] = ((desc.N - 1) ** 2, desc.nt, k, want_diag)
        return t.value

    def wait(self, ticket: int):
        """(eigenvalues (k,), variance (nt, nx) or None, latency in s)."""
        nx, nt, k, want = self._sizes.pop(ticket)
        lam = np.zeros(k)
        D = np.zeros((nt, nx)) if want else None
        lat = ctypes.c_double()
        _check(_lib.lrpost_server_wait(self.h, ctypes.c_uint64(ticket), _hptr(lam), k,
                                       D.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want else None,
                                       ctypes.byref(lat)))
        return lam, D, lat.value

    def info(self):
        pr = ctypes.c_int()
        pb = ctypes.c_size_t()
        _check(_lib.lrpost_server_info(self.h, ctypes.byref(pr), ctypes.byref(pb)))
        sv = ctypes.c_int64()
        hit = ctypes.c_int64()
        _check(_lib.lrpost_server_class_stats(self.h, ctypes.byref(sv), ctypes.byref(hit)))
        return {"peak_running": pr.value, "peak_admitted_bytes": pb.value, "served": sv.value,
                "resident_hits": hit.value}

    def close(self):
        if getattr(self, "h", None):
            _lib.lrpost_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A posterior problem on the GPU.  `desc` has the fields of synthetic.ProblemDesc."""

    def __init__(self, desc, seed: int = 2, mg_levels: int = 0, stream=None):
        torch = _torch()
        lib = load()
        # without a stream the library works on a blocking stream of its own,
        # which is ordered after the work queued on torch's (null) default stream
        self.stream = stream
        d = _make_desc(desc, seed, mg_levels, stream.cuda_stream if stream is not None else None)
        self._d = d
        h = ctypes.c_void_p()
        _check(lib.lrpost_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.N, self.nt = desc.N, desc.nt
        self.n = desc.N - 1
        self.nx = self.n * self.n
        self.desc = desc

    def close(self):
        if getattr(self, "h", None):
            _lib.lrpost_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def retarget(self, desc, seed: int = 2):
        """Switch to desc's alpha, sigma and box (same mesh, nt, tolerance, rank cap, precision)."""
        box = np.ascontiguousarray(desc.box, dtype=np.float64)
        _check(_lib.lrpost_retarget(self.h, desc.alpha, desc.sigma, _hptr(box), seed))
        self.desc = desc

    # ---- helpers --------------------------------------------------------
    def _lr_in(self, W1, W2) -> LowRankC:
        torch = _torch()
        r = int(W1.shape[0])
        assert W1.dtype == torch.float64 and W1.is_cuda and W1.is_contiguous() and tuple(W1.shape) == (r, self.nx)
        W2 = np.ascontiguousarray(W2, dtype=np.float64)
        assert W2.shape == (r, self.nt)
        x = LowRankC(self.nx, self.nt, r, r, ctypes.c_void_p(W1.data_ptr()), W2.ctypes.data_as(ctypes.c_void_p))
        x._keep = (W1, W2)
        return x

    def _device_empty(self, shape, like=None):
        """A float64 CUDA tensor; when the device is full, the problem's cached
        blocks are released and the allocation tried once more."""
        torch = _torch()

        def make():
            if like is not None:
                return torch.empty_like(like)
            return torch.empty(shape, dtype=torch.float64, device="cuda")

        try:
            return make()
        except torch.OutOfMemoryError:
            self.release_cache()
            return make()

    def _lr_out(self, cap: int) -> Tuple[LowRankC, object, np.ndarray]:
        cap = max(int(cap), 1)
        W1 = self._device_empty((cap, self.nx))
        W2 = np.zeros((cap, self.nt))
        y = LowRankC(self.nx, self.nt, 0, cap, ctypes.c_void_p(W1.data_ptr()), W2.ctypes.data_as(ctypes.c_void_p))
        return y, W1, W2

    # ---- entry points ---------------------------------------------------
    def hess_apply(self, W1, W2, which: int = LRPOST_PRECOND):
        x = self._lr_in(W1, W2)
        y, Y1, Y2 = self._lr_out(max(self.desc.rank_cap, 1))
        _check(_lib.lrpost_hess_apply(self.h, ctypes.byref(x), ctypes.byref(y), which))
        r = y.rank
        return Y1[:r].clone(), Y2[:r].copy()

    def hess_apply_batch(self, vecs, which: int = LRPOST_PRECOND):
        """Applies to several low-rank vectors [(W1, W2), ...] with fused multigrid solves."""
        n = len(vecs)
        xs = (LowRankC * n)()
        ys = (LowRankC * n)()
        keep = []
        for i, (W1, W2) in enumerate(vecs):
            x = self._lr_in(W1, W2)
            y, Y1, Y2 = self._lr_out(max(self.desc.rank_cap, 1))
            keep.append((x, Y1, Y2))
            xs[i] = x
            ys[i] = y
        _check(_lib.lrpost_hess_apply_batch(self.h, n, xs, ys, which))
        return [(keep[i][1][:ys[i].rank].clone(), keep[i][2][:ys[i].rank].copy()) for i in range(n)]

    def spacetime_solve(self, W1, W2, adjoint: bool = False):
        x = self._lr_in(W1, W2)
        y, Y1, Y2 = self._lr_out(max(self.desc.rank_cap, 1))
        _check(_lib.lrpost_spacetime_solve(self.h, ctypes.byref(x), ctypes.byref(y), 1 if adjoint else 0))
        r = y.rank
        return Y1[:r].clone(), Y2[:r].copy()

    def truncate(self, W1, W2, tol: float = -1.0, weighted: bool = False):
        x = self._lr_in(W1.clone(), W2.copy())
        _check(_lib.lrpost_truncate(self.h, ctypes.byref(x), tol, 1 if weighted else 0))
        r = x.rank
        W1o, W2o = x._keep
        return W1o[:r].clone(), W2o[:r].copy()

    def stencil_apply(self, X, coef, Z=None):
        """Y[c] = (a_c K + b_c M) X[c] + z_c Z[c]; X: (ncols, nx) float64 CUDA; coef: (ncols, 3)."""
        torch = _torch()
        coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1, 3)
        ncols = X.shape[0]
        Y = torch.empty_like(X)
        zp = _dptr(Z) if Z is not None else None
        _check(_lib.lrpost_stencil_apply(self.h, ncols, _dptr(X), _dptr(Y), zp, _hptr(coef)))
        return Y

    def mg_solve(self, B, coef, cycles: int):
        torch = _torch()
        coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1, 2)
        X = torch.empty_like(B)
        _check(_lib.lrpost_mg_solve(self.h, B.shape[0], _dptr(B), _dptr(X), _hptr(coef), cycles))
        return X

    def gram(self, A, B):
        m, q = A.shape[0], B.shape[0]
        C = np.zeros((q, m))  # column-major m x q == row-major q x m
        _check(_lib.lrpost_gram(self.h, m, _dptr(A), q, _dptr(B), _hptr(C)))
        return C.T.copy()

    def gram_f32(self, A32, B):
        """C = A^T B with A (m, nx) float32 CUDA, B (q, nx) float64 CUDA, on the float32 matrix cores."""
        m, q = A32.shape[0], B.shape[0]
        C = np.zeros((q, m))
        _check(_lib.lrpost_gram_f32(self.h, m, _dptr(A32), q, _dptr(B), _hptr(C)))
        return C.T.copy()

    def set_sweep_precision(self, fp32_first: bool):
        """Mixed precision: first Gram-Schmidt sweep of the basis building on float32 matrix cores (default)."""
        _check(_lib.lrpost_set_sweep_precision(self.h, 1 if fp32_first else 0))

    def gram_noalloc(self, A, B, C):
        """C (q, m) float64 CUDA, caller-allocated: C^T = A^T B enqueued on the
        problem's stream with the library's static scratch (no allocation, no sync)."""
        m, q = A.shape[0], B.shape[0]
        assert tuple(C.shape) == (q, m) and C.is_contiguous()
        _check(_lib.lrpost_gram_noalloc(self.h, m, _dptr(A), q, _dptr(B), _dptr(C)))
        return C

    def prior_variance(self):
        out = np.zeros(self.nx)
        _check(_lib.lrpost_prior_variance(self.h, _hptr(out)))
        return out

    def eigensolve(self, k: int, method: int = LRPOST_BLOCK_LANCZOS, oversample: int = 10,
                   allow_unconverged: bool = False) -> "Eigs":
        """k leading eigenpairs.  On LRPOST_ENOCONV the pairs reached are still
        returned (with .converged False) when allow_unconverged, else it raises."""
        e = ctypes.c_void_p()
        rc = _lib.lrpost_eigensolve(self.h, k, method, oversample, ctypes.byref(e))
        return self._eigs_result(rc, e, allow_unconverged)

    def _eigs_result(self, rc, e, allow_unconverged):
        if rc == -3 and e.value:
            out = Eigs(self, e)
            out.converged = False
            out.message = _lib.lrpost_last_error().decode()
            if allow_unconverged:
                return out
            out.close()
        _check(rc)
        return Eigs(self, e)

    def set_eig_limits(self, max_vectors: int = 0, rtol: float = 0.0):
        """Block-Lanczos vector limit and relative Ritz residual target (0: defaults)."""
        _check(_lib.lrpost_set_eig_limits(self.h, int(max_vectors), float(rtol)))

    def set_st_check(self, mode: int = 2, rtol: float = 0.0):
        """Residual check of the space-time solves: 0 off, 1 measure, 2 measure and enrich, 3 strict."""
        _check(_lib.lrpost_set_st_check(self.h, int(mode), float(rtol)))

    def eigensolve_probes(self, k: int, probes, allow_unconverged: bool = False) -> "Eigs":
        """Randomized two-pass eigensolver on caller probes [(W1 (r, nx) CUDA, W2 (r, nt) host), ...]."""
        arr = (LowRankC * len(probes))()
        keep = []
        for i, (W1, W2) in enumerate(probes):
            x = self._lr_in(W1, W2)
            keep.append(x)
            arr[i] = x
        e = ctypes.c_void_p()
        rc = _lib.lrpost_eigensolve_probes(self.h, k, len(probes), arr, ctypes.byref(e))
        return self._eigs_result(rc, e, allow_unconverged)

    def eigs_from_pairs(self, lam, vecs) -> "Eigs":
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        arr = (LowRankC * len(vecs))()
        keep = []
        for i, (W1, W2) in enumerate(vecs):
            x = self._lr_in(W1, W2)
            keep.append(x)
            arr[i] = x
        e = ctypes.c_void_p()
        _check(_lib.lrpost_eigs_from_pairs(self.h, len(vecs), _hptr(lam), arr, ctypes.byref(e)))
        return Eigs(self, e)

    def obs_count(self) -> int:
        return _lib.lrpost_obs_count(self.h)

    # ---- the initial-condition problem --------------------------------
    def set_obs_mask(self, mask):
        """Observed interior nodes from a boolean mask of length nx (node j n + i, x1 fastest)."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=bool).astype(np.uint8))
        assert m.shape == (self.nx,)
        _check(_lib.lrpost_set_obs_mask(self.h, m.ctypes.data_as(ctypes.c_void_p)))

    def set_convection(self, nu: float, wind: float = 1.0, delta: float = -1.0):
        """Spatial operator -nu Laplace + (0, wind) . grad (SUPG; delta < 0: Peclet rule) for the
        space-time solves and the initial-condition problem; nu <= 0: back to the heat operator."""
        _check(_lib.lrpost_set_convection(self.h, float(nu), float(wind), float(delta)))

    def _cd_call(self, fn, X, coef, transpose):
        torch = _torch()
        assert X.dtype == torch.float64 and X.is_cuda and X.dim() == 2 and X.shape[1] == self.nx
        X = X.contiguous()
        c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(-1))
        assert c.size == 2 * X.shape[0]
        Y = self._device_empty(None, like=X)
        _check(fn(self.h, int(X.shape[0]), _dptr(X), _dptr(Y), _hptr(c), int(bool(transpose))))
        return Y

    def convdiff_apply(self, X, coef, transpose: bool = False):
        """(a_j L + b_j M) X_j (L^T with transpose) for CUDA float64 X (ncols, nx); coef (ncols, 2)."""
        return self._cd_call(_lib.lrpost_convdiff_apply, X, coef, transpose)

    def convdiff_solve(self, B, coef, transpose: bool = False):
        """(a_j L + b_j M)^{-1} B_j (exact; L^T with transpose) for CUDA float64 B (ncols, nx)."""
        return self._cd_call(_lib.lrpost_convdiff_solve, B, coef, transpose)

    def ic_apply(self, U, prior_var: float):
        """G U for initial states U: CUDA float64 (nvec, nx) -> (nvec, nx)."""
        torch = _torch()
        assert U.dtype == torch.float64 and U.is_cuda and U.dim() == 2 and U.shape[1] == self.nx
        U = U.contiguous()
        Y = self._device_empty(None, like=U)
        _check(_lib.lrpost_ic_apply(self.h, float(prior_var), int(U.shape[0]), _dptr(U), _dptr(Y)))
        return Y

    def ic_eigensolve(self, k: int, prior_var: float, max_vectors: int = 0, rtol: float = 0.0,
                      allow_unconverged: bool = False):
        """k leading eigenpairs of G: (values (k,) descending, vectors CUDA (k, nx), basis size)."""
        vals = np.zeros(int(k))
        V = self._device_empty((int(k), self.nx))
        used = ctypes.c_int()
        rc = _lib.lrpost_ic_eigensolve(self.h, float(prior_var), int(k), int(max_vectors), float(rtol), _hptr(vals),
                                       _dptr(V), ctypes.byref(used))
        if not (rc == -3 and allow_unconverged):
            _check(rc)
        return vals, V, used.value

    def ic_post_variance(self, values, vectors, prior_var: float, on_device: bool = True):
        """diag(prior_var (I + G)^{-1}) from eigenpairs (values (k,), vectors CUDA (k, nx))."""
        vals = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
        k = int(vals.size)
        vectors = vectors.contiguous()
        assert tuple(vectors.shape) == (k, self.nx)
        if on_device:
            out = self._device_empty((self.nx,))
            _check(_lib.lrpost_ic_post_variance(self.h, float(prior_var), k, _hptr(vals), _dptr(vectors), _dptr(out), 1))
            return out
        out = np.zeros(self.nx)
        _check(_lib.lrpost_ic_post_variance(self.h, float(prior_var), k, _hptr(vals), _dptr(vectors),
                                            out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def posterior_mean(self, y_obs, max_vectors: int = 0, rtol: float = 0.0, allow_unconverged: bool = False):
        """Posterior mean for observations y_obs (nobs, nt): (W1 (r, nx) CUDA, W2 (r, nt), residual estimate)."""
        y = np.asfortranarray(np.asarray(y_obs, dtype=np.float64))
        assert y.shape == (self.obs_count(), self.nt)
        out, W1, W2 = self._lr_out(max(self.desc.rank_cap, 1))
        res = ctypes.c_double()
        rc = _lib.lrpost_posterior_mean(self.h, _hptr(y), int(max_vectors), float(rtol), ctypes.byref(out),
                                        ctypes.byref(res))
        if not (rc == -3 and allow_unconverged):
            _check(rc)
        r = out.rank
        return W1[:r].clone(), W2[:r].copy(), res.value

    def post_variance(self, eigs: "Eigs", on_device: bool = True):
        """diag(Gamma_post,k) as an (nt, nx) array (row t = time step t)."""
        torch = _torch()
        if on_device:
            D = self._device_empty((self.nt, self.nx))
            _check(_lib.lrpost_post_variance(self.h, eigs.h, _dptr(D), 1))
            return D
        D = np.zeros((self.nt, self.nx))
        _check(_lib.lrpost_post_variance(self.h, eigs.h, D.ctypes.data_as(ctypes.c_void_p), 0))
        return D

    def sample(self, eigs: "Eigs", xi):
        """Posterior samples for standard normal draws xi of shape (ns, nt, nx)
        (row t of sample s = time step t).  A CUDA float64 tensor stays on the
        device; a NumPy array goes through host memory.  Same shape returned."""
        torch = _torch()
        if torch is not None and isinstance(xi, torch.Tensor):
            if xi.device.type != "cuda" or xi.dtype != torch.float64 or xi.dim() != 3:
                raise ValueError("xi must be a CUDA float64 tensor (ns, nt, nx)")
            xi = xi.contiguous()
            out = self._device_empty(None, like=xi)
            _check(_lib.lrpost_sample(self.h, eigs.h, xi.shape[0], _dptr(xi), _dptr(out), 1))
            return out
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        if xi.ndim != 3:
            raise ValueError("xi must have shape (ns, nt, nx)")
        out = np.zeros_like(xi)
        _check(_lib.lrpost_sample(self.h, eigs.h, xi.shape[0], xi.ctypes.data_as(ctypes.c_void_p),
                                  out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def set_log(self, level: int):
        """Progress lines (JSON on stderr) from the eigensolvers when level > 0."""
        _check(_lib.lrpost_set_log(self.h, level))

    def profile(self, enable: bool):
        """Turn event timing of the multigrid kernels on or off."""
        _check(_lib.lrpost_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel: int = None):
        """(launches, kernel ms, algorithmic bytes, flops) of one kernel kind
        (LRPOST_KERNEL_*; default the level-fused up kernel) since the last read."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        fl = ctypes.c_double()
        k = LRPOST_KERNEL_MG_UP if kernel is None else kernel
        _check(_lib.lrpost_profile_read(self.h, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                        ctypes.byref(fl)))
        return n.value, ms.value, by.value, fl.value

    def set_mg_fused(self, on: bool):
        """Level-fused multigrid kernels (default) or one kernel per step."""
        _check(_lib.lrpost_set_mg_fused(self.h, 1 if on else 0))

    def set_apply_batch(self, n: int):
        """Probe applies per batched pass of the randomized eigensolver (0: as many as fit)."""
        _check(_lib.lrpost_set_apply_batch(self.h, int(n)))

    def set_graphs(self, on: bool):
        """V-cycles replayed from captured HIP graphs (default) or launched kernel by kernel."""
        _check(_lib.lrpost_set_graphs(self.h, 1 if on else 0))

    def release_cache(self) -> int:
        """Return the problem's cached device blocks to the device; bytes released."""
        b = ctypes.c_uint64()
        _check(_lib.lrpost_release_cache(self.h, ctypes.byref(b)))
        return b.value

    def graph_info(self):
        """(graphs captured, graph launches) since creation."""
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        _check(_lib.lrpost_graph_info(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.lrpost_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}


class Eigs:
    def __init__(self, prob: Problem, h):
        self.prob = prob
        self.h = h
        self.converged = True
        self.message = ""

    def residuals(self) -> np.ndarray:
        """Measured ||G v - lambda v||_P / |lambda| of every stored pair (one apply each)."""
        out = np.zeros(len(self))
        _check(_lib.lrpost_eig_residuals(self.prob.h, self.h, _hptr(out)))
        return out

    def __len__(self):
        return _lib.lrpost_eig_count(self.h)

    def values(self) -> np.ndarray:
        k = len(self)
        out = np.zeros(k)
        _check(_lib.lrpost_eig_values(self.h, _hptr(out)))
        return out

    def vector(self, i: int):
        r = _lib.lrpost_eig_vector_rank(self.h, i)
        y, W1, W2 = self.prob._lr_out(max(r, 1))
        _check(_lib.lrpost_eig_vector(self.h, i, ctypes.byref(y)))
        return W1[:y.rank].clone(), W2[:y.rank].copy()

    def close(self):
        if getattr(self, "h", None):
            _lib.lrpost_eigs_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

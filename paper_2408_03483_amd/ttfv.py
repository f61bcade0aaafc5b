"""Python binding of libttfv.so (include/tt_fv.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm).  A core of n rows and capacity `cap`
is a contiguous torch tensor of shape (cap, n): column a of the column-major n x cap core
is row a of the tensor.  Every computation runs in the HIP library; if the library cannot
be loaded, or no GPU is present, the calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttfv.so")

TT_FN_IDENTITY = 0
TT_FN_LLF_LAMBDA = 1
TT_FN_WENO_FACE_M = 2
TT_FN_WENO_FACE_P = 3
TT_FN_WENO_QUAD = 4
TT_FN_RECIP = 5

TT_WRANKCAP = 1
TT_WNOCONV = 2
TT_WSKETCH = 4
TT_WJACOBI = 8
TT_EDOMAIN = -5
TT_ENONFINITE = -4


class TTMatrixC(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n2", ctypes.c_int), ("rank", ctypes.c_int),
                ("cap", ctypes.c_int), ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p)]


class ParamsC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nonlinear", ctypes.c_int), ("scheme", ctypes.c_int),
                ("periodic", ctypes.c_int), ("g", ctypes.c_double), ("H0", ctypes.c_double),
                ("f", ctypes.c_double), ("eps", ctypes.c_double), ("r_max", ctypes.c_int),
                ("taylor_terms", ctypes.c_int), ("cross_sweeps", ctypes.c_int),
                ("cross_kick", ctypes.c_int), ("recip", ctypes.c_int), ("workers", ctypes.c_int),
                ("precision", ctypes.c_int), ("qr", ctypes.c_int), ("cross_drop", ctypes.c_double),
                ("eps_rule", ctypes.c_int), ("c_eps", ctypes.c_double),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("t0", ctypes.c_double),
                ("flux", ctypes.c_int), ("cross_enrich", ctypes.c_int),
                ("graph", ctypes.c_int), ("graph_iters", ctypes.c_int)]


class TensorC(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.POINTER(ctypes.c_int)),
                ("r", ctypes.POINTER(ctypes.c_int)),
                ("cores", ctypes.POINTER(ctypes.c_void_p))]


class TermC(ctypes.Structure):
    _fields_ = [("var", ctypes.c_int), ("where", ctypes.c_int), ("amp", ctypes.c_double),
                ("omega", ctypes.c_double), ("phase", ctypes.c_double),
                ("X", ctypes.POINTER(ctypes.c_double)), ("Y", ctypes.POINTER(ctypes.c_double))]


class StatsC(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_longlong), ("ranks", ctypes.c_int * 3),
                ("roundings", ctypes.c_longlong), ("crosses", ctypes.c_longlong),
                ("last_taylor_terms", ctypes.c_int), ("last_taylor_err", ctypes.c_double),
                ("warnings", ctypes.c_int), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double), ("timed_ms", ctypes.c_double),
                ("timed_launches", ctypes.c_longlong), ("timed_flops", ctypes.c_double),
                ("timed_bytes", ctypes.c_double), ("cross_sweeps_run", ctypes.c_longlong),
                ("learned_crosses", ctypes.c_longlong), ("learned_fallbacks", ctypes.c_longlong),
                ("max_learned_err", ctypes.c_double), ("sketch_fallbacks", ctypes.c_longlong),
                ("sketch_unconverged", ctypes.c_longlong), ("jacobi_capped", ctypes.c_longlong),
                ("qr_redos", ctypes.c_longlong), ("eps_inner", ctypes.c_double),
                ("eps_var", ctypes.c_double * 3), ("time", ctypes.c_double),
                ("graph_launches", ctypes.c_longlong)]


PRECISIONS = {"f64": 0, "f32": 1}
QR_METHODS = {"auto": 0, "cholesky": 1, "householder": 2}
EPS_RULES = {"fixed": 0, "paper": 1}
FLUXES = {"products": 0, "lf_cross": 1}
ENRICH = {"kicks": 0, "residual": 1}
BCS = {None: 0, "periodic": 1, "wall": 2, "exact": 3}
TERM_WHERE = {"forcing": 0, "x_lo": 1, "x_hi": 2, "y_lo": 3, "y_hi": 4}


def _terms_c(terms):
    """ctypes array of tt_fv_term from objects with var, where, amp, omega, phase, X, Y; the
    returned list keeps the factor arrays alive for the call."""
    import numpy as np
    keep, arr = [], (TermC * max(len(terms), 1))()
    for k, t in enumerate(terms):
        X = np.ascontiguousarray(t.X, dtype=np.float64)
        Y = np.ascontiguousarray(t.Y, dtype=np.float64)
        keep += [X, Y]
        arr[k] = TermC(int(t.var), TERM_WHERE[t.where], float(t.amp), float(t.omega),
                       float(t.phase), X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       Y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return arr, keep

EXPORTS = ["tt_ctx_create", "tt_ctx_destroy", "tt_ctx_set_sketch", "tt_ctx_set_precision",
           "tt_round", "tt_round_noalloc",
           "tt_hadamard_round", "tt_reciprocal", "tt_maxvol", "tt_cross", "tt_recon_core",
           "tt_fv_init", "tt_fv_step", "tt_fv_get_state", "tt_fv_get_stats", "tt_fv_destroy",
           "tt_fv_time_kernel", "tt_ens_create", "tt_ens_step", "tt_ens_destroy",
           "tt_pm_create", "tt_pm_destroy", "tt_pm_set_weights", "tt_pm_get_weights",
           "tt_pm_forward", "tt_pm_grad", "tt_pm_train", "tt_pm_dataset", "tt_pm_features",
           "tt_pm_topk", "tt_fv_set_pivots", "tt_gemm_autotune", "tt_last_error",
           "tt_fv_replay_pivots", "tt_fv_get_pivots", "tt_cross_skeleton", "tt_pm_adam",
           "tt_ctx_set_limits", "tt_ctx_set_qr", "tt_fv_set_pivot_acceptance",
           "tt_grid_init", "tt_grid_step", "tt_grid_destroy", "tt_grid_set_terms",
           "tt_fv_set_terms", "tt_compress", "tt_fv_max_speed", "tt_fv_cfl_dt",
           "tt_ctx_set_enrichment", "tt_round_nd", "tt_ctx_set_fixed", "tt_rule_trunc_rank",
           "tt_rule_kicks"]

PM_NPARAM = 70401
PIVOTS = {"maxvol": 0, "log": 1, "learned": 2, "replay": 3, "kicks": 4}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libttfv.so and declare its signatures (no GPU needed for this step)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libttfv.so not built ({path}); run paper_2408_03483_amd.build")
    L = ctypes.CDLL(path)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    pM = ctypes.POINTER(TTMatrixC)
    L.tt_last_error.restype = ctypes.c_char_p
    L.tt_ctx_create.argtypes = [ctypes.POINTER(P), S, P]
    L.tt_ctx_destroy.argtypes = [P]
    L.tt_ctx_destroy.restype = None
    L.tt_ctx_set_sketch.argtypes = [P, I, I]
    L.tt_ctx_set_precision.argtypes = [P, I]
    L.tt_ctx_set_limits.argtypes = [P, I, I]
    L.tt_ctx_set_qr.argtypes = [P, I, I]
    L.tt_ctx_set_enrichment.argtypes = [P, I]
    L.tt_ctx_set_fixed.argtypes = [P, I]
    L.tt_rule_trunc_rank.argtypes = [ctypes.POINTER(ctypes.c_double), I, ctypes.c_double, I,
                                     ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    L.tt_rule_kicks.argtypes = [ctypes.POINTER(ctypes.c_int), I, I, I, ctypes.c_uint64,
                                ctypes.POINTER(ctypes.c_int)]
    L.tt_round.argtypes = [P, pM, D, I, pM, ctypes.POINTER(D)]
    L.tt_round_noalloc.argtypes = [pM, D, I, pM, ctypes.POINTER(D), P]
    L.tt_compress.argtypes = [P, P, I, I, I, D, I, pM, ctypes.POINTER(D)]
    L.tt_fv_max_speed.argtypes = [P, ctypes.POINTER(D)]
    L.tt_round_nd.argtypes = [P, ctypes.POINTER(TensorC), D, I, ctypes.POINTER(TensorC),
                              ctypes.POINTER(D)]
    L.tt_fv_cfl_dt.argtypes = [P, D, ctypes.POINTER(D)]
    L.tt_hadamard_round.argtypes = [P, pM, pM, D, I, pM]
    L.tt_reciprocal.argtypes = [P, pM, D, I, I, pM, ctypes.POINTER(D), ctypes.POINTER(I)]
    L.tt_maxvol.argtypes = [P, P, I, I, I, D, I, ctypes.POINTER(I)]
    L.tt_cross.argtypes = [P, I, pM, I, ctypes.POINTER(D), I, I, ctypes.POINTER(I), I, D, I, I,
                           I, ctypes.c_uint64, pM, ctypes.POINTER(I), ctypes.POINTER(I)]
    L.tt_recon_core.argtypes = [P, P, I, I, I, I, D, P, P, P]
    L.tt_fv_init.argtypes = [ctypes.POINTER(P), ctypes.POINTER(ParamsC), pM, P, S]
    L.tt_fv_step.argtypes = [P, D, I]
    L.tt_fv_get_state.argtypes = [P, pM]
    L.tt_fv_get_stats.argtypes = [P, ctypes.POINTER(StatsC)]
    L.tt_fv_time_kernel.argtypes = [P, ctypes.c_char_p, I]
    L.tt_fv_destroy.argtypes = [P]
    L.tt_fv_destroy.restype = None
    L.tt_grid_init.argtypes = [ctypes.POINTER(P), ctypes.POINTER(ParamsC), P]
    L.tt_grid_step.argtypes = [P, P, D, I]
    L.tt_grid_destroy.argtypes = [P]
    L.tt_grid_destroy.restype = None
    L.tt_grid_set_terms.argtypes = [P, ctypes.POINTER(TermC), I]
    L.tt_fv_set_terms.argtypes = [P, ctypes.POINTER(TermC), I]
    L.tt_ens_create.argtypes = [ctypes.POINTER(P), I, S]
    L.tt_ens_step.argtypes = [P, ctypes.POINTER(P), I, ctypes.POINTER(D), I, I]
    L.tt_ens_destroy.argtypes = [P]
    L.tt_ens_destroy.restype = None
    pF = ctypes.POINTER(ctypes.c_float)
    L.tt_pm_create.argtypes = [ctypes.POINTER(P), S, ctypes.c_ulonglong]
    L.tt_pm_destroy.argtypes = [P]
    L.tt_pm_destroy.restype = None
    L.tt_pm_set_weights.argtypes = [P, pF, S]
    L.tt_pm_get_weights.argtypes = [P, pF, S]
    L.tt_pm_forward.argtypes = [P, P, I, P]
    L.tt_pm_grad.argtypes = [P, P, P, I, D, pF, S, ctypes.POINTER(D)]
    L.tt_pm_train.argtypes = [P, I, I, D, ctypes.POINTER(D)]
    L.tt_pm_adam.argtypes = [P, pF, S, D]
    L.tt_pm_dataset.argtypes = [P, ctypes.POINTER(S), ctypes.POINTER(S)]
    L.tt_pm_features.argtypes = [P, P, I, I, I, P, I, P]
    L.tt_pm_topk.argtypes = [P, P, I, I, P]
    L.tt_fv_set_pivots.argtypes = [P, I, P]
    L.tt_fv_set_pivot_acceptance.argtypes = [P, D, D]
    L.tt_gemm_autotune.argtypes = [I, ctypes.POINTER(I)]
    pI = ctypes.POINTER(I)
    L.tt_fv_replay_pivots.argtypes = [P, ctypes.c_longlong, I, pI, I, pI, I]
    L.tt_fv_get_pivots.argtypes = [P, I, pI, I, pI, pI, I, pI]
    L.tt_cross_skeleton.argtypes = [P, I, pM, I, ctypes.POINTER(D), I, I, pI, I, pI, I, D, I, pM]
    for name in EXPORTS:
        if not hasattr(L, name):
            raise RuntimeError(f"libttfv.so lacks {name}")
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the TT-FV library runs on the GPU only")
    return torch


def _check(code: int, what: str) -> int:
    if code < 0:
        msg = _lib.tt_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed ({code}): {msg}")
    return code


class DeviceTT:
    """Two device cores: g1 (cap, n1), g2 (cap, n2) float64 tensors (column-major cores)."""

    def __init__(self, n1: int, n2: int, cap: int, device="cuda"):
        torch = _torch()
        self.n1, self.n2, self.cap, self.rank = n1, n2, cap, 0
        self.g1 = torch.zeros((cap, n1), dtype=torch.float64, device=device)
        self.g2 = torch.zeros((cap, n2), dtype=torch.float64, device=device)

    @classmethod
    def from_factors(cls, A: np.ndarray, B: np.ndarray, cap: Optional[int] = None,
                     device="cuda") -> "DeviceTT":
        torch = _torch()
        r = A.shape[1]
        t = cls(A.shape[0], B.shape[0], max(cap or r, r), device)
        t.g1[:r] = torch.from_numpy(np.ascontiguousarray(A.T)).to(device)
        t.g2[:r] = torch.from_numpy(np.ascontiguousarray(B.T)).to(device)
        t.rank = r
        return t

    def c(self) -> TTMatrixC:
        return TTMatrixC(self.n1, self.n2, self.rank, self.cap, self.g1.data_ptr(),
                         self.g2.data_ptr())

    def factors(self):
        A = self.g1[:self.rank].T.cpu().numpy().copy()
        B = self.g2[:self.rank].T.cpu().numpy().copy()
        return A, B

    def full(self) -> np.ndarray:
        A, B = self.factors()
        return A @ B.T


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Ctx:
    def __init__(self, arena_bytes: int = 1 << 30, stream=None):
        L = load_library()
        _torch()
        self._stream = stream
        self.h = ctypes.c_void_p()
        _check(L.tt_ctx_create(ctypes.byref(self.h), arena_bytes, _stream_ptr(stream)),
               "tt_ctx_create")

    def close(self):
        if self.h:
            _lib.tt_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tt_ctx_create(arena_bytes: int = 1 << 30, stream=None) -> Ctx:
    return Ctx(arena_bytes, stream)


def tt_ctx_set_sketch(ctx: Ctx, width: int, power_iters: int) -> None:
    _check(_lib.tt_ctx_set_sketch(ctx.h, width, power_iters), "tt_ctx_set_sketch")


def tt_ctx_set_qr(ctx: Ctx, method: str, max_passes: int = 6) -> None:
    _check(_lib.tt_ctx_set_qr(ctx.h, QR_METHODS[method], max_passes), "tt_ctx_set_qr")


def tt_ctx_set_enrichment(ctx: Ctx, mode: str) -> None:
    _check(_lib.tt_ctx_set_enrichment(ctx.h, ENRICH[mode]), "tt_ctx_set_enrichment")


def tt_rule_trunc_rank(s, eps: float, r_max: int, floor_rel: float = 0.0):
    """The library's kept-rank rule on host singular values (no GPU): (rank, capped)."""
    L = load_library()
    import numpy as np
    a = np.ascontiguousarray(s, dtype=np.float64)
    cap = ctypes.c_int()
    k = _check(L.tt_rule_trunc_rank(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size,
                                    eps, r_max, floor_rel, ctypes.byref(cap)),
               "tt_rule_trunc_rank")
    return k, bool(cap.value)


def tt_rule_kicks(have, n: int, count: int, key: int):
    """The library's seeded fresh cross columns (no GPU)."""
    L = load_library()
    h = (ctypes.c_int * max(len(have), 1))(*[int(v) for v in have])
    out = (ctypes.c_int * max(count, 1))()
    m = _check(L.tt_rule_kicks(h, len(have), n, count, ctypes.c_uint64(key & 0xFFFFFFFFFFFFFFFF),
                               out), "tt_rule_kicks")
    return [out[i] for i in range(m)]


def tt_ctx_set_fixed(ctx: Ctx, on: bool) -> None:
    """Fixed shapes (device-side ranks) for this context's tt_round and tt_cross."""
    _check(_lib.tt_ctx_set_fixed(ctx.h, 1 if on else 0), "tt_ctx_set_fixed")


def tt_ctx_set_limits(ctx: Ctx, jacobi_max_sweeps: int, sketch_max_iters: int) -> None:
    _check(_lib.tt_ctx_set_limits(ctx.h, jacobi_max_sweeps, sketch_max_iters),
           "tt_ctx_set_limits")


def tt_ctx_set_precision(ctx: Ctx, precision: str) -> None:
    _check(_lib.tt_ctx_set_precision(ctx.h, PRECISIONS[precision]), "tt_ctx_set_precision")


def tt_round(ctx: Ctx, x: DeviceTT, eps: float, r_max: int, y: DeviceTT):
    xc, yc = x.c(), y.c()
    sig = (ctypes.c_double * max(r_max, 1))()
    w = _check(_lib.tt_round(ctx.h, ctypes.byref(xc), eps, r_max, ctypes.byref(yc), sig),
               "tt_round")
    y.rank = yc.rank
    return w, np.array(sig[:y.rank])


class DeviceTTnd:
    """d cores on the device, core k a float64 tensor with room for cap_k = (r_in or r_max)^2
    n_k entries; the data of core k is its first r[k] n[k] r[k+1] entries, left rank index
    fastest (G(a, i, b) at a + r[k] (i + n[k] b))."""

    def __init__(self, modes, ranks, room, device="cuda"):
        torch = _torch()
        self.n, self.r = list(modes), list(ranks)
        self.cores = [torch.zeros(max(int(rm), 1), dtype=torch.float64, device=device)
                      for rm in room]

    @classmethod
    def from_cores(cls, cores, device="cuda"):
        torch = _torch()
        modes = [c.shape[1] for c in cores]
        ranks = [cores[0].shape[0]] + [c.shape[2] for c in cores]
        t = cls(modes, ranks, [c.size for c in cores], device)
        for k, c in enumerate(cores):
            t.cores[k][:c.size] = torch.from_numpy(
                np.ascontiguousarray(np.transpose(c, (2, 1, 0))).reshape(-1)).to(device)
        return t

    def to_cores(self):
        out = []
        for k, n in enumerate(self.n):
            r0, r1 = self.r[k], self.r[k + 1]
            flat = self.cores[k][:r0 * n * r1].cpu().numpy()
            out.append(np.transpose(flat.reshape(r1, n, r0), (2, 1, 0)).copy())
        return out

    def c(self):
        d = len(self.n)
        self._n = (ctypes.c_int * d)(*self.n)
        self._r = (ctypes.c_int * (d + 1))(*self.r)
        self._p = (ctypes.c_void_p * d)(*[t.data_ptr() for t in self.cores])
        return TensorC(d, self._n, self._r, self._p)


def tt_round_nd(ctx: Ctx, x: DeviceTTnd, eps: float, r_max: int):
    """Rounding of a d-core TT; returns (output DeviceTTnd, warnings, bond singular values)."""
    d = len(x.n)
    y = DeviceTTnd(x.n, [1] * (d + 1), [r_max * n * r_max for n in x.n])
    xc, yc = x.c(), y.c()
    sig = (ctypes.c_double * ((d - 1) * r_max))()
    w = _check(_lib.tt_round_nd(ctx.h, ctypes.byref(xc), eps, r_max, ctypes.byref(yc), sig),
               "tt_round_nd")
    y.r = [int(yc.r[k]) for k in range(d + 1)]
    kept = sum(y.r[1:d])
    return y, w, np.array(sig[:kept])


def tt_compress(ctx: Ctx, F, eps: float, r_max: int):
    """TT of a full field F (torch float64 CUDA tensor, n1 x n2, row-major, F[i, j] with i the
    first TT index): the library compresses the column-major matrix F^T that this memory is,
    and the cores are swapped back.  Returns (DeviceTT with rank <= r_max, warnings, sigma)."""
    if (F.dim() != 2 or not F.is_cuda or str(F.dtype) != "torch.float64" or
            not F.is_contiguous()):
        raise ValueError("tt_compress: F must be a contiguous 2-D float64 CUDA tensor")
    n1, n2 = int(F.shape[0]), int(F.shape[1])
    yt = DeviceTT(n2, n1, r_max)
    yc = yt.c()
    sig = (ctypes.c_double * max(r_max, 1))()
    w = _check(_lib.tt_compress(ctx.h, ctypes.c_void_p(F.data_ptr()), n2, n1, n2, eps, r_max,
                                ctypes.byref(yc), sig), "tt_compress")
    y = DeviceTT.__new__(DeviceTT)
    y.n1, y.n2, y.cap, y.rank = n1, n2, r_max, yc.rank
    y.g1, y.g2 = yt.g2, yt.g1
    return y, w, np.array(sig[:y.rank])


def tt_round_noalloc(x: DeviceTT, eps: float, r_max: int, y: DeviceTT, stream=None):
    """tt_round without a context: temporaries in the library's fixed per-GPU scratch array."""
    L = load_library()
    xc, yc = x.c(), y.c()
    sig = (ctypes.c_double * max(r_max, 1))()
    w = _check(L.tt_round_noalloc(ctypes.byref(xc), eps, r_max, ctypes.byref(yc), sig,
                                  _stream_ptr(stream)), "tt_round_noalloc")
    y.rank = yc.rank
    return w, np.array(sig[:y.rank])


def tt_hadamard_round(ctx: Ctx, x: DeviceTT, z: DeviceTT, eps: float, r_max: int,
                      y: DeviceTT) -> int:
    xc, zc, yc = x.c(), z.c(), y.c()
    w = _check(_lib.tt_hadamard_round(ctx.h, ctypes.byref(xc), ctypes.byref(zc), eps, r_max,
                                      ctypes.byref(yc)), "tt_hadamard_round")
    y.rank = yc.rank
    return w


def tt_reciprocal(ctx: Ctx, x: DeviceTT, eps: float, max_terms: int, r_max: int, y: DeviceTT):
    xc, yc = x.c(), y.c()
    err = ctypes.c_double()
    terms = ctypes.c_int()
    w = _check(_lib.tt_reciprocal(ctx.h, ctypes.byref(xc), eps, max_terms, r_max,
                                  ctypes.byref(yc), ctypes.byref(err), ctypes.byref(terms)),
               "tt_reciprocal")
    y.rank = yc.rank
    return w, err.value, terms.value


def tt_maxvol(ctx: Ctx, q, tau: float = 1.05, maxit: int = 100) -> np.ndarray:
    """q: torch float64 (r, n) tensor = column-major n x r basis."""
    r, n = q.shape
    rows = (ctypes.c_int * r)()
    _check(_lib.tt_maxvol(ctx.h, ctypes.c_void_p(q.data_ptr()), n, r, n, tau, maxit, rows),
           "tt_maxvol")
    return np.array(rows[:], dtype=np.int64)


def tt_cross(ctx: Ctx, fn: int, inputs: Sequence[DeviceTT], fparams: Sequence[float], n1: int,
             n2: int, J0: Sequence[int], eps: float, r_max: int, sweeps: int, kick: int,
             key: int, y: DeviceTT):
    arr = (TTMatrixC * len(inputs))(*[t.c() for t in inputs])
    fp = (ctypes.c_double * max(1, len(fparams)))(*fparams)
    J = (ctypes.c_int * len(J0))(*[int(j) for j in J0])
    jcap = len(J0) + r_max + kick * sweeps + 8
    Jo = (ctypes.c_int * jcap)()
    nJ = ctypes.c_int()
    yc = y.c()
    w = _check(_lib.tt_cross(ctx.h, fn, arr, len(inputs), fp, n1, n2, J, len(J0), eps, r_max,
                             sweeps, kick, ctypes.c_uint64(key & 0xFFFFFFFFFFFFFFFF),
                             ctypes.byref(yc), Jo, ctypes.byref(nJ)), "tt_cross")
    y.rank = yc.rank
    return w, np.array(Jo[:nJ.value], dtype=np.int64)


def tt_cross_skeleton(ctx: Ctx, fn: int, inputs: Sequence[DeviceTT], fparams: Sequence[float],
                      n1: int, n2: int, J: Sequence[int], I: Sequence[int], eps: float,
                      r_max: int, y: DeviceTT) -> int:
    arr = (TTMatrixC * len(inputs))(*[t.c() for t in inputs])
    fp = (ctypes.c_double * max(1, len(fparams)))(*fparams)
    Jc = (ctypes.c_int * max(1, len(J)))(*[int(j) for j in J])
    Ic = (ctypes.c_int * max(1, len(I)))(*[int(i) for i in I])
    yc = y.c()
    w = _check(_lib.tt_cross_skeleton(ctx.h, fn, arr, len(inputs), fp, n1, n2, Jc, len(J), Ic,
                                      len(I), eps, r_max, ctypes.byref(yc)), "tt_cross_skeleton")
    y.rank = yc.rank
    return w


def tt_recon_core(ctx: Ctx, core, scheme: int, periodic: bool, sign: float = 1.0):
    """core: torch (r, n).  Returns (face_m, face_p, quad) torch tensors (r, n_f) and (r, n*nq)."""
    torch = _torch()
    r, n = core.shape
    nf = n if periodic else n + 1
    nq = 2 if scheme == 3 else 3
    fm = torch.empty((r, nf), dtype=torch.float64, device=core.device)
    fp = torch.empty((r, nf), dtype=torch.float64, device=core.device)
    q = torch.empty((r, n * nq), dtype=torch.float64, device=core.device)
    _check(_lib.tt_recon_core(ctx.h, ctypes.c_void_p(core.data_ptr()), n, r, scheme,
                              1 if periodic else 0, sign, ctypes.c_void_p(fm.data_ptr()),
                              ctypes.c_void_p(fp.data_ptr()), ctypes.c_void_p(q.data_ptr())),
           "tt_recon_core")
    return fm, fp, q


SCHEMES = {"upwind3": 3, "upwind5": 5, "weno5": 55}


class Solver:
    def __init__(self, h, params: ParamsC, ctx_stream):
        self.h, self.params, self._stream = h, params, ctx_stream

    def close(self):
        if self.h:
            _lib.tt_fv_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tt_fv_init(n: int, scheme: str, nonlinear: bool, periodic: bool, q0: Sequence[DeviceTT],
               g: float = 9.81, H0: float = 1.0, f: float = 0.0, eps: float = 1e-10,
               r_max: int = 32, taylor_terms: int = 8, cross_sweeps: int = 3,
               cross_kick: int = 4, recip: str = "taylor", workers: int = 0, stream=None,
               arena_bytes: int = 4 << 30, precision: str = "f64",
               qr: str = "auto", cross_drop: float = 0.0, eps_rule: str = "fixed",
               c_eps: float = 1.0, bc=None, t0: float = 0.0, terms=(),
               flux: str = "products", cross_enrich: str = "kicks",
               graph: bool = False, graph_iters: int = 0) -> Solver:
    """bc: per-axis boundary kinds ("periodic", "wall", "exact") overriding `periodic`;
    terms: separable forcing / ghost terms (see tt_fv_set_terms); graph: fixed shapes and a
    captured HIP graph per step (tt_fv_params.graph)."""
    L = load_library()
    _torch()
    bx, by = (None, None) if bc is None else bc
    p = ParamsC(n, 1 if nonlinear else 0, SCHEMES[scheme], 1 if periodic else 0, g, H0, f, eps,
                r_max, taylor_terms, cross_sweeps, cross_kick, 1 if recip == "cross" else 0,
                workers, PRECISIONS[precision], QR_METHODS[qr], cross_drop,
                EPS_RULES[eps_rule], c_eps, BCS[bx], BCS[by], t0, FLUXES[flux],
                ENRICH[cross_enrich], 1 if graph else 0, graph_iters)
    arr = (TTMatrixC * 3)(*[t.c() for t in q0])
    h = ctypes.c_void_p()
    _check(L.tt_fv_init(ctypes.byref(h), ctypes.byref(p), arr, _stream_ptr(stream), arena_bytes),
           "tt_fv_init")
    s = Solver(h, p, stream)
    if terms:
        tt_fv_set_terms(s, terms)
    return s


def tt_fv_max_speed(s: Solver):
    sp = (ctypes.c_double * 2)()
    _check(_lib.tt_fv_max_speed(s.h, sp), "tt_fv_max_speed")
    return float(sp[0]), float(sp[1])


def tt_fv_cfl_dt(s: Solver, cfl: float) -> float:
    dt = ctypes.c_double()
    _check(_lib.tt_fv_cfl_dt(s.h, cfl, ctypes.byref(dt)), "tt_fv_cfl_dt")
    return dt.value


def tt_fv_set_terms(s: Solver, terms) -> None:
    """Separable terms amp cos(omega t + phase) X Y: forcing of L, or ghost cells of an exact
    boundary ("x_lo", "x_hi", "y_lo", "y_hi")."""
    arr, keep = _terms_c(list(terms))
    _check(_lib.tt_fv_set_terms(s.h, arr, len(terms)), "tt_fv_set_terms")


def tt_fv_step(s: Solver, dt: float, nsteps: int = 1) -> int:
    return _check(_lib.tt_fv_step(s.h, dt, nsteps), "tt_fv_step")


def tt_fv_get_state(s: Solver) -> List[DeviceTT]:
    n, cap = s.params.n, s.params.r_max
    out = [DeviceTT(n, n, cap) for _ in range(3)]
    arr = (TTMatrixC * 3)(*[t.c() for t in out])
    _check(_lib.tt_fv_get_state(s.h, arr), "tt_fv_get_state")
    for t, c in zip(out, arr):
        t.rank = c.rank
    return out


def tt_fv_get_stats(s: Solver) -> dict:
    st = StatsC()
    _check(_lib.tt_fv_get_stats(s.h, ctypes.byref(st)), "tt_fv_get_stats")
    return {"steps": st.steps, "ranks": list(st.ranks), "roundings": st.roundings,
            "crosses": st.crosses, "last_taylor_terms": st.last_taylor_terms,
            "last_taylor_err": st.last_taylor_err, "warnings": st.warnings,
            "flops": st.flops, "bytes": st.bytes, "timed_ms": st.timed_ms,
            "timed_launches": st.timed_launches, "timed_flops": st.timed_flops,
            "timed_bytes": st.timed_bytes, "cross_sweeps_run": st.cross_sweeps_run,
            "learned_crosses": st.learned_crosses, "learned_fallbacks": st.learned_fallbacks,
            "max_learned_err": st.max_learned_err, "sketch_fallbacks": st.sketch_fallbacks,
            "sketch_unconverged": st.sketch_unconverged, "jacobi_capped": st.jacobi_capped,
            "qr_redos": st.qr_redos, "eps_inner": st.eps_inner,
            "eps_var": list(st.eps_var), "time": st.time, "graph_launches": st.graph_launches}


def tt_fv_time_kernel(s: Solver, name: Optional[str], every: int = 32) -> None:
    _check(_lib.tt_fv_time_kernel(s.h, (name or "").encode(), every), "tt_fv_time_kernel")


def tt_fv_destroy(s: Solver) -> None:
    s.close()


class Grid:
    """Full-grid comparator (tt_grid_*): the same scheme on n x n cell-average arrays."""

    def __init__(self, n: int, scheme: str, nonlinear: bool, periodic: bool, g: float = 9.81,
                 H0: float = 1.0, f: float = 0.0, stream=None, bc=None, t0: float = 0.0,
                 terms=()):
        L = load_library()
        _torch()
        bx, by = (None, None) if bc is None else bc
        self.params = ParamsC(n, 1 if nonlinear else 0, SCHEMES[scheme], 1 if periodic else 0,
                              g, H0, f, 0.0, 1, 1, 1, 0, 0, 0, 0, 0, 0.0, 0, 1.0,
                              BCS[bx], BCS[by], t0, 0, 0)
        self.h = ctypes.c_void_p()
        self._stream = stream
        _check(L.tt_grid_init(ctypes.byref(self.h), ctypes.byref(self.params),
                              _stream_ptr(stream)), "tt_grid_init")
        if terms:
            self.set_terms(terms)

    def set_terms(self, terms) -> None:
        arr, keep = _terms_c(list(terms))
        _check(_lib.tt_grid_set_terms(self.h, arr, len(terms)), "tt_grid_set_terms")

    def step(self, U, dt: float, nsteps: int = 1) -> None:
        """Advance U (torch float64 CUDA tensor, 3 x n x n, contiguous) in place; asynchronous
        on the grid's stream."""
        n = self.params.n
        if (tuple(U.shape) != (3, n, n) or not U.is_contiguous() or not U.is_cuda or
                str(U.dtype) != "torch.float64"):
            raise ValueError("tt_grid_step: U must be a contiguous float64 CUDA tensor 3 x n x n")
        _check(_lib.tt_grid_step(self.h, ctypes.c_void_p(U.data_ptr()), dt, nsteps),
               "tt_grid_step")

    def close(self):
        if self.h:
            _lib.tt_grid_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tt_grid_init(n: int, scheme: str, nonlinear: bool, periodic: bool, g: float = 9.81,
                 H0: float = 1.0, f: float = 0.0, stream=None, bc=None, t0: float = 0.0,
                 terms=()) -> Grid:
    return Grid(n, scheme, nonlinear, periodic, g, H0, f, stream, bc, t0, terms)


def tt_grid_step(grid: Grid, U, dt: float, nsteps: int = 1) -> None:
    grid.step(U, dt, nsteps)


def tt_grid_destroy(grid: Grid) -> None:
    grid.close()


class Ensemble:
    def __init__(self, workers: int = 8, arena_bytes_per_worker: int = 1 << 30):
        L = load_library()
        _torch()
        self.h = ctypes.c_void_p()
        _check(L.tt_ens_create(ctypes.byref(self.h), workers, arena_bytes_per_worker),
               "tt_ens_create")

    def close(self):
        if self.h:
            _lib.tt_ens_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tt_ens_create(workers: int = 8, arena_bytes_per_worker: int = 1 << 30) -> Ensemble:
    return Ensemble(workers, arena_bytes_per_worker)


def tt_ens_step(e: Ensemble, members: Sequence[Solver], dts: Sequence[float], nsteps: int = 1,
                concurrency: int = 8) -> int:
    hs = (ctypes.c_void_p * len(members))(*[m.h.value for m in members])
    d = (ctypes.c_double * len(members))(*dts)
    return _check(_lib.tt_ens_step(e.h, hs, len(members), d, nsteps, concurrency), "tt_ens_step")


def tt_ens_destroy(e: Ensemble) -> None:
    e.close()


# ---- learned pivot proposer -------------------------------------------------------------

class PivotModel:
    """Handle of a pivot-proposer model (weights on the device, training log)."""

    def __init__(self, max_rows: int = 0, seed: int = 0):
        L = load_library()
        _torch()
        self.h = ctypes.c_void_p()
        _check(L.tt_pm_create(ctypes.byref(self.h), max_rows, seed), "tt_pm_create")

    def close(self):
        if self.h:
            _lib.tt_pm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, flat: np.ndarray) -> None:
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(_lib.tt_pm_set_weights(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                      a.size), "tt_pm_set_weights")

    def get_weights(self) -> np.ndarray:
        a = np.zeros(PM_NPARAM, dtype=np.float32)
        _check(_lib.tt_pm_get_weights(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                      a.size), "tt_pm_get_weights")
        return a

    def forward(self, X):
        """X: torch float32 (N, 16) on the GPU -> scores (N,) float32."""
        torch = _torch()
        X = X.contiguous()
        s = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(_lib.tt_pm_forward(self.h, X.data_ptr(), X.shape[0], s.data_ptr()),
               "tt_pm_forward")
        return s

    def grad(self, X, y, pos_weight: float):
        X, y = X.contiguous(), y.contiguous()
        g = np.zeros(PM_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        _check(_lib.tt_pm_grad(self.h, X.data_ptr(), y.data_ptr(), X.shape[0], pos_weight,
                               g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), g.size,
                               ctypes.byref(loss)), "tt_pm_grad")
        return loss.value, g

    def adam(self, grad: np.ndarray, lr: float) -> None:
        """One Adam step of the weights with a given (host) gradient."""
        a = np.ascontiguousarray(grad, dtype=np.float32)
        _check(_lib.tt_pm_adam(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size,
                               lr), "tt_pm_adam")

    def train(self, epochs: int = 4, batch: int = 8192, lr: float = 1e-3) -> float:
        loss = ctypes.c_double()
        _check(_lib.tt_pm_train(self.h, epochs, batch, lr, ctypes.byref(loss)), "tt_pm_train")
        return loss.value

    def dataset(self):
        rows, pos = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.tt_pm_dataset(self.h, ctypes.byref(rows), ctypes.byref(pos)), "tt_pm_dataset")
        return rows.value, pos.value


def pm_flat(p: dict) -> np.ndarray:
    """Flat parameter vector from W1, b1, W2, b2, w3, b3 arrays."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def pm_unflat(flat: np.ndarray) -> dict:
    F, H = 16, 256
    sizes = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
    out, o = {}, 0
    for k, shp in sizes:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def tt_pm_features(ctx: Ctx, B0, r: int, J_prev):
    """Features (n2, 16) float32 of a cross whose starting TT has second core B0 (torch
    float64 tensor (cap, n2) as in DeviceTT.g2; the first r rows are used)."""
    torch = _torch()
    n2 = B0.shape[1]
    Jd = torch.tensor(list(J_prev) or [0], dtype=torch.int32, device=B0.device)
    X = torch.empty((n2, 16), dtype=torch.float32, device=B0.device)
    _check(_lib.tt_pm_features(ctx.h, B0.data_ptr(), n2, r, n2, Jd.data_ptr(), len(J_prev),
                               X.data_ptr()), "tt_pm_features")
    return X


def tt_pm_topk(ctx: Ctx, s, k: int):
    torch = _torch()
    out = torch.empty(k, dtype=torch.int32, device=s.device)
    _check(_lib.tt_pm_topk(ctx.h, s.data_ptr(), s.shape[0], k, out.data_ptr()), "tt_pm_topk")
    return out


def tt_fv_set_pivots(s: Solver, mode: str, model: Optional[PivotModel] = None) -> None:
    _check(_lib.tt_fv_set_pivots(s.h, PIVOTS[mode], model.h if model is not None else None),
           "tt_fv_set_pivots")


def tt_fv_set_pivot_acceptance(s: Solver, abs_tol: float = 1e-6, rel_slack: float = -1.0) -> None:
    _check(_lib.tt_fv_set_pivot_acceptance(s.h, abs_tol, rel_slack),
           "tt_fv_set_pivot_acceptance")


def tt_fv_replay_pivots(s: Solver, step: int, site: int, J: Sequence[int],
                        I: Sequence[int]) -> None:
    Jc = (ctypes.c_int * max(1, len(J)))(*[int(j) for j in J])
    Ic = (ctypes.c_int * max(1, len(I)))(*[int(i) for i in I])
    _check(_lib.tt_fv_replay_pivots(s.h, step, site, Jc, len(J), Ic, len(I)),
           "tt_fv_replay_pivots")


def tt_fv_get_pivots(s: Solver, site: int, cap: int = 256):
    """(J, I) of the latest cross at `site`, or None when the site has not run."""
    Jc, Ic = (ctypes.c_int * cap)(), (ctypes.c_int * cap)()
    nJ, nI = ctypes.c_int(), ctypes.c_int()
    had = _check(_lib.tt_fv_get_pivots(s.h, site, Jc, cap, ctypes.byref(nJ), Ic, cap,
                                       ctypes.byref(nI)), "tt_fv_get_pivots")
    if not had:
        return None
    return (np.array(Jc[:nJ.value], dtype=np.int64), np.array(Ic[:nI.value], dtype=np.int64))


def tt_gemm_autotune(on: bool) -> int:
    """Switch the GEMM tile-shape autotuner on or off; returns the number of tuned classes."""
    load_library()
    n = ctypes.c_int()
    _check(_lib.tt_gemm_autotune(1 if on else 0, ctypes.byref(n)), "tt_gemm_autotune")
    return n.value

"""Python binding of libapx (MI355X dense affinity propagation).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libapx.so``; PyTorch supplies device memory and the stream.
The function names match the C ABI in ``include/apx.h``.

Matrices are 2-D float32 CUDA tensors of shape (n, n) with unit column
stride; their row stride is the leading dimension ``ld`` (a multiple of 4).
``empty_matrix`` allocates such a view with rows padded to 64 elements.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapx.so")

APX_OK, APX_EINVAL, APX_ENOMEM, APX_EDEVICE, APX_ENOTIMPL = range(5)
APX_PREF_MEDIAN, APX_PREF_SCALAR, APX_PREF_VECTOR = range(3)
APX_COLD, APX_WARM_A, APX_WARM_AR, APX_WARM_COLUMNS = range(4)
APX_MLP_FEATURES, APX_MLP_PARAMS = 16, 18946
APX_RAW_LABELS, APX_CHECK_FINITE, APX_MSG_THRESHOLD = 1, 2, 4
(APX_OP_SIMILARITY, APX_OP_ITERATE, APX_OP_SOLVE, APX_OP_SOLVE_BATCHED, APX_OP_PAP, APX_OP_LAP,
 APX_OP_FEATURES, APX_OP_MLP_BACKWARD, APX_OP_WARMSTART, APX_OP_LAP_FULL, APX_OP_SOLVE_MF) = range(11)
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTIMPL"}


class ApxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"apx {_STATUS.get(status, status)}: {msg}")
        self.status = status


class apx_params(ctypes.Structure):
    _fields_ = [("damping", ctypes.c_float), ("max_iter", ctypes.c_int32),
                ("conv_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("msg_tol", ctypes.c_float)]


class apx_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_exemplars", ctypes.c_int32), ("status", ctypes.c_int32),
                ("dpsim", ctypes.c_double), ("expref", ctypes.c_double),
                ("netsim", ctypes.c_double)]


class apx_lap_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("step1_centres", ctypes.c_int32),
                ("assigned", ctypes.c_int64), ("unassigned", ctypes.c_int64),
                ("merged_centres", ctypes.c_int32), ("step3_mode", ctypes.c_int32),
                ("refined_centres", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("preference", ctypes.c_double)]


class apx_instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("S", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("A", ctypes.c_void_p), ("idx", ctypes.c_void_p)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32

# name -> (restype, argtypes); every symbol include/apx.h declares
SIGNATURES = {
    "apx_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "apx_destroy": (None, [_P]),
    "apx_set_stream": (ctypes.c_int, [_P, _P]),
    "apx_last_error": (ctypes.c_char_p, [_P]),
    "apx_workspace_bytes": (ctypes.c_size_t, [_P]),
    "apx_workspace_size": (ctypes.c_size_t, [_P, _I32, _I64, _I64, _I64, _I32, _P]),
    "apx_set_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "apx_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "apx_set_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "apx_set_lean_scan": (ctypes.c_int, [_P, ctypes.c_int]),
    "apx_last_lean_rescans": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "apx_set_implicit": (ctypes.c_int, [_P, _I32, _I64]),
    "apx_set_implicit_a": (ctypes.c_int, [_P, _I32, _I64]),
    "apx_last_solve_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "apx_last_fallback": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "apx_autotune": (ctypes.c_int, [_P, _I64]),
    "apx_set_autotune": (ctypes.c_int, [_P, ctypes.c_int]),
    "apx_tune_set": (ctypes.c_int, [_P, _I64, _I32, _I32, _I32]),
    "apx_tune_get": (ctypes.c_int, [_P, _I64, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                    ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)]),
    "apx_tune_clear": (ctypes.c_int, [_P]),
    "apx_autotune_form": (ctypes.c_int, [_P, _I64, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)]),
    "apx_tune_set_form": (ctypes.c_int, [_P, _I64, _I32]),
    "apx_autotune_batched": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                                            ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)]),
    "apx_tune_get_form": (ctypes.c_int, [_P, _I64, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)]),
    "apx_tune_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "apx_tune_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "apx_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double)]),
    "ap_similarity": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _P, _I64, _I32, _P, ctypes.c_float,
                                     ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "ap_iterate": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P, ctypes.c_float, _I32, _P]),
    "ap_iterate_noalloc": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P, ctypes.c_float, _I32, _P]),
    "ap_solve": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P, _I32, ctypes.POINTER(apx_params), _P,
                                ctypes.POINTER(apx_result)]),
    "ap_solve_mf": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _I32, _P, ctypes.c_float, ctypes.c_uint64,
                                   ctypes.c_double, _I64, ctypes.POINTER(apx_params), _P,
                                   ctypes.POINTER(apx_result), ctypes.POINTER(ctypes.c_double)]),
    "ap_solve_batched": (ctypes.c_int, [_P, _I32, ctypes.POINTER(apx_instance), _I32,
                                        ctypes.POINTER(apx_params), ctypes.POINTER(apx_result)]),
    "pap_solve": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P, _I32, _P, _P, ctypes.POINTER(apx_params),
                                 _P, ctypes.POINTER(apx_result), ctypes.POINTER(apx_result)]),
    "lap_solve": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _I64, _P, ctypes.c_uint64, ctypes.c_double,
                                 _I32, ctypes.c_float, ctypes.POINTER(apx_params), _P,
                                 ctypes.POINTER(apx_result), _P]),
    "lap_full_solve": (ctypes.c_int, [_P, _P, _I64, _I64, _I64, _I64, _P, ctypes.c_uint64, ctypes.c_double,
                                      _I32, ctypes.c_float, _I64, ctypes.POINTER(apx_params), _P,
                                      ctypes.POINTER(apx_result), ctypes.POINTER(apx_lap_stats), _P]),
    "apx_lap_landmarks": (ctypes.c_int, [_I64, _I64, _P, _I64, ctypes.c_uint64, _P]),
    "apx_features": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P]),
    "apx_mlp_forward": (ctypes.c_int, [_P, _P, _P, _I64, _P]),
    "apx_mlp_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _I64, _P, _P]),
    "apx_mlp_adam": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _I32, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float]),
    "apx_targets": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P]),
    "apx_warm_a0": (ctypes.c_int, [_P, _P, _P, _I64, _P, _I64]),
    "ap_warmstart": (ctypes.c_int, [_P, _P, _I64, _I64, _P, _P, _P, _P]),
}


def lib() -> ctypes.CDLL:
    """Load libapx.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0910_1650_amd/build.py "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


_ctxs: dict[int, ctypes.c_void_p] = {}


def context(device: torch.device | int | None = None) -> ctypes.c_void_p:
    """The library context of a device, bound to torch's current stream."""
    if device is None:
        device = torch.cuda.current_device()
    dev = torch.device("cuda", device) if isinstance(device, int) else device
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    L = lib()
    stream = torch.cuda.current_stream(idx).cuda_stream
    if idx not in _ctxs:
        h = _P()
        st = L.apx_create(ctypes.byref(h), idx, _P(stream))
        if st != APX_OK:
            raise ApxError(st, f"apx_create on device {idx}")
        _ctxs[idx] = h
    else:
        L.apx_set_stream(_ctxs[idx], _P(stream))
    return _ctxs[idx]


def _check(ctx, st: int, what: str):
    if st != APX_OK:
        raise ApxError(st, f"{what}: {lib().apx_last_error(ctx).decode()}")


def round_ld(n: int, align: int = 64) -> int:
    return max(align, (n + align - 1) // align * align)


def empty_matrix(n: int, device="cuda", fill: float | None = None) -> torch.Tensor:
    """(n, n) float32 view whose rows are padded to a multiple of 64 elements."""
    ld = round_ld(n)
    base = torch.empty((max(n, 1), ld), dtype=torch.float32, device=device)
    if fill is not None:
        base.fill_(fill)
    return base[:n, :n]


def to_matrix(M: torch.Tensor) -> torch.Tensor:
    """Copy a dense (n, n) tensor into a padded device matrix."""
    n = M.shape[0]
    out = empty_matrix(n, device="cuda")
    out.copy_(M.to(device="cuda", dtype=torch.float32))
    return out


def _mat(M: torch.Tensor, name: str, n: int | None = None):
    if not (M.is_cuda and M.dtype == torch.float32 and M.dim() == 2):
        raise ValueError(f"{name} must be a 2-D float32 CUDA tensor")
    if M.shape[0] != M.shape[1] or M.stride(1) != 1:
        raise ValueError(f"{name} must be square with unit column stride")
    if n is not None and M.shape[0] != n:
        raise ValueError(f"{name} has {M.shape[0]} rows, expected {n}")
    return _P(M.data_ptr()), M.shape[0], M.stride(0)


@dataclass
class Result:
    iterations: int
    converged: bool
    n_exemplars: int
    dpsim: float
    expref: float
    netsim: float


def _res(r: apx_result) -> Result:
    return Result(r.iterations, bool(r.converged), r.n_exemplars, r.dpsim, r.expref, r.netsim)


def ap_similarity(X: torch.Tensor, S: torch.Tensor | None = None, pref: str | float | torch.Tensor = "median",
                  noise_seed: int = 0, noise_rel: float = 1e-12):
    """S (padded (n,n) view) from points X (n,d) float32; returns (S, preference)."""
    if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
        raise ValueError("X must be a 2-D float32 CUDA tensor with unit column stride")
    n, d = X.shape
    if S is None:
        S = empty_matrix(n, device=X.device)
    Sp, _, ld = _mat(S, "S", n)
    ctx = context(X.device)
    if isinstance(pref, str):
        mode, vec, scal = APX_PREF_MEDIAN, None, 0.0
    elif isinstance(pref, torch.Tensor):
        mode, vec, scal = APX_PREF_VECTOR, pref.contiguous(), 0.0
    else:
        mode, vec, scal = APX_PREF_SCALAR, None, float(pref)
    out = ctypes.c_double(float("nan"))
    st = lib().ap_similarity(ctx, _P(X.data_ptr()), n, d, X.stride(0), Sp, ld, mode,
                             _P(vec.data_ptr()) if vec is not None else None, scal,
                             noise_seed, noise_rel, ctypes.byref(out))
    _check(ctx, st, "ap_similarity")
    return S, out.value


def ap_iterate(S: torch.Tensor, R: torch.Tensor, A: torch.Tensor, damping: float, n_iter: int,
               decision: torch.Tensor | None = None) -> None:
    """n_iter damped AP iterations on (R, A) in place (asynchronous)."""
    Sp, n, ld = _mat(S, "S")
    Rp, _, ldr = _mat(R, "R", n)
    Ap, _, lda = _mat(A, "A", n)
    if not (ld == ldr == lda):
        raise ValueError("S, R and A must share one leading dimension")
    dp = None
    if decision is not None:
        if not (decision.is_cuda and decision.dtype == torch.int32 and decision.numel() == n):
            raise ValueError("decision must be an int32 CUDA tensor of n entries")
        dp = _P(decision.data_ptr())
    ctx = context(S.device)
    _check(ctx, lib().ap_iterate(ctx, Sp, n, ld, Rp, Ap, damping, n_iter, dp), "ap_iterate")


def ap_iterate_noalloc(S: torch.Tensor, R: torch.Tensor, A: torch.Tensor, damping: float, n_iter: int,
                       decision: torch.Tensor | None = None) -> None:
    """ap_iterate on the library's fixed scratch array (no device allocation;
    n <= 8192; calls overlapping on one GPU race)."""
    Sp, n, ld = _mat(S, "S")
    Rp, _, ldr = _mat(R, "R", n)
    Ap, _, lda = _mat(A, "A", n)
    if not (ld == ldr == lda):
        raise ValueError("S, R and A must share one leading dimension")
    dp = None
    if decision is not None:
        if not (decision.is_cuda and decision.dtype == torch.int32 and decision.numel() == n):
            raise ValueError("decision must be an int32 CUDA tensor of n entries")
        dp = _P(decision.data_ptr())
    ctx = context(S.device)
    _check(ctx, lib().ap_iterate_noalloc(ctx, Sp, n, ld, Rp, Ap, damping, n_iter, dp), "ap_iterate_noalloc")


def ap_solve(S: torch.Tensor, R: torch.Tensor, A: torch.Tensor, damping: float = 0.5,
             max_iter: int = 200, conv_iter: int = 15, warm: int = APX_COLD,
             idx: torch.Tensor | None = None, check_every: int = 0, flags: int = 0,
             msg_tol: float = 0.0):
    """Algorithm 1 to its stop rule; returns (idx int32 tensor, Result).
    flags: APX_RAW_LABELS | APX_CHECK_FINITE | APX_MSG_THRESHOLD (with msg_tol)."""
    Sp, n, ld = _mat(S, "S")
    Rp, _, ldr = _mat(R, "R", n)
    Ap, _, lda = _mat(A, "A", n)
    if not (ld == ldr == lda):
        raise ValueError("S, R and A must share one leading dimension")
    if idx is None:
        idx = torch.empty(n, dtype=torch.int32, device=S.device)
    prm = apx_params(damping, max_iter, conv_iter, check_every, flags, msg_tol)
    res = apx_result()
    ctx = context(S.device)
    _check(ctx, lib().ap_solve(ctx, Sp, n, ld, Rp, Ap, warm, ctypes.byref(prm), _P(idx.data_ptr()),
                               ctypes.byref(res)), "ap_solve")
    return idx, _res(res)


def ap_solve_mf(X: torch.Tensor, pref: str | float | torch.Tensor = "median", noise_seed: int = 0,
                noise_rel: float = 1e-12, damping: float = 0.5, max_iter: int = 200, conv_iter: int = 15,
                panel_rows: int = 0, check_every: int = 0, flags: int = 0):
    """Matrix-free Algorithm 1 from the points X (n,d) float32: S is rebuilt panel by
    panel each iteration (no n x n buffer); returns (idx int32 tensor, Result, preference)."""
    if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
        raise ValueError("X must be a 2-D float32 CUDA tensor with unit column stride")
    n, d = X.shape
    if isinstance(pref, str):
        mode, vec, scal = APX_PREF_MEDIAN, None, 0.0
    elif isinstance(pref, torch.Tensor):
        mode, vec, scal = APX_PREF_VECTOR, pref.contiguous(), 0.0
    else:
        mode, vec, scal = APX_PREF_SCALAR, None, float(pref)
    idx = torch.empty(n, dtype=torch.int32, device=X.device)
    prm = apx_params(damping, max_iter, conv_iter, check_every, flags, 0.0)
    res = apx_result()
    out = ctypes.c_double(float("nan"))
    ctx = context(X.device)
    _check(ctx, lib().ap_solve_mf(ctx, _P(X.data_ptr()), n, d, X.stride(0), mode,
                                  _P(vec.data_ptr()) if vec is not None else None, scal, noise_seed, noise_rel,
                                  panel_rows, ctypes.byref(prm), _P(idx.data_ptr()), ctypes.byref(res),
                                  ctypes.byref(out)), "ap_solve_mf")
    return idx, _res(res), out.value


def apx_workspace_size(op: int, n: int = 0, ld: int = 0, d: int = 0, count: int = 0, sizes=None,
                       device=None) -> int:
    """Device workspace bytes one call of `op` (APX_OP_*) needs."""
    import numpy as np
    sz = None if sizes is None else np.ascontiguousarray(sizes, dtype=np.int64)
    ctx = context(device)
    return int(lib().apx_workspace_size(ctx, op, n, ld, d, count,
                                        None if sz is None else _P(sz.ctypes.data)))


def apx_set_workspace(buf: torch.Tensor | None, device=None) -> None:
    """Hand a caller-owned uint8 CUDA tensor to the library as its workspace
    (None: back to a library-owned one).  Keep `buf` alive while it is set."""
    ctx = context(device)
    if buf is None:
        _check(ctx, lib().apx_set_workspace(ctx, None, 0), "apx_set_workspace")
        return
    if not (buf.is_cuda and buf.dtype == torch.uint8 and buf.is_contiguous()):
        raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
    _check(ctx, lib().apx_set_workspace(ctx, _P(buf.data_ptr()), buf.numel()), "apx_set_workspace")


def apx_workspace_bytes(device=None) -> int:
    ctx = context(device)
    return int(lib().apx_workspace_bytes(ctx))


def apx_set_implicit(list_capacity: int, min_n: int = 8192, device=None) -> None:
    """Implicit responsibilities in ap_solve for n >= min_n: list capacity
    1..16, or 0 for explicit R."""
    ctx = context(device)
    _check(ctx, lib().apx_set_implicit(ctx, list_capacity, min_n), "apx_set_implicit")


def apx_set_implicit_a(list_capacity: int, min_n: int = 4096, device=None) -> None:
    """Implicit availabilities in ap_solve on a cold start with n >= min_n
    (with implicit R): exception list capacity 1..1024 per row, or 0 for
    explicit A."""
    ctx = context(device)
    _check(ctx, lib().apx_set_implicit_a(ctx, list_capacity, min_n), "apx_set_implicit_a")


def apx_last_solve_info(device=None) -> tuple[int, int, int]:
    """(iterations with implicit R, iterations with explicit R, iterations
    with implicit A) of the last ap_solve."""
    ctx = context(device)
    a, b, c = _I32(), _I32(), _I32()
    _check(ctx, lib().apx_last_solve_info(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "apx_last_solve_info")
    return a.value, b.value, c.value


APX_FALLBACK_R_LIST, APX_FALLBACK_A_LIST, APX_FALLBACK_R_OWNER, APX_NOTE_R_OWNER = 1, 2, 4, 8


def apx_last_fallback(device=None) -> int:
    """Why the last ap_solve left an implicit form (OR of APX_FALLBACK_*; 0: it did not)."""
    ctx = context(device)
    a = _I32()
    _check(ctx, lib().apx_last_fallback(ctx, ctypes.byref(a)), "apx_last_fallback")
    return a.value


def apx_set_lean_scan(enable: bool, device=None) -> None:
    """Lean implicit-A scan (default) or r formed for every element; results are identical."""
    ctx = context(device)
    _check(ctx, lib().apx_set_lean_scan(ctx, int(bool(enable))), "apx_set_lean_scan")


def apx_last_lean_rescans(device=None) -> int:
    """Rows of the last ap_solve whose ordinary columns decided the exemplar flag after the reduction."""
    ctx = context(device)
    a = _I32()
    _check(ctx, lib().apx_last_lean_rescans(ctx, ctypes.byref(a)), "apx_last_lean_rescans")
    return a.value


def apx_set_graphs(enable: bool, device=None) -> None:
    """Replay ap_solve's iteration loop as a captured HIP graph (default) or not."""
    ctx = context(device)
    _check(ctx, lib().apx_set_graphs(ctx, int(bool(enable))), "apx_set_graphs")


def apx_autotune(n: int, device=None) -> dict:
    """Tune the row pass for size n now; returns the chosen entry."""
    ctx = context(device)
    _check(ctx, lib().apx_autotune(ctx, n), "apx_autotune")
    return apx_tune_get(n, device)


def apx_set_autotune(enable: bool, device=None) -> None:
    ctx = context(device)
    _check(ctx, lib().apx_set_autotune(ctx, int(bool(enable))), "apx_set_autotune")


def apx_tune_set(n: int, threads: int, lds: bool, check_every: int = 0, device=None) -> None:
    ctx = context(device)
    _check(ctx, lib().apx_tune_set(ctx, n, threads, int(bool(lds)), check_every), "apx_tune_set")


def apx_tune_get(n: int, device=None) -> dict:
    ctx = context(device)
    t, l, c = _I32(), _I32(), _I32()
    ms = ctypes.c_double()
    _check(ctx, lib().apx_tune_get(ctx, n, ctypes.byref(t), ctypes.byref(l), ctypes.byref(c),
                                   ctypes.byref(ms)), "apx_tune_get")
    return dict(threads=t.value, lds=bool(l.value), check_every=c.value, ms_per_iter=ms.value)


APX_FORM_DEFAULT, APX_FORM_EXPLICIT, APX_FORM_IMPLICIT_R, APX_FORM_IMPLICIT_RA = range(4)


def apx_autotune_form(n: int, device=None) -> dict:
    """Time the three message forms at n (synthetic problem) and keep the fastest."""
    ctx = context(device)
    f = _I32()
    ms = (ctypes.c_double * 3)()
    _check(ctx, lib().apx_autotune_form(ctx, n, ctypes.byref(f), ms), "apx_autotune_form")
    return dict(form=f.value, ms=list(ms))


def apx_autotune_batched(sizes, device=None) -> dict:
    """Time the batched launch plans for a batch of these sizes and keep the fastest."""
    ctx = context(device)
    arr = (_I64 * len(sizes))(*[int(x) for x in sizes])
    w, m = _I32(), _I32()
    ms = ctypes.c_double()
    _check(ctx, lib().apx_autotune_batched(ctx, len(sizes), arr, ctypes.byref(w), ctypes.byref(m), ctypes.byref(ms)),
           "apx_autotune_batched")
    return dict(wpc=w.value, min_rows=m.value, ms=ms.value)


def apx_tune_set_form(n: int, form: int, device=None) -> None:
    ctx = context(device)
    _check(ctx, lib().apx_tune_set_form(ctx, n, form), "apx_tune_set_form")


def apx_tune_get_form(n: int, device=None) -> dict:
    ctx = context(device)
    f = _I32()
    ms = (ctypes.c_double * 3)()
    _check(ctx, lib().apx_tune_get_form(ctx, n, ctypes.byref(f), ms), "apx_tune_get_form")
    return dict(form=f.value, ms=list(ms))


def apx_tune_clear(device=None) -> None:
    ctx = context(device)
    _check(ctx, lib().apx_tune_clear(ctx), "apx_tune_clear")


def apx_tune_save(path: str, device=None) -> None:
    ctx = context(device)
    _check(ctx, lib().apx_tune_save(ctx, os.fsencode(path)), "apx_tune_save")


def apx_tune_load(path: str, device=None) -> None:
    ctx = context(device)
    _check(ctx, lib().apx_tune_load(ctx, os.fsencode(path)), "apx_tune_load")


def apx_profile(enable: bool, device=None) -> None:
    """Enable/disable event timing of the full row passes inside ap_solve."""
    ctx = context(device)
    _check(ctx, lib().apx_profile(ctx, int(bool(enable))), "apx_profile")


def apx_profile_read(device=None) -> tuple[int, float]:
    """(launches, total milliseconds) of timed row passes since the last read."""
    ctx = context(device)
    n, ms = _I64(0), ctypes.c_double(0.0)
    _check(ctx, lib().apx_profile_read(ctx, ctypes.byref(n), ctypes.byref(ms)), "apx_profile_read")
    return int(n.value), float(ms.value)


def ap_solve_batched(S_list, R_list=None, A_list=None, damping: float = 0.5, max_iter: int = 200,
                     conv_iter: int = 15, warm: int = APX_COLD, check_every: int = 0, flags: int = 0):
    """Algorithm 1 on many instances in one batch; returns ([idx tensors], [Result])."""
    count = len(S_list)
    R_list = R_list or [empty_matrix(S.shape[0], device=S.device) for S in S_list]
    A_list = A_list or [empty_matrix(S.shape[0], device=S.device) for S in S_list]
    insts = (apx_instance * count)()
    idxs = []
    for j, (S, R, A) in enumerate(zip(S_list, R_list, A_list)):
        Sp, n, ld = _mat(S, f"S[{j}]")
        Rp, _, ldr = _mat(R, f"R[{j}]", n)
        Ap, _, lda = _mat(A, f"A[{j}]", n)
        if not (ld == ldr == lda):
            raise ValueError("S, R and A of an instance must share one leading dimension")
        idx = torch.empty(n, dtype=torch.int32, device=S.device)
        idxs.append(idx)
        insts[j] = apx_instance(n, ld, Sp, Rp, Ap, _P(idx.data_ptr()))
    prm = apx_params(damping, max_iter, conv_iter, check_every, flags, 0.0)
    res = (apx_result * count)()
    ctx = context(S_list[0].device)
    _check(ctx, lib().ap_solve_batched(ctx, count, insts, warm, ctypes.byref(prm), res), "ap_solve_batched")
    return idxs, [_res(r) for r in res]


def pap_solve(S: torch.Tensor, R: torch.Tensor, A: torch.Tensor, k: int, perm=None, offsets=None,
              damping: float = 0.5, max_iter: int = 200, conv_iter: int = 15, check_every: int = 0,
              flags: int = 0, msg_tol: float = 0.0):
    """Partition AP (Algorithm 2); returns (idx, Result, [Result per part])."""
    import numpy as np
    Sp, n, ld = _mat(S, "S")
    Rp, _, ldr = _mat(R, "R", n)
    Ap, _, lda = _mat(A, "A", n)
    if not (ld == ldr == lda):
        raise ValueError("S, R and A must share one leading dimension")
    pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    of = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int64)
    idx = torch.empty(n, dtype=torch.int32, device=S.device)
    prm = apx_params(damping, max_iter, conv_iter, check_every, flags, msg_tol)
    res = apx_result()
    sub = (apx_result * k)()
    ctx = context(S.device)
    _check(ctx, lib().pap_solve(ctx, Sp, n, ld, Rp, Ap, k,
                                None if pm is None else _P(pm.ctypes.data),
                                None if of is None else _P(of.ctypes.data),
                                ctypes.byref(prm), _P(idx.data_ptr()), ctypes.byref(res), sub), "pap_solve")
    return idx, _res(res), [_res(r) for r in sub]


def lap_solve(X: torch.Tensor, n_landmarks: int, landmarks=None, seed: int = 0, noise_rel: float = 1e-12,
              damping: float = 0.9, max_iter: int = 2000, conv_iter: int = 15, check_every: int = 0,
              pref: str | float = "median", flags: int = 0, msg_tol: float = 0.0):
    """Landmark AP (Algorithm 3, Steps 1-2); returns (idx, Result, exemplar indices).
    pref: "median" (of the landmark similarities) or one float for every landmark."""
    import numpy as np
    if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
        raise ValueError("X must be a 2-D float32 CUDA tensor with unit column stride")
    n, d = X.shape
    lm = None if landmarks is None else np.ascontiguousarray(landmarks, dtype=np.int64)
    if lm is not None and lm.size != n_landmarks:
        raise ValueError(f"landmarks has {lm.size} entries, expected {n_landmarks}")
    idx = torch.empty(n, dtype=torch.int32, device=X.device)
    prm = apx_params(damping, max_iter, conv_iter, check_every, flags, msg_tol)
    res = apx_result()
    ex = np.zeros(n_landmarks, dtype=np.int64)
    mode, scal = (APX_PREF_MEDIAN, 0.0) if isinstance(pref, str) else (APX_PREF_SCALAR, float(pref))
    ctx = context(X.device)
    _check(ctx, lib().lap_solve(ctx, _P(X.data_ptr()), n, d, X.stride(0), n_landmarks,
                                None if lm is None else _P(lm.ctypes.data), seed, noise_rel,
                                mode, scal, ctypes.byref(prm), _P(idx.data_ptr()), ctypes.byref(res),
                                _P(ex.ctypes.data)), "lap_solve")
    r = _res(res)
    return idx, r, ex[: r.n_exemplars].copy()


def apx_lap_landmarks(n: int, n_landmarks: int, keep=None, seed: int = 0):
    """Landmark set keeping `keep` (e.g. previous exemplars) plus a uniform
    sample of the other points (host only); ascending int64 array."""
    import numpy as np
    kp = np.zeros(0, dtype=np.int64) if keep is None else np.ascontiguousarray(keep, dtype=np.int64)
    out = np.zeros(n_landmarks, dtype=np.int64)
    st = lib().apx_lap_landmarks(n, n_landmarks, _P(kp.ctypes.data) if kp.size else None, kp.size, seed,
                                 _P(out.ctypes.data))
    if st != APX_OK:
        raise ApxError(st, "apx_lap_landmarks: bad arguments")
    return out


def lap_full_solve(X: torch.Tensor, n_landmarks: int, m0: int = 20000, landmarks=None, seed: int = 0,
                   noise_rel: float = 1e-12, damping: float = 0.9, max_iter: int = 2000, conv_iter: int = 15,
                   check_every: int = 0, pref: str | float = "median", flags: int = 0, msg_tol: float = 0.0):
    """Landmark AP, Algorithm 3 Steps 1-4; returns (idx, Result, exemplar
    indices, stats dict)."""
    import numpy as np
    if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
        raise ValueError("X must be a 2-D float32 CUDA tensor with unit column stride")
    n, d = X.shape
    lm = None if landmarks is None else np.ascontiguousarray(landmarks, dtype=np.int64)
    if lm is not None and lm.size != n_landmarks:
        raise ValueError(f"landmarks has {lm.size} entries, expected {n_landmarks}")
    idx = torch.empty(n, dtype=torch.int32, device=X.device)
    prm = apx_params(damping, max_iter, conv_iter, check_every, flags, msg_tol)
    res = apx_result()
    st = apx_lap_stats()
    ex = np.zeros(n, dtype=np.int64)
    mode, scal = (APX_PREF_MEDIAN, 0.0) if isinstance(pref, str) else (APX_PREF_SCALAR, float(pref))
    ctx = context(X.device)
    _check(ctx, lib().lap_full_solve(ctx, _P(X.data_ptr()), n, d, X.stride(0), n_landmarks,
                                     None if lm is None else _P(lm.ctypes.data), seed, noise_rel, mode, scal,
                                     m0, ctypes.byref(prm), _P(idx.data_ptr()), ctypes.byref(res),
                                     ctypes.byref(st), _P(ex.ctypes.data)), "lap_full_solve")
    r = _res(res)
    stats = {f: getattr(st, f) for f, _ in apx_lap_stats._fields_ if f != "pad"}
    return idx, r, ex[: r.n_exemplars].copy(), stats


# --------------------------------------------------------------------------
# Learned warm start
# --------------------------------------------------------------------------
def _vec(t: torch.Tensor, name: str, numel: int | None = None, dtype=torch.float32):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return _P(t.data_ptr())


def apx_features(S: torch.Tensor, F: torch.Tensor | None = None, sigma: torch.Tensor | None = None):
    """Per-point features (n, 16) of S and the scale sigma (1-element tensor)."""
    Sp, n, ld = _mat(S, "S")
    if F is None:
        F = torch.empty((n, APX_MLP_FEATURES), dtype=torch.float32, device=S.device)
    if sigma is None:
        sigma = torch.empty(1, dtype=torch.float32, device=S.device)
    ctx = context(S.device)
    _check(ctx, lib().apx_features(ctx, Sp, n, ld, _vec(F, "F", n * APX_MLP_FEATURES),
                                   _vec(sigma, "sigma", 1)), "apx_features")
    return F, sigma


def apx_mlp_forward(theta: torch.Tensor, F: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
    """Network outputs (count, 2) for features F (count, 16)."""
    count = F.shape[0]
    if Y is None:
        Y = torch.empty((count, 2), dtype=torch.float32, device=F.device)
    ctx = context(F.device)
    _check(ctx, lib().apx_mlp_forward(ctx, _vec(theta, "theta", APX_MLP_PARAMS),
                                      _vec(F, "F", count * APX_MLP_FEATURES), count,
                                      _vec(Y, "Y", count * 2)), "apx_mlp_forward")
    return Y


def apx_mlp_backward(theta, F, T, w, rows: torch.Tensor | None = None, grad=None, loss=None):
    """Gradient of the weighted Huber loss over the batch; returns (grad, loss tensor)."""
    total = F.shape[0]
    count = total if rows is None else rows.numel()
    if grad is None:
        grad = torch.empty(APX_MLP_PARAMS, dtype=torch.float32, device=F.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=F.device)
    rp = None if rows is None else _vec(rows, "rows", dtype=torch.int64)
    ctx = context(F.device)
    _check(ctx, lib().apx_mlp_backward(ctx, _vec(theta, "theta", APX_MLP_PARAMS),
                                       _vec(F, "F", total * APX_MLP_FEATURES), _vec(T, "T", total * 2),
                                       _vec(w, "w", total), rp, count, _vec(grad, "grad", APX_MLP_PARAMS),
                                       _vec(loss, "loss", 1, torch.float64)), "apx_mlp_backward")
    return grad, loss


def apx_mlp_adam(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8) -> None:
    """One Adam step on theta in place (moments m, v updated in place)."""
    count = theta.numel()
    ctx = context(theta.device)
    _check(ctx, lib().apx_mlp_adam(ctx, _vec(theta, "theta"), _vec(m, "m", count), _vec(v, "v", count),
                                   _vec(grad, "grad", count), count, step, lr, beta1, beta2, eps),
           "apx_mlp_adam")


def apx_targets(R: torch.Tensor, sigma: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
    """Training targets (n, 2) = (t_k, c_k) / sigma from converged responsibilities."""
    Rp, n, ld = _mat(R, "R")
    if Y is None:
        Y = torch.empty((n, 2), dtype=torch.float32, device=R.device)
    ctx = context(R.device)
    _check(ctx, lib().apx_targets(ctx, Rp, n, ld, _vec(sigma, "sigma", 1), _vec(Y, "Y", n * 2)),
           "apx_targets")
    return Y


def apx_warm_a0(Y: torch.Tensor, sigma: torch.Tensor, A: torch.Tensor) -> torch.Tensor:
    """A_0 from predictions Y (n, 2) into A."""
    Ap, n, ld = _mat(A, "A")
    ctx = context(A.device)
    _check(ctx, lib().apx_warm_a0(ctx, _vec(Y, "Y", n * 2), _vec(sigma, "sigma", 1), n, Ap, ld),
           "apx_warm_a0")
    return A


def ap_warmstart(S: torch.Tensor, theta: torch.Tensor, R: torch.Tensor, A: torch.Tensor,
                 sigma: torch.Tensor | None = None):
    """Predicted (R_0, A_0) for ap_solve(..., warm=APX_WARM_AR), or A_0 alone for
    warm=APX_WARM_COLUMNS (column-structured; the solve forms R_0); returns sigma."""
    Sp, n, ld = _mat(S, "S")
    Rp, _, ldr = _mat(R, "R", n)
    Ap, _, lda = _mat(A, "A", n)
    if not (ld == ldr == lda):
        raise ValueError("S, R and A must share one leading dimension")
    if sigma is None:
        sigma = torch.empty(1, dtype=torch.float32, device=S.device)
    ctx = context(S.device)
    _check(ctx, lib().ap_warmstart(ctx, Sp, n, ld, _vec(theta, "theta", APX_MLP_PARAMS), Rp, Ap,
                                   _vec(sigma, "sigma", 1)), "ap_warmstart")
    return sigma

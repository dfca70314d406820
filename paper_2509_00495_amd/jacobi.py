"""Python binding of libjacobi (ctypes).

Argument marshalling only: every step of the solver runs in the HIP kernels
of libjacobi.so.  Tensors must be CUDA (ROCm) float64 tensors; the library
works on the current torch stream and uses torch only for device memory.
There is no CPU fallback: without the built library or a GPU these functions
raise.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjacobi.so")
HEADER = os.path.join(_HERE, "..", "include", "jacobi.h")

OK, NOCONV, NOTSYM, NONFINITE, DEGENERATE, DEVICE, WORKSPACE = range(7)


class JacobiError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        msg = _lib().jacobi_status_string(status).decode()
        if status == DEVICE:
            msg += ": " + _lib().jacobi_last_hip_error().decode()
        super().__init__(f"{fn} returned {status} ({msg})")


class Opts(ctypes.Structure):
    _fields_ = [
        ("max_sweeps", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("inner_sweeps", ctypes.c_int32),
        ("ns_iters", ctypes.c_int32),
        ("c32", ctypes.c_double),
        ("check_symmetry", ctypes.c_int32),
        ("small_max_n", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("serial_v", ctypes.c_int32),
        ("tune", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("no_pair_skip", ctypes.c_int32),
        ("gemm_slots", ctypes.c_int32),
        ("pair_v_split", ctypes.c_int32),
        ("orth", ctypes.c_int32),
        ("ladder", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int32),
        ("sweeps32", ctypes.c_int32),
        ("ns_iters", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("polished", ctypes.c_int32),
        ("skipped_tiles", ctypes.c_int32),
        ("sweeps16", ctypes.c_int32),
        ("norm_f", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("off_final", ctypes.c_double),
        ("off32", ctypes.c_double),
        ("off_cond", ctypes.c_double),
        ("orth_ns", ctypes.c_double),
        ("orth_est", ctypes.c_double),
        ("t_pair_ms", ctypes.c_double * 2),
        ("t_apply_ms", ctypes.c_double * 2),
        ("t_applyv_ms", ctypes.c_double * 2),
        ("n_pair", ctypes.c_int32 * 2),
        ("n_apply", ctypes.c_int32 * 2),
        ("n_applyv", ctypes.c_int32 * 2),
        ("reserved_i2", ctypes.c_int32 * 2),
        ("orth_qd", ctypes.c_double),
        ("t_orth_ms", ctypes.c_double),
        ("off16", ctypes.c_double),
        ("orth_ql", ctypes.c_double),
    ]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            if k.startswith("reserved"):
                continue
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2509_00495_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        P, i64, d, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        eigh_args = [P, i64, i64, P, P, i64, d, ctypes.POINTER(Opts), P,
                     ctypes.c_size_t, P, ctypes.POINTER(Info)]
        lib.jacobi_eigh.argtypes = eigh_args
        lib.jacobi_eigh.restype = i32
        lib.jacobi_eigh_mixed.argtypes = eigh_args
        lib.jacobi_eigh_mixed.restype = i32
        lib.jacobi_eigh_batched.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), i64,
                                            P, ctypes.POINTER(i64), P, d, i32,
                                            ctypes.POINTER(Opts), P, ctypes.c_size_t, P, P]
        lib.jacobi_eigh_batched.restype = i32
        lib.jacobi_eigh_batched_noalloc.argtypes = [P, ctypes.POINTER(i64),
                                                    ctypes.POINTER(i64), i64, P,
                                                    ctypes.POINTER(i64), P, d, i32,
                                                    ctypes.POINTER(Opts), P, P]
        lib.jacobi_eigh_batched_noalloc.restype = i32
        lib.jacobi_eigh_backward.argtypes = [P, P, P, P, i64, i64, i64, P, d, P,
                                             ctypes.c_size_t, P]
        lib.jacobi_eigh_backward.restype = i32
        lib.jacobi_workspace_bytes.argtypes = [i32, i64, i64, ctypes.POINTER(Opts)]
        lib.jacobi_workspace_bytes.restype = ctypes.c_size_t
        lib.jacobi_status_string.argtypes = [i32]
        lib.jacobi_status_string.restype = ctypes.c_char_p
        lib.jacobi_version.restype = ctypes.c_char_p
        lib.jacobi_last_hip_error.restype = ctypes.c_char_p
        lib.jacobi_device_summary.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        lib.jacobi_device_summary.restype = i32
        _LIB = lib
    return _LIB


def declared_functions():
    """Names of the functions declared in include/jacobi.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(jacobi_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


def make_opts(**kw) -> Opts:
    o = Opts()
    for k, v in kw.items():
        if v is None:
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def workspace_bytes(op: int, n_max: int, batch: int = 1, opts: Opts | None = None) -> int:
    return int(_lib().jacobi_workspace_bytes(op, n_max, batch,
                                             ctypes.byref(opts) if opts else None))


def device_summary() -> str:
    buf = ctypes.create_string_buffer(512)
    st = _lib().jacobi_device_summary(buf, 512)
    if st:
        raise JacobiError("jacobi_device_summary", st)
    return buf.value.decode()


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libjacobi needs a ROCm GPU; torch.cuda is not available")
    return torch


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_square(A):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"A must be square, got shape {tuple(A.shape)}")
    if A.dtype != __import__("torch").float64:
        raise TypeError("A must be float64")
    if not A.is_cuda:
        raise TypeError("A must be a GPU tensor")


@dataclass
class Workspace:
    """Reusable device scratch (a torch uint8 tensor)."""
    buf: object = None

    def get(self, nbytes: int):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self.buf


_default_ws = Workspace()


def _eigh_impl(fn_name, op, A, tol, opts, ws, check, return_info):
    torch = _torch()
    _check_square(A)
    if A.stride(1) != 1:
        A = A.contiguous()
    n = A.shape[0]
    lda = max(A.stride(0), 1) if n else 1
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    V = torch.empty((n, n), dtype=torch.float64, device=A.device)
    o = opts or Opts()
    need = workspace_bytes(op, n, 1, o)
    buf = (ws or _default_ws).get(need)
    info = Info()
    st = getattr(_lib(), fn_name)(
        A.data_ptr(), n, lda, W.data_ptr(), V.data_ptr(), max(n, 1),
        float(tol or 0.0), ctypes.byref(o), buf.data_ptr(), buf.numel(), _stream(torch),
        ctypes.byref(info))
    if st != OK and (check or st not in (NOCONV,)):
        raise JacobiError(fn_name, st)
    if return_info:
        d = info.as_dict()
        d["status"] = st
        return W, V, d
    return W, V


def eigh(A, tol: float | None = None, opts: Opts | None = None, ws: Workspace | None = None,
         check: bool = True, return_info: bool = False):
    """Plain FP64 Jacobi: (W ascending, V) with A = V diag(W) V^T."""
    return _eigh_impl("jacobi_eigh", 0, A, tol, opts, ws, check, return_info)


def eigh_mixed(A, tol: float | None = None, opts: Opts | None = None,
               ws: Workspace | None = None, check: bool = True, return_info: bool = False):
    """Mixed precision (FP32 Jacobi -> Newton-Schulz -> FP64 Jacobi)."""
    return _eigh_impl("jacobi_eigh_mixed", 1, A, tol, opts, ws, check, return_info)


def eigh_batched(A_packed, ns, tol: float | None = None, opts: Opts | None = None,
                 ws: Workspace | None = None, check: bool = True, out=None, a_off=None,
                 w_off=None):
    """jacobi_eigh_batched: a batch of uneven orders <= 128 in one persistent
    launch, or a batch of one order above 128 on the block path (one launch
    per step for the whole batch; each result bitwise that of eigh on the
    matrix).  A_packed: 1-D float64 GPU tensor holding the matrices
    (row-major, ld = n_i), back to back or at the element offsets a_off (host
    ints); eigenvalues go back to back or to w_off.  Returns (W, V, status):
    V has A_packed's layout, status is an int32 GPU tensor of per-matrix
    codes.  `out` = (W, V, status) reuses caller tensors (fixed addresses,
    which a graph replay with opts.graph needs)."""
    torch = _torch()
    ns = [int(x) for x in ns]
    batch = len(ns)
    if A_packed.dtype != torch.float64 or not A_packed.is_cuda:
        raise TypeError("A_packed must be a float64 GPU tensor")
    if a_off is None:
        tot = sum(x * x for x in ns)
        if A_packed.numel() != tot:
            raise ValueError(f"A_packed has {A_packed.numel()} entries, orders need {tot}")
    else:
        a_off = [int(x) for x in a_off]
        if len(a_off) != batch or any(o < 0 for o in a_off):
            raise ValueError("a_off needs one offset >= 0 per matrix")
        tot = A_packed.numel()
        if any(o + x * x > tot for o, x in zip(a_off, ns)):
            raise ValueError("a matrix extends past the end of A_packed")
    if w_off is None:
        wtot = sum(ns)
    else:
        w_off = [int(x) for x in w_off]
        if len(w_off) != batch or any(o < 0 for o in w_off):
            raise ValueError("w_off needs one offset >= 0 per matrix")
        wtot = max((o + x for o, x in zip(w_off, ns)), default=0)
    A_packed = A_packed.contiguous()
    if out is None:
        W = torch.empty(wtot, dtype=torch.float64, device=A_packed.device)
        V = torch.empty(tot, dtype=torch.float64, device=A_packed.device)
        status = torch.zeros(batch, dtype=torch.int32, device=A_packed.device)
    else:
        W, V, status = out
        for t, cnt, dt in ((W, wtot, torch.float64), (V, tot, torch.float64),
                           (status, batch, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != cnt:
                raise ValueError("out tensors must be contiguous GPU tensors of the packed sizes")
    o = opts or Opts()
    n_arr = (ctypes.c_int64 * max(batch, 1))(*ns)
    ao = None if a_off is None else (ctypes.c_int64 * max(batch, 1))(*a_off)
    wo = None if w_off is None else (ctypes.c_int64 * max(batch, 1))(*w_off)
    need = workspace_bytes(2, max(ns) if ns else 1, batch, o)
    buf = (ws or _default_ws).get(need)
    st = _lib().jacobi_eigh_batched(A_packed.data_ptr(), n_arr, ao, batch, W.data_ptr(),
                                    wo, V.data_ptr(), float(tol or 0.0), 0, ctypes.byref(o),
                                    buf.data_ptr(), buf.numel(), _stream(torch),
                                    status.data_ptr())
    if st < 0 or st in (DEVICE, WORKSPACE) or (check and st != OK):
        raise JacobiError("jacobi_eigh_batched", st)
    return W, V, status


def eigh_batched_noalloc(A_packed, ns, W, V, status, tol: float | None = None,
                         opts: Opts | None = None, a_off=None, w_off=None):
    """jacobi_eigh_batched_noalloc: the batched solve into caller tensors
    (W, V, status: contiguous GPU tensors of the packed or offset layout, as
    eigh_batched returns them) with the library's fixed device scratch; no
    workspace and no allocation.  Returns the call's status."""
    torch = _torch()
    ns = [int(x) for x in ns]
    batch = len(ns)
    for t in (A_packed, W, V):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError("A_packed, W and V must be contiguous float64 GPU tensors")
    if status.dtype != torch.int32 or not status.is_cuda or status.numel() != batch:
        raise TypeError("status must be an int32 GPU tensor with one entry per matrix")
    o = opts or Opts()
    n_arr = (ctypes.c_int64 * max(batch, 1))(*ns)
    ao = None if a_off is None else (ctypes.c_int64 * max(batch, 1))(*[int(x) for x in a_off])
    wo = None if w_off is None else (ctypes.c_int64 * max(batch, 1))(*[int(x) for x in w_off])
    return int(_lib().jacobi_eigh_batched_noalloc(
        A_packed.data_ptr(), n_arr, ao, batch, W.data_ptr(), wo, V.data_ptr(),
        float(tol or 0.0), 0, ctypes.byref(o), _stream(torch), status.data_ptr()))


def eigh_backward(W, V, dW=None, dV=None, gap_tol: float = 0.0, ws: Workspace | None = None,
                  return_status: bool = False):
    """dA = sym(V (diag(dW) + F o (V^T dV)) V^T) for (batch x) n x n inputs."""
    torch = _torch()
    squeeze = W.dim() == 1
    if squeeze:
        W, V = W[None], V[None]
        dW = None if dW is None else dW[None]
        dV = None if dV is None else dV[None]
    batch, n = W.shape
    if V.shape != (batch, n, n):
        raise ValueError("V must be batch x n x n")
    W = W.contiguous()
    V = V.contiguous()
    dW = None if dW is None else dW.contiguous()
    dV = None if dV is None else dV.contiguous()
    dA = torch.empty((batch, n, n), dtype=torch.float64, device=W.device)
    need = workspace_bytes(3, n, batch)
    buf = (ws or _default_ws).get(need)
    st = _lib().jacobi_eigh_backward(
        W.data_ptr(), V.data_ptr(), None if dW is None else dW.data_ptr(),
        None if dV is None else dV.data_ptr(), n, max(n, 1), batch, dA.data_ptr(), float(gap_tol),
        buf.data_ptr(), buf.numel(), _stream(torch))
    if st not in (OK, DEGENERATE):
        raise JacobiError("jacobi_eigh_backward", st)
    out = dA[0] if squeeze else dA
    return (out, st) if return_status else out


def _autograd():
    import torch

    class EighFn(torch.autograd.Function):
        """(W, V) = eigh(A) with the adjoint of jacobi_eigh_backward.  A is a
        (batch x) n x n float64 GPU tensor; a plain batch runs in one
        jacobi_eigh_batched call (one persistent launch for order <= 128, the
        block path with one launch per step for the whole batch above), a
        mixed batch per matrix."""

        @staticmethod
        def forward(ctx, A, mixed=False, tol=None):
            fn = eigh_mixed if mixed else eigh
            if A.dim() == 2:
                W, V = fn(A, tol)
            elif not mixed and A.shape[-1] >= 1:
                # one jacobi_eigh_batched call for the whole batch
                b, n = A.shape[0], A.shape[-1]
                Wp, Vp, _ = eigh_batched(A.contiguous().reshape(-1), [n] * b, tol)
                W = Wp.reshape(b, n)
                V = Vp.reshape(b, n, n)
            else:
                outs = [fn(A[k], tol) for k in range(A.shape[0])]
                W = torch.stack([o[0] for o in outs])
                V = torch.stack([o[1] for o in outs])
            ctx.save_for_backward(W, V)
            return W, V

        @staticmethod
        def backward(ctx, gW, gV):
            W, V = ctx.saved_tensors
            dA = eigh_backward(W, V, gW, gV)
            return dA, None, None

    return EighFn


_EighFn = None


def EighFn():
    global _EighFn
    if _EighFn is None:
        _EighFn = _autograd()
    return _EighFn


def eigh_autograd(A, mixed: bool = False, tol: float | None = None):
    return EighFn().apply(A, mixed, tol)

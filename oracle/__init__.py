"""CPU oracle (test infrastructure only).

Plain FP64 cyclic-by-row Jacobi and its companions, written in C in
``jacobi_oracle.c`` and loaded here through ctypes.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
GPU library never does, and the two share no code.

Every function takes and returns row-major numpy arrays.  The C calls release
the GIL, so a thread pool over matrices runs them in parallel.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U_D = 2.0 ** -53   # unit roundoff, double (Section 1.2 table)
U_L = 2.0 ** -24   # unit roundoff, single


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no BLAS, no OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        lib.orc_jacobi_pair.argtypes = [d, d, d, P, P]
        lib.orc_off.argtypes = [i64, P]
        lib.orc_off.restype = d
        lib.orc_rotate.argtypes = [i64, P, P, i64, i64, d, d]
        lib.orc_jacobi_cyclic.argtypes = [i64, P, P, d, d, i32, P, P, P]
        lib.orc_jacobi_cyclic.restype = i32
        lib.orc_jacobi_cyclic_f32.argtypes = [i64, P, P, d, d, i32, P, P, P]
        lib.orc_jacobi_cyclic_f32.restype = i32
        lib.orc_sort_signfix.argtypes = [i64, P, P, P]
        lib.orc_eigh.argtypes = [i64, P, P, P, d, i32, P, P]
        lib.orc_eigh.restype = i32
        lib.orc_newton_schulz.argtypes = [i64, P, i32]
        lib.orc_qtaq.argtypes = [i64, P, P, P]
        lib.orc_eigh_mixed.argtypes = [i64, P, P, P, d, i32, i32, d, i32, P]
        lib.orc_eigh_mixed.restype = i32
        lib.orc_jacobi_rows.argtypes = [i64, P, P, i64, i64, d]
        lib.orc_jacobi_rows.restype = i64
        lib.orc_eigh_backward.argtypes = [i64, P, P, P, P, d, P]
        lib.orc_eigh_backward.restype = i32
        lib.orc_rayleigh.argtypes = [i64, P, P, P, P]
        lib.orc_round_half.argtypes = [d]
        lib.orc_round_half.restype = d
        lib.orc_jacobi_cyclic_h.argtypes = [i64, P, P, d, d, d, i32, P, P]
        lib.orc_jacobi_cyclic_h.restype = i32
        lib.orc_ns_iterations.argtypes = [d, d, d]
        lib.orc_ns_iterations.restype = i32
        lib.orc_house.argtypes = [i64, P, P, P]
        lib.orc_householder_qr.argtypes = [i64, P, P, P]
        lib.orc_cholesky.argtypes = [i64, P, P]
        lib.orc_cholesky.restype = i32
        lib.orc_cholesky_qr.argtypes = [i64, P, P, P]
        lib.orc_cholesky_qr.restype = i32
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data


def jacobi_pair(app: float, aqq: float, apq: float):
    """(c, s) of Algorithm 2 with approach 2 of Appendix A."""
    c, s = ctypes.c_double(), ctypes.c_double()
    _load().orc_jacobi_pair(app, aqq, apq, ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def off(A) -> float:
    A = _f64(A)
    return _load().orc_off(A.shape[0], _p(A))


def rotate(A, V, p: int, q: int, c: float, s: float):
    """One rotation on copies of A (and V); returns the new arrays."""
    A = _f64(A).copy()
    V = None if V is None else _f64(V).copy()
    _load().orc_rotate(A.shape[0], _p(A), _p(V), p, q, c, s)
    return A, V


def jacobi_cyclic(A, tol_abs: float, rel_eps: float = U_D,
                  max_sweeps: int = 30, V0=None):
    """Algorithm 4 on a copy of A.  Returns (A_final, V, sweeps, status,
    off_history, rotations)."""
    A = _f64(A).copy()
    n = A.shape[0]
    V = np.eye(n) if V0 is None else _f64(V0).copy()
    sw = ctypes.c_int()
    rot = ctypes.c_int64()
    hist = np.zeros(max_sweeps + 1)
    st = _load().orc_jacobi_cyclic(n, _p(A), _p(V), tol_abs, rel_eps,
                                   max_sweeps, ctypes.byref(sw), _p(hist),
                                   ctypes.byref(rot))
    return A, V, sw.value, st, hist[: sw.value + 1].copy(), rot.value


def jacobi_rows(A, V, p_begin: int, p_end: int, rel_eps: float = U_D) -> int:
    """Pivot rows [p_begin, p_end) of one cyclic-by-row sweep, in place on
    the float64 C-contiguous arrays A and V.  Returns the rotations made."""
    assert A.dtype == np.float64 and A.flags.c_contiguous
    assert V.dtype == np.float64 and V.flags.c_contiguous
    return int(_load().orc_jacobi_rows(A.shape[0], _p(A), _p(V), p_begin, p_end, rel_eps))


def jacobi_cyclic_f32(A, tol_abs: float, rel_eps: float = U_L,
                      max_sweeps: int = 30):
    A = np.ascontiguousarray(A, dtype=np.float32).copy()
    n = A.shape[0]
    V = np.eye(n, dtype=np.float32)
    sw = ctypes.c_int()
    hist = np.zeros(max_sweeps + 1)
    st = _load().orc_jacobi_cyclic_f32(n, _p(A), _p(V), tol_abs, rel_eps,
                                       max_sweeps, ctypes.byref(sw), _p(hist),
                                       None)
    return A, V, sw.value, st, hist[: sw.value + 1].copy()


def default_tol(A) -> float:
    """1e-15 n ||A||_F, the FP64 stopping threshold on off(B)."""
    A = np.asarray(A)
    return 1e-15 * A.shape[0] * float(np.linalg.norm(A))


def eigh(A, tol: float | None = None, max_sweeps: int = 30):
    """Plain FP64 Jacobi eigendecomposition.  Returns (W, V, sweeps, status,
    off_history)."""
    A = _f64(A)
    n = A.shape[0]
    tol = default_tol(A) if tol is None or tol <= 0 else tol
    W = np.zeros(n)
    V = np.zeros((n, n))
    sw = ctypes.c_int()
    hist = np.zeros(max_sweeps + 1)
    st = _load().orc_eigh(n, _p(A), _p(W), _p(V), tol, max_sweeps,
                          ctypes.byref(sw), _p(hist))
    return W, V, sw.value, st, hist[: sw.value + 1].copy()


def sort_signfix(D, V):
    D = _f64(D)
    V = _f64(V).copy()
    W = np.zeros_like(D)
    _load().orc_sort_signfix(D.shape[0], _p(D), _p(V), _p(W))
    return W, V


def newton_schulz(X, iters: int = 2):
    X = _f64(X).copy()
    _load().orc_newton_schulz(X.shape[0], _p(X), iters)
    return X


def qtaq(Q, A):
    Q, A = _f64(Q), _f64(A)
    B = np.zeros_like(A)
    _load().orc_qtaq(A.shape[0], _p(Q), _p(A), _p(B))
    return B


ORTH = {"ns": 0, "householder": 1, "cholesky": 2}


def eigh_mixed(A, tol: float | None = None, max_sweeps: int = 30,
               ns_iters: int = 2, c32: float = 1.0, orth: str = "ns"):
    """Algorithm 9 with an FP32 Jacobi first stage; Q_l -> Q_d by Newton-Schulz
    (orth="ns"), Householder QR or Cholesky QR.  Returns (W, Q, status, diag)
    with diag = dict(sweeps32, sweeps64, orth_ql, orth_qd, off_cond)."""
    A = _f64(A)
    n = A.shape[0]
    tol = default_tol(A) if tol is None or tol <= 0 else tol
    W = np.zeros(n)
    Q = np.zeros((n, n))
    dg = np.zeros(6)
    st = _load().orc_eigh_mixed(n, _p(A), _p(W), _p(Q), tol, max_sweeps,
                                ns_iters, c32, ORTH[orth], _p(dg))
    return W, Q, st, dict(sweeps32=int(dg[0]), sweeps64=int(dg[1]),
                          orth_ql=dg[2], orth_qd=dg[3], off_cond=dg[4],
                          status32=int(dg[5]))


def rayleigh(A, V):
    """Rayleigh quotients and residual norms of the columns of V against A:
    rq_k = v_k^T A v_k / v_k^T v_k, res_k = ||A v_k - rq_k v_k|| / ||v_k||."""
    A, V = _f64(A), _f64(V)
    n = A.shape[0]
    rq = np.zeros(n)
    res = np.zeros(n)
    _load().orc_rayleigh(n, _p(A), _p(V), _p(rq), _p(res))
    return rq, res


U_H = 2.0 ** -11  # unit roundoff, binary16


def round_half(x: float) -> float:
    """x rounded to the nearest binary16 value (ties to even)."""
    return _load().orc_round_half(float(x))


def jacobi_cyclic_h(A, tol_abs: float = 0.0, rel_eps: float = U_H, stall: float = 0.9,
                    max_sweeps: int = 30, V0=None):
    """The binary16 stage: Algorithm 4 with A stored in binary16 (every update
    rounded), float angles and float V.  A is rounded to binary16 first.
    Returns (A_final, V, sweeps, status, off_history)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    Ah = np.array([[round_half(v) for v in row] for row in A], dtype=np.float32) \
        if n <= 64 else _round_half_array(A)
    V = np.eye(n, dtype=np.float32) if V0 is None else np.ascontiguousarray(V0, np.float32).copy()
    sw = ctypes.c_int()
    hist = np.zeros(max_sweeps + 1)
    st = _load().orc_jacobi_cyclic_h(n, _p(Ah), _p(V), tol_abs, rel_eps, stall, max_sweeps,
                                     ctypes.byref(sw), _p(hist))
    return Ah, V, sw.value, st, hist[: sw.value + 1].copy()


def _round_half_array(A):
    f = np.vectorize(round_half, otypes=[np.float64])
    return f(A).astype(np.float32)


def ns_iterations(n: float, u_low: float, u_high: float = U_D) -> int:
    """Newton-Schulz iterations for low-precision vectors with unit roundoff
    u_low (Section 4.3.4 analysis); -1 when n u_low >= 2."""
    return int(_load().orc_ns_iterations(float(n), float(u_low), float(u_high)))


def house(x):
    """Householder vector and coefficient of Algorithm 1: (v, beta) with
    (I - beta v v^T) x = -sign(x_1) ||x|| e_1."""
    x = _f64(x)
    v = np.zeros_like(x)
    b = ctypes.c_double()
    _load().orc_house(x.shape[0], _p(x), _p(v), ctypes.byref(b))
    return v, b.value


def householder_qr(A):
    """Algorithm 5: (Q, R) with A = Q R."""
    A = _f64(A).copy()
    n = A.shape[0]
    Q = np.zeros((n, n))
    R = np.zeros((n, n))
    _load().orc_householder_qr(n, _p(A), _p(Q), _p(R))
    return Q, R


def cholesky(G):
    """Upper R with G = R^T R.  Returns (R, status)."""
    G = _f64(G)
    R = np.zeros_like(G)
    st = _load().orc_cholesky(G.shape[0], _p(G), _p(R))
    return R, st


def cholesky_qr(X):
    """Cholesky QR: (Q, R, status) with X = Q R."""
    X = _f64(X)
    n = X.shape[0]
    Q = np.zeros((n, n))
    R = np.zeros((n, n))
    st = _load().orc_cholesky_qr(n, _p(X), _p(Q), _p(R))
    return Q, R, st


def eigh_backward(W, V, dW=None, dV=None, gap_tol: float = 0.0):
    """dA = sym(V (diag(dW) + F o (V^T dV)) V^T), F_ij = 1/(W_j - W_i).
    Returns (dA, status)."""
    W, V = _f64(W), _f64(V)
    n = W.shape[0]
    dW = None if dW is None else _f64(dW)
    dV = None if dV is None else _f64(dV)
    dA = np.zeros((n, n))
    st = _load().orc_eigh_backward(n, _p(W), _p(V), _p(dW), _p(dV), gap_tol,
                                   _p(dA))
    return dA, st

"""CPU oracle for the batched small dense solvers (test infrastructure only).

What it computes follows the Fig. 2 caption of the paper: the upper Cholesky
factor X^T X = A, the triangular Sylvester solution of L X + X U = C and the
triangular Lyapunov solution of L X + X L^T = S, in FP64, by plain element
recurrences (``tla_oracle.c``), plus brute-force Kronecker solves, backward
error measures, a mixed-precision refinement model, and (``mlp_ref``) an FP64
reference of the small MLP cost model.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never loads it and shares no code
with it.

Matrices are numpy arrays of shape (n, n) or (batch, n, n), indexed [i, j]
as in the paper; they are handed to C in column-major order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tla_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

# flag bits of the refinement model
CONVERGED, FALLBACK, BREAKDOWN, NONFINITE = 1, 2, 4, 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        sig = {
            "orc_potrf": (c_int, [c_int, D, c_int, D, c_int]),
            "orc_trsyl": (c_int, [c_int, D, c_int, D, c_int, D, c_int, D, c_int]),
            "orc_trlyap": (c_int, [c_int, D, c_int, D, c_int, D, c_int]),
            "orc_gepp": (c_int, [c_int, D, D]),
            "orc_kron_sylv": (c_int, [c_int, D, c_int, D, c_int, D, c_int, D, c_int, D]),
            "orc_kron_lyap": (c_int, [c_int, D, c_int, D, c_int, D, c_int, D]),
            "orc_eta_potrf": (c_double, [c_int, D, c_int, D, c_int]),
            "orc_eta_trsyl": (c_double, [c_int, D, c_int, D, c_int, D, c_int, D, c_int]),
            "orc_eta_trlyap": (c_double, [c_int, D, c_int, D, c_int, D, c_int]),
            "orc_potrf_batch": (None, [c_int, c_int, D, D, I, c_int]),
            "orc_potrs": (c_int, [c_int, c_int, D, c_int, D, c_int]),
            "orc_potrs_batch": (None, [c_int, c_int, c_int, D, D, I, c_int]),
            "orc_potri": (c_int, [c_int, D, c_int, D, c_int]),
            "orc_potri_batch": (None, [c_int, c_int, D, D, I, c_int]),
            "orc_trsyl_batch": (None, [c_int, c_int, D, D, D, D, I, c_int]),
            "orc_trlyap_batch": (None, [c_int, c_int, D, D, D, I, c_int]),
            "orc_eta_potrf_batch": (None, [c_int, c_int, D, D, D, c_int]),
            "orc_eta_trsyl_batch": (None, [c_int, c_int, D, D, D, D, D, c_int]),
            "orc_eta_trlyap_batch": (None, [c_int, c_int, D, D, D, D, c_int]),
            "orc_refine": (c_int, [c_int, c_int, D, D, D, D, c_int, c_double, I, I, D]),
            "orc_max_threads": (c_int, []),
            "orc_kron_gesyl": (c_int, [c_int, D, c_int, D, c_int, D, c_int, D, c_int, D]),
            "orc_kron_gelyap": (c_int, [c_int, D, c_int, D, c_int, D, c_int, D]),
            "orc_eta_gesyl": (c_double, [c_int, D, c_int, D, c_int, D, c_int, D, c_int]),
            "orc_eta_gelyap": (c_double, [c_int, D, c_int, D, c_int, D, c_int]),
            "orc_kron_gesyl_batch": (None, [c_int, c_int, D, D, D, D, I, c_int]),
            "orc_kron_gelyap_batch": (None, [c_int, c_int, D, D, D, I, c_int]),
            "orc_eta_gesyl_batch": (None, [c_int, c_int, D, D, D, D, D, c_int]),
            "orc_eta_gelyap_batch": (None, [c_int, c_int, D, D, D, D, c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _cm(a):
    """Column-major FP64 copy of a (n, n) or (batch, n, n) array."""
    a = np.asarray(a, dtype=np.float64)
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _from_cm(a):
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


def max_threads() -> int:
    return lib().orc_max_threads()


# ---------------------------------------------------------------- single solves
def potrf(A):
    """Upper Cholesky factor X (X^T X = A) from the upper triangle of A -> (X, info)."""
    n = A.shape[-1]
    a = _cm(A)
    x = np.zeros_like(a)
    info = lib().orc_potrf(n, _dp(a), n, _dp(x), n)
    return _from_cm(x), info


def potrs(X, B):
    """A^{-1} B for A = X^T X, from the upper triangle of the factor X; B is (n, m) -> (Y, info)."""
    n, m = B.shape
    x = _cm(X)
    y = _cm(B).copy()   # the solve overwrites it; never the caller's array
    info = lib().orc_potrs(n, m, _dp(x), n, _dp(y), n)
    return _from_cm(y), info


def potri(X):
    """(X^T X)^{-1}, full n x n, from the upper triangle of the factor X -> (Ainv, info)."""
    n = X.shape[-1]
    x = _cm(X)
    y = np.zeros_like(x)
    info = lib().orc_potri(n, _dp(x), n, _dp(y), n)
    return _from_cm(y), info


def trsyl(L, U, C):
    """Solution X of L X + X U = C (L lower, U upper) -> (X, info)."""
    n = C.shape[-1]
    l, u, c = _cm(L), _cm(U), _cm(C)
    x = np.zeros_like(c)
    info = lib().orc_trsyl(n, _dp(l), n, _dp(u), n, _dp(c), n, _dp(x), n)
    return _from_cm(x), info


def trlyap(L, S):
    """Symmetric solution X of L X + X L^T = S (lower triangles of L, S read) -> (X, info)."""
    n = S.shape[-1]
    l, s = _cm(L), _cm(S)
    x = np.zeros_like(s)
    info = lib().orc_trlyap(n, _dp(l), n, _dp(s), n, _dp(x), n)
    return _from_cm(x), info


def kron_sylv(L, U, C):
    """Brute force: dense GEPP on (I (x) L + U^T (x) I) vec X = vec C."""
    n = C.shape[-1]
    l, u, c = _cm(L), _cm(U), _cm(C)
    x = np.zeros_like(c)
    w = np.zeros(n ** 4 + n ** 2)
    st = lib().orc_kron_sylv(n, _dp(l), n, _dp(u), n, _dp(c), n, _dp(x), n, _dp(w))
    return _from_cm(x), st


def kron_lyap(L, S):
    """Brute force: dense GEPP on (I (x) L + L (x) I) vec X = vec S."""
    n = S.shape[-1]
    l, s = _cm(L), _cm(S)
    x = np.zeros_like(s)
    w = np.zeros(n ** 4 + n ** 2)
    st = lib().orc_kron_lyap(n, _dp(l), n, _dp(s), n, _dp(x), n, _dp(w))
    return _from_cm(x), st


def gepp(M, r):
    """Dense Gaussian elimination with partial pivoting: solve M y = r."""
    m = M.shape[0]
    mm = _cm(M)
    rr = np.array(r, dtype=np.float64, copy=True)
    st = lib().orc_gepp(m, _dp(mm), _dp(rr))
    return rr, st


def eta_potrf(A, X):
    n = A.shape[-1]
    a, x = _cm(A), _cm(X)
    return lib().orc_eta_potrf(n, _dp(a), n, _dp(x), n)


def eta_trsyl(L, U, C, X):
    n = C.shape[-1]
    l, u, c, x = _cm(L), _cm(U), _cm(C), _cm(X)
    return lib().orc_eta_trsyl(n, _dp(l), n, _dp(u), n, _dp(c), n, _dp(x), n)


def eta_trlyap(L, S, X):
    n = S.shape[-1]
    l, s, x = _cm(L), _cm(S), _cm(X)
    return lib().orc_eta_trlyap(n, _dp(l), n, _dp(s), n, _dp(x), n)


def refine(op, A, B=None, C=None, max_iter=8, tau=1e-13):
    """Mixed-precision model: op 0 potrf(A), 1 trsyl(L=A, U=B, C), 2 trlyap(L=A, S=C).
    Returns (X, info, iters, flags, eta)."""
    n = A.shape[-1]
    a = _cm(A)
    b = _cm(B) if B is not None else np.zeros_like(a)
    c = _cm(C) if C is not None else np.zeros_like(a)
    x = np.zeros_like(a)
    it, fl, eta = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
    info = lib().orc_refine(op, n, _dp(a), _dp(b), _dp(c), _dp(x), max_iter, tau,
                            ctypes.byref(it), ctypes.byref(fl), ctypes.byref(eta))
    return _from_cm(x), info, it.value, fl.value, eta.value


# ------------------------------------------------------------- batched solves
def potrf_batch(A, threads=0):
    b, n = A.shape[0], A.shape[-1]
    a = _cm(A)
    x = np.empty_like(a)
    info = np.zeros(b, dtype=np.int32)
    lib().orc_potrf_batch(b, n, _dp(a), _dp(x), _ip(info), threads)
    return _from_cm(x), info


def potrs_batch(X, B, threads=0):
    """Batched potrs: X (batch, n, n) upper factors, B (batch, n, m) -> (Y, info)."""
    b, n, m = B.shape
    x = _cm(X)
    y = _cm(B).copy()   # the solve overwrites it; never the caller's array
    info = np.zeros(b, dtype=np.int32)
    lib().orc_potrs_batch(b, n, m, _dp(x), _dp(y), _ip(info), threads)
    return _from_cm(y), info


def potri_batch(X, threads=0):
    b, n = X.shape[0], X.shape[-1]
    x = _cm(X)
    y = np.zeros_like(x)
    info = np.zeros(b, dtype=np.int32)
    lib().orc_potri_batch(b, n, _dp(x), _dp(y), _ip(info), threads)
    return _from_cm(y), info


def trsyl_batch(L, U, C, threads=0):
    b, n = C.shape[0], C.shape[-1]
    l, u, c = _cm(L), _cm(U), _cm(C)
    x = np.empty_like(c)
    info = np.zeros(b, dtype=np.int32)
    lib().orc_trsyl_batch(b, n, _dp(l), _dp(u), _dp(c), _dp(x), _ip(info), threads)
    return _from_cm(x), info


def trlyap_batch(L, S, threads=0):
    b, n = S.shape[0], S.shape[-1]
    l, s = _cm(L), _cm(S)
    x = np.empty_like(s)
    info = np.zeros(b, dtype=np.int32)
    lib().orc_trlyap_batch(b, n, _dp(l), _dp(s), _dp(x), _ip(info), threads)
    return _from_cm(x), info


def eta_potrf_batch(A, X, threads=0):
    b, n = A.shape[0], A.shape[-1]
    a, x = _cm(A), _cm(X)
    eta = np.zeros(b)
    lib().orc_eta_potrf_batch(b, n, _dp(a), _dp(x), _dp(eta), threads)
    return eta


def eta_trsyl_batch(L, U, C, X, threads=0):
    b, n = C.shape[0], C.shape[-1]
    l, u, c, x = _cm(L), _cm(U), _cm(C), _cm(X)
    eta = np.zeros(b)
    lib().orc_eta_trsyl_batch(b, n, _dp(l), _dp(u), _dp(c), _dp(x), _dp(eta), threads)
    return eta


def eta_trlyap_batch(L, S, X, threads=0):
    b, n = S.shape[0], S.shape[-1]
    l, s, x = _cm(L), _cm(S), _cm(X)
    eta = np.zeros(b)
    lib().orc_eta_trlyap_batch(b, n, _dp(l), _dp(s), _dp(x), _dp(eta), threads)
    return eta


def forward_error(X, Xref):
    """||X - Xref||_F / ||Xref||_F per instance (last two axes)."""
    X = np.asarray(X, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    num = np.sqrt(((X - Xref) ** 2).sum(axis=(-1, -2)))
    den = np.sqrt((Xref ** 2).sum(axis=(-1, -2)))
    return num / np.where(den == 0, 1.0, den)


# ------------------------------------------------ general (non-triangular) equations
def gesyl(A, B, C):
    """General Sylvester A X + X B = C by its Kronecker system (dense GEPP)."""
    n = C.shape[-1]
    a, b, c = _cm(A), _cm(B), _cm(C)
    x = np.zeros_like(c)
    w = np.zeros(n ** 4 + n ** 2)
    st = lib().orc_kron_gesyl(n, _dp(a), n, _dp(b), n, _dp(c), n, _dp(x), n, _dp(w))
    return _from_cm(x), st


def gelyap(A, S):
    """General Lyapunov A X + X A^T = S (S by its lower triangle) by its Kronecker system."""
    n = S.shape[-1]
    a, s = _cm(A), _cm(S)
    x = np.zeros_like(s)
    w = np.zeros(n ** 4 + n ** 2)
    st = lib().orc_kron_gelyap(n, _dp(a), n, _dp(s), n, _dp(x), n, _dp(w))
    return _from_cm(x), st


def eta_gesyl(A, B, C, X):
    n = C.shape[-1]
    return lib().orc_eta_gesyl(n, _dp(_cm(A)), n, _dp(_cm(B)), n, _dp(_cm(C)), n, _dp(_cm(X)), n)


def eta_gelyap(A, S, X):
    n = S.shape[-1]
    return lib().orc_eta_gelyap(n, _dp(_cm(A)), n, _dp(_cm(S)), n, _dp(_cm(X)), n)


def gesyl_batch(A, B, C, threads=0):
    batch, n = C.shape[0], C.shape[-1]
    a, b, c = _cm(A), _cm(B), _cm(C)
    x = np.zeros_like(c)
    info = np.zeros(batch, dtype=np.int32)
    lib().orc_kron_gesyl_batch(batch, n, _dp(a), _dp(b), _dp(c), _dp(x), _ip(info), threads)
    return _from_cm(x), info


def gelyap_batch(A, S, threads=0):
    batch, n = S.shape[0], S.shape[-1]
    a, s = _cm(A), _cm(S)
    x = np.zeros_like(s)
    info = np.zeros(batch, dtype=np.int32)
    lib().orc_kron_gelyap_batch(batch, n, _dp(a), _dp(s), _dp(x), _ip(info), threads)
    return _from_cm(x), info


def eta_gesyl_batch(A, B, C, X, threads=0):
    batch, n = C.shape[0], C.shape[-1]
    eta = np.zeros(batch)
    lib().orc_eta_gesyl_batch(batch, n, _dp(_cm(A)), _dp(_cm(B)), _dp(_cm(C)), _dp(_cm(X)), _dp(eta), threads)
    return eta


def eta_gelyap_batch(A, S, X, threads=0):
    batch, n = S.shape[0], S.shape[-1]
    eta = np.zeros(batch)
    lib().orc_eta_gelyap_batch(batch, n, _dp(_cm(A)), _dp(_cm(S)), _dp(_cm(X)), _dp(eta), threads)
    return eta


"""ctypes loader of the oracle's plain C dense kernels (oracle/dense.c).

TEST INFRASTRUCTURE ONLY.  The shared object is built with gcc into
oracle/_build/ by build(); it is never linked into the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dense.c")
_OUT = os.path.join(_HERE, "_build", "liboracle_dense.so")
_RSRC = os.path.join(_HERE, "refine.c")
_ROUT = os.path.join(_HERE, "_build", "liboracle_refine.so")
_lib = None
_rlib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    for src, out, extra in ((_SRC, _OUT, ["-fopenmp", "-lm"]), (_RSRC, _ROUT, ["-lquadmath", "-lm"])):
        if force or not os.path.exists(out):
            tmp = out + f".tmp{os.getpid()}"
            cmd = ["gcc", "-O2", "-shared", "-fPIC", "-Wall", src, "-o", tmp]
            subprocess.check_call(cmd[:2] + [e for e in extra if e.startswith("-f")] + cmd[2:]
                                  + [e for e in extra if e.startswith("-l")])
            os.replace(tmp, out)
    return _OUT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_OUT):
            build(force=True)
        L = ctypes.CDLL(_OUT)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_cholesky.argtypes = [ctypes.c_int, dp]
        L.oracle_cholesky.restype = ctypes.c_int
        L.oracle_jacobi.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int]
        L.oracle_jacobi.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class NotSPD(ArithmeticError):
    pass


def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a dense SPD matrix (oracle_cholesky)."""
    L = np.array(A, dtype=np.float64, order="C", copy=True)
    n = L.shape[0]
    rc = lib().oracle_cholesky(n, _ptr(L))
    if rc != 0:
        raise NotSPD(f"non-positive pivot at row {-rc - 1} of {n}")
    return L


def jacobi_eigh(A: np.ndarray, max_sweeps: int = 60, abs_floor: float = 1e-18,
                threads: int = 0):
    """Eigenvalues (ascending) and eigenvectors (columns) by cyclic Jacobi (oracle_jacobi)."""
    a = np.array(A, dtype=np.float64, order="C", copy=True)
    a = 0.5 * (a + a.T)
    a = np.ascontiguousarray(a)
    n = a.shape[0]
    v = np.zeros((n, n))
    w = np.zeros(n)
    if threads <= 0:
        threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    rc = lib().oracle_jacobi(n, _ptr(a), _ptr(v), _ptr(w), max_sweeps, abs_floor, threads)
    if rc < 0:
        raise ArithmeticError("Jacobi did not converge")
    order = np.argsort(w, kind="stable")
    return w[order], v[:, order]


def rlib():
    global _rlib
    if _rlib is None:
        if not os.path.exists(_ROUT):
            build(force=True)
        L = ctypes.CDLL(_ROUT)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_refine.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, ip,
                                    ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp, dp]
        L.oracle_refine.restype = ctypes.c_int
        L.oracle_rayleigh.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp,
                                      ctypes.c_int, dp, dp]
        L.oracle_rayleigh.restype = ctypes.c_int
        _rlib = L
    return _rlib


def refine_pairs(eloc: np.ndarray, emat: np.ndarray, d: np.ndarray, X0: np.ndarray,
                 iters: int = 3, bmask: np.ndarray = None):
    """Binary128 Rayleigh-Ritz + subspace iteration of abar x = lambda D abar D x
    (oracle/refine.c).  eloc: (ne, k) local dof index or -1; emat: (ne, k, k);
    d: weights; X0: (n, kv) start vectors.  Returns (lam_hi, lam_lo, bound, cond, X),
    lambda ascending."""
    n, kv = X0.shape
    ne, kk = eloc.shape
    el = np.ascontiguousarray(eloc, dtype=np.int32)
    em = np.ascontiguousarray(emat, dtype=np.float64)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    x0 = np.asfortranarray(X0, dtype=np.float64)
    hi = np.zeros(kv)
    lo = np.zeros(kv)
    bd = np.zeros(kv)
    cd = np.zeros(kv)
    X = np.zeros((n, kv), order="F")
    ip = ctypes.POINTER(ctypes.c_int)
    bm = None if bmask is None else np.ascontiguousarray(bmask, dtype=np.int32)
    rc = rlib().oracle_refine(n, ne, kk, el.ctypes.data_as(ip), _ptr(em), _ptr(dd),
                              None if bm is None else bm.ctypes.data_as(ip), kv,
                              x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), iters,
                              _ptr(hi), _ptr(lo), _ptr(bd), _ptr(cd),
                              X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ArithmeticError(f"oracle_refine failed ({rc})")
    return hi, lo, bd, cd, np.array(X)


def rayleigh_exact(eloc: np.ndarray, emat: np.ndarray, d: np.ndarray, X: np.ndarray):
    """x^T abar x / x^T (D abar D) x in binary128 for each column of X (oracle/refine.c)."""
    n, kv = X.shape
    ne, kk = eloc.shape
    el = np.ascontiguousarray(eloc, dtype=np.int32)
    em = np.ascontiguousarray(emat, dtype=np.float64)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    x = np.asfortranarray(X, dtype=np.float64)
    lam = np.zeros(kv)
    ip = ctypes.POINTER(ctypes.c_int)
    rc = rlib().oracle_rayleigh(n, ne, kk, el.ctypes.data_as(ip), _ptr(em), _ptr(dd), kv,
                                x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(lam))
    if rc != 0:
        raise ArithmeticError(f"oracle_rayleigh failed ({rc})")
    return lam

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
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT):
        tmp = _OUT + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _OUT)
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

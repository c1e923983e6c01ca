"""Thin ctypes binding of libmsdd (include/msdd.h): argument marshalling only.

Arrays may be torch tensors (host or device; their data pointers are passed
through) or numpy arrays (host).  Every numerical step runs in the HIP library;
if it is not built this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; MSDD_LIB may name another build of the same sources (the host-code
# sanitizer build under _build_ubsan/)
LIB_PATH = os.environ.get("MSDD_LIB") or os.path.join(_HERE, "_build", "libmsdd.so")

MSDD_OK = 0
MSDD_EINVAL = -1
MSDD_ENOTSPD = -2
MSDD_EEIG = -3
MSDD_ENOCONV = -4
MSDD_EDEVICE = -5
MSDD_ENOMEM = -6
MSDD_ESTATE = -7
MSDD_FP64 = 0
MSDD_MIXED = 1

_ERRNAMES = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "EEIG", -4: "ENOCONV", -5: "EDEVICE",
             -6: "ENOMEM", -7: "ESTATE"}


class MsddOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("sigma", ctypes.c_double),
                ("eps_reg_rel", ctypes.c_double), ("nev_max", ctypes.c_int),
                ("eig_tol", ctypes.c_double), ("eig_maxit", ctypes.c_int),
                ("block", ctypes.c_int), ("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("verbose", ctypes.c_int), ("geneo_rhs", ctypes.c_int), ("nev_fixed", ctypes.c_int),
                ("eig_tol_energy", ctypes.c_double), ("dirichlet_rule", ctypes.c_int),
                ("eig_fp32", ctypes.c_int)]


class MsddStats(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("n", ctypes.c_int64 * 8),
                ("n_sub", ctypes.c_int32 * 8), ("m_max", ctypes.c_int32 * 8),
                ("max_local", ctypes.c_int32 * 8), ("max_band", ctypes.c_int32),
                ("eig_iters_max", ctypes.c_int32), ("eig_restarts", ctypes.c_int32),
                ("eig_resid_max", ctypes.c_double), ("t_plan_ms", ctypes.c_double),
                ("t_local_ms", ctypes.c_double), ("t_gevp_ms", ctypes.c_double),
                ("t_coarse_ms", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("pcg_iters", ctypes.c_int32),
                ("pcg_relres", ctypes.c_double), ("eig_iters_sum", ctypes.c_int64),
                ("warm_started", ctypes.c_int32), ("warm_fallbacks", ctypes.c_int32),
                ("eig_unconverged", ctypes.c_int32), ("eig_stagnated", ctypes.c_int32),
                ("eig_energy_resid_max", ctypes.c_double), ("eig_fp64_fallbacks", ctypes.c_int32)]

    def as_dict(self):
        L = self.n_levels
        d = {f: getattr(self, f) for f, _ in self._fields_}
        for f in ("n", "n_sub", "m_max", "max_local"):
            d[f] = list(getattr(self, f))[:L]
        return d


MSDD_TUNE_EIG = 1
MSDD_TUNE_SOLVE = 2


class MsddTuning(ctypes.Structure):
    _fields_ = [("eig_solve", ctypes.c_int32), ("eig_splits", ctypes.c_int32),
                ("fine_solve", ctypes.c_int32), ("spmv_group", ctypes.c_int32),
                ("eig_solve_ms", ctypes.c_float * 10), ("eig_splits_ms", ctypes.c_float * 5),
                ("fine_solve_ms", ctypes.c_float * 4), ("spmv_ms", ctypes.c_float * 4)]

    def as_dict(self):
        return {f: (list(getattr(self, f)) if f.endswith("_ms") else getattr(self, f))
                for f, _ in self._fields_}


EXPORTS = ["msdd_default_options", "msdd_create", "msdd_setup", "msdd_setup_batch", "msdd_solve",
           "msdd_solve_batch", "msdd_solve_history", "msdd_apply",
           "msdd_stats", "msdd_get_level_counts", "msdd_get_eigs", "msdd_get_basis",
           "msdd_profile", "msdd_profile_query", "msdd_profile_name", "msdd_last_error",
           "msdd_destroy", "msdd_get_eig_iters", "msdd_warm_start", "msdd_warm_targets",
           "msdd_net_create", "msdd_net_param_count", "msdd_net_set_params",
           "msdd_net_get_params", "msdd_net_forward", "msdd_net_grad", "msdd_net_train_step",
           "msdd_net_last_error", "msdd_net_destroy", "msdd_autotune", "msdd_get_tuning",
           "msdd_set_tuning", "msdd_solve_noalloc",
           "msdd_apply_hybrid", "msdd_solve_gmres"]
MSDD_NPROF = 19

_lib = None


class MsddError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"msdd error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code
        self.stats = None


def load():
    """Load libmsdd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmsdd.so not built ({LIB_PATH}); run paper_2106_06404_amd/build.py")
    # torch ships its own HIP runtime; it is brought up before the library's own one
    # (the order in which both have been seen to share the device)
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.msdd_default_options.argtypes = [ctypes.POINTER(MsddOptions)]
    L.msdd_default_options.restype = None
    L.msdd_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(MsddOptions)]
    L.msdd_create.restype = ctypes.c_int
    L.msdd_setup.argtypes = [vp, i64, vp, vp, vp, i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, i32,
                             vp, f64]
    L.msdd_setup.restype = ctypes.c_int
    L.msdd_setup_batch.argtypes = [vp, i32, vp, i64, vp, vp, vp, i32, i32, vp, vp, i32, vp, vp, vp,
                                   vp, vp, i32, vp, f64]
    L.msdd_setup_batch.restype = ctypes.c_int
    L.msdd_solve.argtypes = [vp, vp, vp, f64, i32, ctypes.POINTER(i32), ctypes.POINTER(f64)]
    L.msdd_solve.restype = ctypes.c_int
    L.msdd_solve_noalloc.argtypes = [vp, vp, vp, f64, i32, ctypes.POINTER(i32),
                                     ctypes.POINTER(f64)]
    L.msdd_solve_noalloc.restype = ctypes.c_int
    L.msdd_apply_hybrid.argtypes = [vp, vp, vp]
    L.msdd_apply_hybrid.restype = ctypes.c_int
    L.msdd_solve_gmres.argtypes = [vp, vp, vp, f64, i32, i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(f64)]
    L.msdd_solve_gmres.restype = ctypes.c_int
    L.msdd_solve_batch.argtypes = [vp, vp, vp, f64, i32, vp, vp]
    L.msdd_solve_batch.restype = ctypes.c_int
    L.msdd_solve_history.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
    L.msdd_solve_history.restype = ctypes.c_int
    L.msdd_apply.argtypes = [vp, vp, vp]
    L.msdd_apply.restype = ctypes.c_int
    L.msdd_stats.argtypes = [vp, ctypes.POINTER(MsddStats)]
    L.msdd_stats.restype = ctypes.c_int
    L.msdd_get_level_counts.argtypes = [vp, i32, vp]
    L.msdd_get_level_counts.restype = ctypes.c_int
    L.msdd_get_eigs.argtypes = [vp, i32, i32, i32, vp, ctypes.POINTER(i32)]
    L.msdd_get_eigs.restype = ctypes.c_int
    L.msdd_get_basis.argtypes = [vp, i32, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.msdd_get_basis.restype = ctypes.c_int
    L.msdd_profile.argtypes = [vp, ctypes.c_int]
    L.msdd_profile.restype = ctypes.c_int
    L.msdd_profile_query.argtypes = [vp, ctypes.c_int, ctypes.POINTER(f64), ctypes.POINTER(i64),
                                     ctypes.POINTER(f64), ctypes.POINTER(f64)]
    L.msdd_profile_query.restype = ctypes.c_int
    L.msdd_profile_name.argtypes = [ctypes.c_int]
    L.msdd_profile_name.restype = ctypes.c_char_p
    L.msdd_last_error.argtypes = [vp]
    L.msdd_last_error.restype = ctypes.c_char_p
    L.msdd_destroy.argtypes = [vp]
    L.msdd_destroy.restype = None
    L.msdd_get_eig_iters.argtypes = [vp, vp]
    L.msdd_get_eig_iters.restype = ctypes.c_int
    L.msdd_warm_start.argtypes = [vp, vp, i32, i32, vp, i64, vp, i32, i32]
    L.msdd_warm_start.restype = ctypes.c_int
    L.msdd_warm_targets.argtypes = [vp, vp, vp, vp]
    L.msdd_warm_targets.restype = ctypes.c_int
    L.msdd_net_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, ctypes.c_uint64, i32, vp]
    L.msdd_net_create.restype = ctypes.c_int
    L.msdd_net_param_count.argtypes = [vp]
    L.msdd_net_param_count.restype = i64
    L.msdd_net_set_params.argtypes = [vp, vp]
    L.msdd_net_set_params.restype = ctypes.c_int
    L.msdd_net_get_params.argtypes = [vp, vp]
    L.msdd_net_get_params.restype = ctypes.c_int
    L.msdd_net_forward.argtypes = [vp, i32, vp, vp, i32]
    L.msdd_net_forward.restype = ctypes.c_int
    L.msdd_net_grad.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_float), vp]
    L.msdd_net_grad.restype = ctypes.c_int
    L.msdd_net_train_step.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, i32, ctypes.c_float,
                                      ctypes.POINTER(ctypes.c_float)]
    L.msdd_net_train_step.restype = ctypes.c_int
    L.msdd_net_last_error.argtypes = [vp]
    L.msdd_net_last_error.restype = ctypes.c_char_p
    L.msdd_net_destroy.argtypes = [vp]
    L.msdd_net_destroy.restype = None
    L.msdd_autotune.argtypes = [vp, i32, i32]
    L.msdd_autotune.restype = ctypes.c_int
    L.msdd_get_tuning.argtypes = [vp, ctypes.POINTER(MsddTuning)]
    L.msdd_get_tuning.restype = ctypes.c_int
    L.msdd_set_tuning.argtypes = [vp, ctypes.POINTER(MsddTuning)]
    L.msdd_set_tuning.restype = ctypes.c_int
    _lib = L
    return L


def default_options(**kw) -> MsddOptions:
    o = MsddOptions()
    load().msdd_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a, dtype):
    """Data pointer of a contiguous torch tensor or numpy array of the given numpy dtype."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.dtype == dtype and a.flags.c_contiguous, (a.dtype, dtype)
        return ctypes.c_void_p(a.ctypes.data)
    import torch
    tmap = {np.dtype(np.float64): torch.float64, np.dtype(np.int32): torch.int32,
            np.dtype(np.int64): torch.int64, np.dtype(np.float32): torch.float32}
    assert isinstance(a, torch.Tensor) and a.dtype == tmap[np.dtype(dtype)] and a.is_contiguous()
    return ctypes.c_void_p(a.data_ptr())


class Msdd:
    """One context of the library (create / setup / solve / apply / stats / destroy)."""

    def __init__(self, options: Optional[MsddOptions] = None, **kw):
        L = load()
        self._L = L
        o = options if options is not None else default_options(**kw)
        h = ctypes.c_void_p()
        rc = L.msdd_create(ctypes.byref(h), ctypes.byref(o))
        if rc != MSDD_OK:
            raise MsddError(rc, "msdd_create failed")
        self._h = h
        self._keep = []

    def _check(self, rc, allow=()):
        if rc != MSDD_OK and rc not in allow:
            msg = self._L.msdd_last_error(self._h).decode()
            err = MsddError(rc, msg)
            st = MsddStats()
            if self._L.msdd_stats(self._h, ctypes.byref(st)) == MSDD_OK:
                err.stats = st.as_dict()   # what the failed call recorded
            raise err
        return rc

    def setup(self, n, rowptr, col, val, elem_dofs, elem_mat, sub_elem_ptr, sub_elem, sub_dof_ptr,
              sub_dof, sub_pou, n_levels, parent, eta):
        n_elem, k = int(elem_dofs.shape[0]), int(elem_dofs.shape[1])
        n_sub = int(sub_elem_ptr.shape[0]) - 1
        rc = self._L.msdd_setup(self._h, int(n), _ptr(rowptr, np.int64), _ptr(col, np.int32),
                                _ptr(val, np.float64), n_elem, k, _ptr(elem_dofs, np.int32),
                                _ptr(elem_mat, np.float64), n_sub, _ptr(sub_elem_ptr, np.int64),
                                _ptr(sub_elem, np.int32), _ptr(sub_dof_ptr, np.int64),
                                _ptr(sub_dof, np.int32), _ptr(sub_pou, np.float64),
                                int(n_levels), _ptr(parent, np.int32) if parent is not None else None,
                                float(eta))
        return self._check(rc)

    def setup_batch(self, prob_dof_ptr, n, rowptr, col, val, elem_dofs, elem_mat, sub_elem_ptr,
                    sub_elem, sub_dof_ptr, sub_dof, sub_pou, n_levels, parent, eta):
        n_elem, k = int(elem_dofs.shape[0]), int(elem_dofs.shape[1])
        n_sub = int(sub_elem_ptr.shape[0]) - 1
        nprob = int(prob_dof_ptr.shape[0]) - 1
        self._nprob = nprob
        rc = self._L.msdd_setup_batch(
            self._h, nprob, _ptr(prob_dof_ptr, np.int64), int(n), _ptr(rowptr, np.int64),
            _ptr(col, np.int32), _ptr(val, np.float64), n_elem, k, _ptr(elem_dofs, np.int32),
            _ptr(elem_mat, np.float64), n_sub, _ptr(sub_elem_ptr, np.int64),
            _ptr(sub_elem, np.int32), _ptr(sub_dof_ptr, np.int64), _ptr(sub_dof, np.int32),
            _ptr(sub_pou, np.float64), int(n_levels),
            _ptr(parent, np.int32) if parent is not None else None, float(eta))
        return self._check(rc)

    def solve_batch(self, b, x, rtol=1e-8, maxit=1000, allow_noconv=False):
        """One CG per problem of a batch: (iters[nprob], relres[nprob], status)."""
        nprob = getattr(self, "_nprob", 1)
        it = np.zeros(nprob, np.int32)
        rel = np.zeros(nprob, np.float64)
        rc = self._L.msdd_solve_batch(self._h, _ptr(b, np.float64), _ptr(x, np.float64),
                                      float(rtol), int(maxit), ctypes.c_void_p(it.ctypes.data),
                                      ctypes.c_void_p(rel.ctypes.data))
        self._check(rc, allow=(MSDD_ENOCONV,) if allow_noconv else ())
        return it, rel, rc

    def solve(self, b, x, rtol=1e-8, maxit=1000, allow_noconv=False):
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        rc = self._L.msdd_solve(self._h, _ptr(b, np.float64), _ptr(x, np.float64), float(rtol),
                                int(maxit), ctypes.byref(it), ctypes.byref(rel))
        self._check(rc, allow=(MSDD_ENOCONV,) if allow_noconv else ())
        return int(it.value), float(rel.value), rc

    def solve_noalloc(self, b, x, rtol=1e-8, maxit=1000, allow_noconv=False):
        """msdd_solve_noalloc: b, x must be device tensors."""
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        rc = self._L.msdd_solve_noalloc(self._h, _ptr(b, np.float64), _ptr(x, np.float64),
                                        float(rtol), int(maxit), ctypes.byref(it),
                                        ctypes.byref(rel))
        self._check(rc, allow=(MSDD_ENOCONV,) if allow_noconv else ())
        return int(it.value), float(rel.value), rc

    def apply_hybrid(self, r, z):
        self._check(self._L.msdd_apply_hybrid(self._h, _ptr(r, np.float64), _ptr(z, np.float64)))

    def solve_gmres(self, b, x, rtol=1e-8, restart=200, maxit=1000, allow_noconv=False):
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        rc = self._L.msdd_solve_gmres(self._h, _ptr(b, np.float64), _ptr(x, np.float64),
                                      float(rtol), int(restart), int(maxit), ctypes.byref(it),
                                      ctypes.byref(rel))
        self._check(rc, allow=(MSDD_ENOCONV,) if allow_noconv else ())
        return int(it.value), float(rel.value), rc

    def history(self) -> np.ndarray:
        """||r_k|| / ||r_0||, k = 0..iters, of the last solve."""
        cnt = ctypes.c_int32()
        self._check(self._L.msdd_solve_history(self._h, None, 0, ctypes.byref(cnt)))
        buf = np.zeros(max(cnt.value, 1), np.float64)
        self._check(self._L.msdd_solve_history(self._h, ctypes.c_void_p(buf.ctypes.data),
                                               cnt.value, ctypes.byref(cnt)))
        return buf[:cnt.value].copy()

    def apply(self, r, z):
        return self._check(self._L.msdd_apply(self._h, _ptr(r, np.float64), _ptr(z, np.float64)))

    def stats(self) -> dict:
        s = MsddStats()
        self._check(self._L.msdd_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def level_counts(self, level: int, nsub: int) -> np.ndarray:
        m = np.zeros(nsub, np.int32)
        self._check(self._L.msdd_get_level_counts(self._h, level, ctypes.c_void_p(m.ctypes.data)))
        return m

    def eigs(self, level: int, i: int, n_extra: int = 0) -> np.ndarray:
        buf = np.zeros(1024, np.float64)
        cnt = ctypes.c_int32()
        self._check(self._L.msdd_get_eigs(self._h, level, i, n_extra,
                                          ctypes.c_void_p(buf.ctypes.data), ctypes.byref(cnt)))
        return buf[:cnt.value].copy()

    def basis(self, level: int, i: int) -> np.ndarray:
        r, c = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._L.msdd_get_basis(self._h, level, i, None, ctypes.byref(r), ctypes.byref(c)))
        out = np.zeros((c.value, r.value), np.float64)  # column-major rows x cols
        if r.value * c.value:
            self._check(self._L.msdd_get_basis(self._h, level, i, ctypes.c_void_p(out.ctypes.data),
                                               ctypes.byref(r), ctypes.byref(c)))
        return out.T.copy()

    def eig_iters(self, nsub: int) -> np.ndarray:
        """Local eigensolver iterations per finest-level subdomain of the last setup."""
        it = np.zeros(nsub, np.int32)
        self._check(self._L.msdd_get_eig_iters(self._h, ctypes.c_void_p(it.ctypes.data)))
        return it

    def warm_start(self, net, n_sub, sub_pos, n_pos, feat=None, collect=0):
        """Attach a warm start to the next setup: net (or None: frame layout only, for
        collect), n_sub finest-level subdomains, sub_pos int32 aligned with sub_dof,
        feat n_sub x n_in float32 (needed with a network), collect = m_cap."""
        n_in = int(feat.shape[1]) if feat is not None else 0
        rc = self._L.msdd_warm_start(self._h, net._h if net is not None else None, int(n_sub),
                                     n_in, _ptr(feat, np.float32) if feat is not None else None,
                                     int(sub_pos.shape[0]), _ptr(sub_pos, np.int32), int(n_pos),
                                     int(collect))
        return self._check(rc)

    def warm_detach(self):
        return self._check(self._L.msdd_warm_start(self._h, None, 0, 0, None, 0, None, 1, 0))

    def warm_targets(self, tgt, mask, cnt):
        """Copy the collected training targets into tgt (n_sub x m_cap x n_pos float32),
        mask (n_sub x n_pos float32) and cnt (n_sub int32)."""
        return self._check(self._L.msdd_warm_targets(self._h, _ptr(tgt, np.float32),
                                                     _ptr(mask, np.float32), _ptr(cnt, np.int32)))

    def autotune(self, what=MSDD_TUNE_EIG | MSDD_TUNE_SOLVE, reps=5) -> dict:
        """Time the candidate launch shapes on the last setup's data; keep the fastest."""
        self._check(self._L.msdd_autotune(self._h, int(what), int(reps)))
        return self.tuning()

    def tuning(self) -> dict:
        t = MsddTuning()
        self._check(self._L.msdd_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, eig_solve=0, eig_splits=0, fine_solve=0, spmv_group=0):
        t = MsddTuning(eig_solve=eig_solve, eig_splits=eig_splits, fine_solve=fine_solve,
                       spmv_group=spmv_group)
        return self._check(self._L.msdd_set_tuning(self._h, ctypes.byref(t)))

    def profile(self, enable=True, reset=True):
        """enable=True: reset (unless reset=False) and enable; False: pause, keeping counts."""
        mode = (1 if reset else 2) if enable else 0
        return self._check(self._L.msdd_profile(self._h, mode))

    def profile_query(self) -> dict:
        """{kernel class: (total_ms, launches, algorithmic bytes, algorithmic flops)}"""
        out = {}
        for i in range(MSDD_NPROF):
            ms, n, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            self._check(self._L.msdd_profile_query(self._h, i, ctypes.byref(ms), ctypes.byref(n),
                                                   ctypes.byref(by), ctypes.byref(fl)))
            out[self._L.msdd_profile_name(i).decode()] = (ms.value, n.value, by.value, fl.value)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.msdd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MsddNet:
    """The warm-start network of the local eigensolver (msdd_net_* of msdd.h)."""

    def __init__(self, n_in, n_hidden, n_vec, n_pos, seed=0, device=0, stream=None):
        L = load()
        self._L = L
        h = ctypes.c_void_p()
        rc = L.msdd_net_create(ctypes.byref(h), int(n_in), int(n_hidden), int(n_vec), int(n_pos),
                               ctypes.c_uint64(seed & (2 ** 64 - 1)), int(device), stream)
        if rc != MSDD_OK:
            raise MsddError(rc, "msdd_net_create failed")
        self._h = h
        self.n_in, self.n_hidden, self.n_vec, self.n_pos = int(n_in), int(n_hidden), int(n_vec), int(n_pos)

    def _check(self, rc):
        if rc != MSDD_OK:
            raise MsddError(rc, self._L.msdd_net_last_error(self._h).decode())
        return rc

    @property
    def n_params(self) -> int:
        return int(self._L.msdd_net_param_count(self._h))

    def set_params(self, p):
        return self._check(self._L.msdd_net_set_params(self._h, _ptr(p, np.float32)))

    def get_params(self, out=None):
        if out is None:
            out = np.zeros(self.n_params, np.float32)
        self._check(self._L.msdd_net_get_params(self._h, _ptr(out, np.float32)))
        return out

    def forward(self, x, y, mode=1):
        """y (batch x n_vec*n_pos) = network(x); mode 0 FP32, 1 BF16 matrix cores."""
        return self._check(self._L.msdd_net_forward(self._h, int(x.shape[0]), _ptr(x, np.float32),
                                                    _ptr(y, np.float32), int(mode)))

    def grad(self, idx, x_all, tgt, mask, cnt, grad=None):
        """Mean loss of samples idx and (into grad, if given) its parameter gradient."""
        loss = ctypes.c_float()
        self._check(self._L.msdd_net_grad(self._h, int(idx.shape[0]), _ptr(idx, np.int32),
                                          int(x_all.shape[0]), _ptr(x_all, np.float32),
                                          _ptr(tgt, np.float32), _ptr(mask, np.float32),
                                          _ptr(cnt, np.int32), int(tgt.shape[1]),
                                          ctypes.byref(loss),
                                          _ptr(grad, np.float32) if grad is not None else None))
        return float(loss.value)

    def train_step(self, idx, x_all, tgt, mask, cnt, lr, want_loss=True):
        loss = ctypes.c_float()
        self._check(self._L.msdd_net_train_step(
            self._h, int(idx.shape[0]), _ptr(idx, np.int32), int(x_all.shape[0]),
            _ptr(x_all, np.float32), _ptr(tgt, np.float32), _ptr(mask, np.float32),
            _ptr(cnt, np.int32), int(tgt.shape[1]), float(lr),
            ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.msdd_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_arrays(probs, device=None):
    """Arrays of the union of several problems for Msdd.setup_batch (indices offset per
    problem; problems must share n_levels, eta and the element size)."""
    parts = [problem_arrays(p) for p in probs]
    assert len({a["n_levels"] for a in parts}) == 1 and len({a["eta"] for a in parts}) == 1
    nb = np.cumsum([0] + [a["n"] for a in parts])
    eb = np.cumsum([0] + [a["elem_dofs"].shape[0] for a in parts])
    nnzb = np.cumsum([0] + [a["col"].shape[0] for a in parts])
    sb_e = np.cumsum([0] + [a["sub_elem"].shape[0] for a in parts])
    sb_d = np.cumsum([0] + [a["sub_dof"].shape[0] for a in parts])
    out = dict(n=int(nb[-1]), n_levels=parts[0]["n_levels"], eta=parts[0]["eta"],
               prob_dof_ptr=nb.astype(np.int64))
    out["rowptr"] = np.concatenate([parts[0]["rowptr"][:1]] +
                                   [a["rowptr"][1:] + nnzb[t] for t, a in enumerate(parts)]).astype(np.int64)
    out["col"] = np.concatenate([a["col"] + nb[t] for t, a in enumerate(parts)]).astype(np.int32)
    out["val"] = np.concatenate([a["val"] for a in parts])
    out["elem_dofs"] = np.concatenate([np.where(a["elem_dofs"] >= 0, a["elem_dofs"] + nb[t], -1)
                                       for t, a in enumerate(parts)]).astype(np.int32)
    out["elem_mat"] = np.concatenate([a["elem_mat"] for a in parts])
    out["sub_elem_ptr"] = np.concatenate([[0]] + [a["sub_elem_ptr"][1:] + sb_e[t]
                                                  for t, a in enumerate(parts)]).astype(np.int64)
    out["sub_elem"] = np.concatenate([a["sub_elem"] + eb[t] for t, a in enumerate(parts)]).astype(np.int32)
    out["sub_dof_ptr"] = np.concatenate([[0]] + [a["sub_dof_ptr"][1:] + sb_d[t]
                                                 for t, a in enumerate(parts)]).astype(np.int64)
    out["sub_dof"] = np.concatenate([a["sub_dof"] + nb[t] for t, a in enumerate(parts)]).astype(np.int32)
    out["sub_pou"] = np.concatenate([a["sub_pou"] for a in parts])
    if parts[0]["parent"] is None:
        out["parent"] = None
    else:
        maps = []
        for lvl in range(len(probs[0].parents)):
            base = 0
            for p in probs:
                maps.append(np.asarray(p.parents[lvl], np.int64) + base)
                base += int(np.max(p.parents[lvl])) + 1
        out["parent"] = np.concatenate(maps).astype(np.int32)
    if device is None:
        return out
    import torch
    return {k: (torch.from_numpy(v).to(device) if isinstance(v, np.ndarray) else v)
            for k, v in out.items()}


def problem_arrays(prob, device=None):
    """The problem's arrays as torch tensors on `device` (or numpy if device is None)."""
    rowptr, col, val = prob.csr_arrays()
    par = np.concatenate(prob.parents).astype(np.int32) if prob.parents else None
    arrs = dict(n=prob.n, rowptr=rowptr, col=col, val=val,
                elem_dofs=np.ascontiguousarray(prob.elem_dofs, np.int32),
                elem_mat=np.ascontiguousarray(prob.elem_mat.reshape(prob.n_elem, -1), np.float64),
                sub_elem_ptr=np.ascontiguousarray(prob.sub_elem_ptr, np.int64),
                sub_elem=np.ascontiguousarray(prob.sub_elem, np.int32),
                sub_dof_ptr=np.ascontiguousarray(prob.sub_dof_ptr, np.int64),
                sub_dof=np.ascontiguousarray(prob.sub_dof, np.int32),
                sub_pou=np.ascontiguousarray(prob.sub_pou, np.float64),
                n_levels=prob.n_levels, parent=par, eta=prob.eta)
    if device is None:
        return arrs
    import torch
    out = {}
    for key, v in arrs.items():
        out[key] = torch.from_numpy(v).to(device) if isinstance(v, np.ndarray) else v
    return out

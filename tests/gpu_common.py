"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the CPU oracle)."""
import numpy as np
import scipy.linalg as sla

from paper_2106_06404_amd import binding as B


def gpu_setup(prob, device="cuda:0", **opts):
    import torch
    arrs = B.problem_arrays(prob, device=device)
    torch.cuda.synchronize()
    m = B.Msdd(**opts)
    m.setup(**arrs)
    return m, arrs


def principal_angle_max(U, V):
    """Largest principal angle between span(U) and span(V) (columns)."""
    if U.shape[1] == 0 and V.shape[1] == 0:
        return 0.0
    if U.shape[1] != V.shape[1]:
        return np.pi / 2
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    s = np.linalg.svd(Qu.T @ Qv, compute_uv=False)
    return float(np.arccos(np.clip(s.min(), -1.0, 1.0)))


def eig_close(lam_gpu, lam_ref, eta, rel=1e-10, floor=1e-3):
    """|d lambda| <= rel * max(lambda, floor * eta) elementwise."""
    lam_gpu = np.asarray(lam_gpu)
    lam_ref = np.asarray(lam_ref)
    scale = np.maximum(np.abs(lam_ref), floor * eta)
    return np.abs(lam_gpu - lam_ref) <= rel * scale


def tie_subdomains(lams, eta, tol=1e-8):
    """Subdomains with an eigenvalue within tol*eta of eta (count is ill-posed there)."""
    out = set()
    for i, lam in enumerate(lams):
        if lam is not None and np.any(np.abs(np.asarray(lam) - eta) < tol * eta):
            out.add(i)
    return out


"""Learned warm start of the local eigensolver: gathering training targets from the
method's own setups and training the network.  Marshalling and loops over the C ABI
only; every arithmetic step runs in the library's kernels."""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import binding as B


def collect_targets(prob, feat: np.ndarray, sub_pos: np.ndarray, n_pos: int, m_cap: int = 16,
                    device: str = "cuda:0", options: Optional[B.MsddOptions] = None):
    """Run one setup of `prob` with target collection; returns device tensors
    (feat [P, n_in] float32, tgt [P, m_cap, n_pos], mask [P, n_pos], cnt [P] int32)
    and the setup's statistics."""
    import torch
    arrs = B.problem_arrays(prob, device)
    ctx = B.Msdd(options)
    try:
        P = prob.n_sub
        ctx.warm_start(None, P, np.ascontiguousarray(sub_pos, np.int32), n_pos, collect=m_cap)
        ctx.setup(arrs["n"], arrs["rowptr"], arrs["col"], arrs["val"], arrs["elem_dofs"],
                  arrs["elem_mat"], arrs["sub_elem_ptr"], arrs["sub_elem"], arrs["sub_dof_ptr"],
                  arrs["sub_dof"], arrs["sub_pou"], arrs["n_levels"], arrs["parent"], arrs["eta"])
        tgt = torch.zeros((P, m_cap, n_pos), dtype=torch.float32, device=device)
        mask = torch.zeros((P, n_pos), dtype=torch.float32, device=device)
        cnt = torch.zeros(P, dtype=torch.int32, device=device)
        ctx.warm_targets(tgt, mask, cnt)
        st = ctx.stats()
    finally:
        ctx.close()
    f = torch.from_numpy(np.ascontiguousarray(feat, np.float32)).to(device)
    return f, tgt, mask, cnt, st


def train(net: B.MsddNet, feat, tgt, mask, cnt, epochs: int = 30, batch: int = 64,
          lr: float = 1e-3, seed: int = 0, lr_final: Optional[float] = None):
    """Adam epochs over seeded permutations of the samples (the last partial batch of an
    epoch is dropped); the learning rate decays geometrically to lr_final if given.
    Returns the mean training loss of every epoch."""
    N = int(feat.shape[0])
    batch = min(batch, N)
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    steps = epochs * (N // batch)
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1)) if lr_final else 1.0
    cur = lr
    for _ in range(epochs):
        perm = rng.permutation(N).astype(np.int32)
        tot, nb = 0.0, 0
        for b0 in range(0, N - batch + 1, batch):
            tot += net.train_step(perm[b0:b0 + batch], feat, tgt, mask, cnt, cur)
            nb += 1
            cur *= decay
        losses.append(tot / max(nb, 1))
    return losses


def mean_loss(net: B.MsddNet, feat, tgt, mask, cnt, batch: int = 256) -> float:
    """Mean loss of the network over all samples (no update)."""
    N = int(feat.shape[0])
    tot = 0.0
    for b0 in range(0, N, batch):
        idx = np.arange(b0, min(N, b0 + batch), dtype=np.int32)
        tot += net.grad(idx, feat, tgt, mask, cnt) * len(idx)
    return tot / N

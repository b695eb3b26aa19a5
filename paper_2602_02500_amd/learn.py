"""Training loop of the coefficient network: repeated calls of the device train step.

All arithmetic (features, forward, loss, backward, Adam) runs in the library's kernels; this
module only slices the caller's device tensors into batches. The caller supplies the initial
parameters and the sample order.
"""
from __future__ import annotations

from . import mlp_features, mlp_train_step, mlp_train_workspace_bytes

__all__ = ["train", "PARAM_LAYOUT"]

# Parameter layout of the network (float32, flattened in this order; weights output-major).
PARAM_LAYOUT = (("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (6, 64)), ("b3", (6,)))


def train(sig, nsig, params, epochs: int = 1, batch: int = 256, lr: float = 1e-3, betas=(0.9, 0.999),
          eps: float = 1e-8, losses=None):
    """Trains `params` (device float32 tensor, updated in place) on the spectra `sig`
    (device float32 [n][smax]) with counts `nsig` (device int32 [n]), in consecutive batches,
    for `epochs` passes. Appends each step's batch loss (device float32 tensor) to `losses`."""
    import torch
    n = int(sig.shape[0])
    dev = sig.device
    feats = torch.empty((n, 8), dtype=torch.float32, device=dev)
    mlp_features(sig, nsig, feats)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = torch.empty(mlp_train_workspace_bytes(batch), dtype=torch.uint8, device=dev)
    t = 0
    for _ in range(epochs):
        for b0 in range(0, n - batch + 1, batch):
            t += 1
            lo = torch.empty(1, dtype=torch.float32, device=dev) if losses is not None else None
            mlp_train_step(feats[b0:b0 + batch], sig[b0:b0 + batch], nsig[b0:b0 + batch], params, m, v, t, lr, ws,
                           betas[0], betas[1], eps, loss_out=lo)
            if losses is not None:
                losses.append(lo)
    return params

"""Learned branching policy: device parameters and training driver.

The network (16 -> 64 -> 64 -> 1, ReLU) and its forward, gradient and update
steps run in libmcs.so (mcs_policy_* in include/mcs.h).  This module keeps the
parameters in torch device memory and loops over training steps; it does no
arithmetic of its own beyond marshalling.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import McsError, _abi, _last_error

F = 16


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st):
    if st < 0:
        raise McsError(st, _last_error())


class Policy:
    """float32 master parameters on the device, plus their half-precision
    packing that the search reads (mcs_opts.policy)."""

    def __init__(self, params: np.ndarray | None = None, seed: int = 0):
        import torch
        self.lib = _abi.load()
        n = int(self.lib.mcs_policy_param_count())
        if params is None:
            params = init_params(seed)
        params = np.asarray(params, dtype=np.float32).reshape(-1)
        if params.size != n:
            raise ValueError(f"expected {n} parameters, got {params.size}")
        self.params = torch.from_numpy(params.copy()).cuda()
        self.half_params = torch.empty(n, dtype=torch.float16, device="cuda")
        self.pack()

    @property
    def n_params(self) -> int:
        return int(self.params.numel())

    def pack(self):
        _check(self.lib.mcs_policy_pack_half(_ptr(self.params), _ptr(self.half_params),
                                             _stream()))

    def numpy(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().astype(np.float64)

    def forward(self, x_half):
        import torch
        rows = int(x_half.shape[0])
        out = torch.empty(rows, dtype=torch.float32, device="cuda")
        _check(self.lib.mcs_policy_forward(_ptr(x_half), rows, _ptr(self.params), _ptr(out),
                                           _stream()))
        return out

    def grad(self, x_half, y):
        """(mean loss, gradient) of the binary cross-entropy over the rows."""
        import torch
        rows = int(x_half.shape[0])
        ws = torch.empty(int(self.lib.mcs_policy_workspace_size(rows)) // 4 + 1,
                         dtype=torch.float32, device="cuda")
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(self.lib.mcs_policy_grad(_ptr(x_half), _ptr(y), rows, _ptr(self.params), _ptr(g),
                                        _ptr(loss), _ptr(ws), ws.numel() * 4, _stream()))
        return loss, g

    def sgd(self, g, lr: float):
        _check(self.lib.mcs_policy_sgd(_ptr(self.params), _ptr(g), float(lr), _stream()))

    def train(self, X: np.ndarray, y: np.ndarray, steps: int = 300, lr: float = 0.5,
              log_every: int = 0, log=print) -> list:
        """Full-batch gradient descent on the device.  Returns the loss curve
        (one value per step)."""
        import torch
        xh = torch.from_numpy(np.asarray(X, dtype=np.float16)).cuda()
        yt = torch.from_numpy(np.asarray(y, dtype=np.float32)).cuda()
        curve = []
        for k in range(steps):
            loss, g = self.grad(xh, yt)
            self.sgd(g, lr)
            curve.append(loss)
            if log_every and k % log_every == 0:
                log(f"policy step {k}: loss {float(loss.item()):.4f}")
        self.pack()
        torch.cuda.synchronize()
        return [float(c.item()) for c in curve]


def init_params(seed: int = 0) -> np.ndarray:
    """He-style random start, packed W1, b1, W2, b2, w3, b3."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / F), (64, F))
    W2 = rng.normal(0, np.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0, np.sqrt(1.0 / 64), 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3,
                           np.zeros(1)]).astype(np.float32)

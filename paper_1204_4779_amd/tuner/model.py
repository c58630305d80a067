"""MLP cost model trained on the GPU with the library's own kernels.

The network (features -> 64 -> 64 -> 1, ReLU) regresses the standardised log
of a variant's measured speed.  Forward, loss gradient and Adam run in
libparaiso's HIP kernels (paraiso_mlp_*); torch only holds the buffers.
"""
from __future__ import annotations

import math

import numpy as np

from .. import binding as pb


class CostModel:
    def __init__(self, in_dim: int, hidden: int = 64, seed: int = 0, lr: float = 3e-3,
                 max_batch: int = 4096):
        import torch
        self.torch = torch
        self.in_dim, self.hidden, self.lr = in_dim, hidden, lr
        self.max_batch = max_batch
        self.n_params, self.ws_bytes = pb.paraiso_mlp_sizes(in_dim, hidden, max_batch)
        rng = np.random.default_rng(seed)
        p = np.zeros(self.n_params, dtype=np.float32)
        o = 0
        for fan_in, fan_out in ((in_dim, hidden), (hidden, hidden)):
            p[o:o + fan_in * fan_out] = rng.normal(scale=math.sqrt(2.0 / fan_in), size=fan_in * fan_out)
            o += fan_in * fan_out + fan_out  # weights, then zero biases
        p[o:o + hidden] = rng.normal(scale=math.sqrt(1.0 / hidden), size=hidden)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.dev = dev
        self.params = torch.from_numpy(p).to(dev)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.ws = torch.empty(self.ws_bytes // 4 + 64, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step_count = 0
        self.stream = torch.cuda.current_stream(dev).cuda_stream

    def _dev(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(self.dev)

    def fit(self, X: np.ndarray, y: np.ndarray, epochs: int = 300) -> float:
        """Full-batch Adam on (X, y); returns the final training loss."""
        B = X.shape[0]
        if B > self.max_batch:
            raise ValueError("batch too large")
        Xd, yd = self._dev(X), self._dev(y)
        for _ in range(epochs):
            pb.paraiso_mlp_loss_grad(Xd.data_ptr(), yd.data_ptr(), B, self.in_dim, self.hidden,
                                     self.params.data_ptr(), self.grad.data_ptr(), self.loss.data_ptr(),
                                     self.ws.data_ptr(), self.ws_bytes, self.stream)
            self.step_count += 1
            pb.paraiso_mlp_adam(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(),
                                self.v.data_ptr(), self.n_params, self.lr, 0.9, 0.999, 1e-8,
                                self.step_count, self.stream)
        self.torch.cuda.synchronize()
        return float(self.loss.item())

    def predict(self, X: np.ndarray) -> np.ndarray:
        out = []
        for s in range(0, X.shape[0], self.max_batch):
            xb = X[s:s + self.max_batch]
            Xd = self._dev(xb)
            yd = self.torch.empty(xb.shape[0], dtype=self.torch.float32, device=self.dev)
            pb.paraiso_mlp_forward(Xd.data_ptr(), xb.shape[0], self.in_dim, self.hidden, self.params.data_ptr(),
                                   yd.data_ptr(), self.ws.data_ptr(), self.ws_bytes, self.stream)
            self.torch.cuda.synchronize()
            out.append(yd.cpu().numpy())
        return np.concatenate(out)

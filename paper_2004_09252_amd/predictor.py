"""Page-access predictor on the GPU: a thin owner of device buffers around
the ``ms_mlp_*`` kernels (include/memshield_mlp.h).

All arithmetic (embedding, matrix products, loss, gradients, Adam, top-k)
runs in the native kernels; this class allocates the parameter blobs and
workspace as torch tensors and marshals calls.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import memshield as ms

PARAM_NAMES = ("E", "W1", "b1", "W2", "b2", "W3", "b3")


class Predictor:
    # Confidence gate of pre-decryption: of the top-k deltas, only those
    # with a softmax probability of at least min_prob are pre-decrypted.
    # Ungated (0.0), the trained network's top 8 on the 2M-access traces
    # removed about as many decrypt faults as with 0.1, at 12-13% precision
    # and 6-7 times the baseline's decrypt work; with 0.1, 99.9% precision
    # and 1.09 times the decrypt work.
    DEFAULT_MIN_PROB = 0.1

    def __init__(self, vocab=1024, context=16, embed=64, hidden=256,
                 max_batch=1024, seed=0, device="cuda",
                 min_prob: float = DEFAULT_MIN_PROB):
        self.shape = ms.ms_mlp_shape(vocab, context, embed, hidden)
        self.n_params, self.offsets = ms.ms_mlp_offsets(self.shape)
        if self.n_params == 0:
            raise ValueError("invalid predictor shape")
        self.vocab, self.context = vocab, context
        self.max_batch = max_batch
        self.min_prob = float(min_prob)
        self.device = device
        self.ws_bytes = ms.ms_mlp_workspace_bytes(self.shape, max_batch)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.master = torch.zeros(self.n_params, dtype=torch.float32,
                                  device=device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grads = torch.zeros_like(self.master)
        self.params = torch.zeros(self.n_params, dtype=torch.bfloat16,
                                  device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.logits = torch.empty(max_batch * vocab, dtype=torch.float32,
                                  device=device)
        self.topk_out = torch.empty(max_batch * 16, dtype=torch.int32,
                                    device=device)
        self.topk_prob = torch.empty(max_batch * 16, dtype=torch.float32,
                                     device=device)
        self.step = 0
        self.init_random(seed)

    # --- parameter blobs ---
    def sizes(self):
        ends = list(self.offsets[1:]) + [self.n_params]
        return {n: e - o for n, o, e in zip(PARAM_NAMES, self.offsets, ends)}

    def init_random(self, seed: int) -> None:
        """Scaled normal weights (std 1/sqrt(fan_in)), zero biases."""
        g = torch.Generator().manual_seed(seed)
        s = self.shape
        cd = s.context * s.embed
        std = {"E": 1.0, "W1": cd ** -0.5, "W2": s.hidden ** -0.5,
               "W3": s.hidden ** -0.5}
        host = torch.zeros(self.n_params, dtype=torch.float32)
        for name, off, size in zip(PARAM_NAMES, self.offsets,
                                   self.sizes().values()):
            if name in std:
                host[off:off + size] = torch.randn(size, generator=g) * \
                    std[name]
        self.load_master(host)

    def load_master(self, host_fp32) -> None:
        """Set float32 master weights (blob layout); refresh the bf16 blob."""
        t = torch.as_tensor(np.asarray(host_fp32, dtype=np.float32)
                            if not torch.is_tensor(host_fp32) else host_fp32,
                            dtype=torch.float32)
        self.master.copy_(t.to(self.device))
        self.m.zero_()
        self.v.zero_()
        self.step = 0
        self._check(ms.ms_mlp_to_bf16(self.master.data_ptr(),
                                      self.params.data_ptr(), self.n_params,
                                      self._stream()), "ms_mlp_to_bf16")

    def save(self, path: str) -> None:
        """Write the float32 master weights and the shape (numpy .npz)."""
        s = self.shape
        np.savez(path, master=self.master.cpu().numpy(),
                 shape=np.array([s.vocab, s.context, s.embed, s.hidden]),
                 step=np.array([self.step]))

    def load(self, path: str) -> None:
        """Read weights written by ``save`` (no pickled objects)."""
        with np.load(path, allow_pickle=False) as z:
            s = self.shape
            if z["shape"].tolist() != [s.vocab, s.context, s.embed, s.hidden]:
                raise ValueError("predictor shape mismatch")
            self.load_master(z["master"])

    def unpack(self, blob: torch.Tensor) -> dict:
        out = {}
        for name, off, size in zip(PARAM_NAMES, self.offsets,
                                   self.sizes().values()):
            out[name] = blob[off:off + size]
        return out

    # --- kernels ---
    @staticmethod
    def _stream():
        return torch.cuda.current_stream().cuda_stream

    @staticmethod
    def _check(st, what):
        if st != ms.MS_OK:
            raise ms.MemShieldError(st, what)

    def _ids(self, ids) -> torch.Tensor:
        t = torch.as_tensor(ids, dtype=torch.int32)
        if t.device.type != "cuda":
            t = t.to(self.device)
        t = t.contiguous()
        assert t.dim() == 2 and t.shape[1] == self.context
        assert t.shape[0] <= self.max_batch
        return t

    def forward(self, ids) -> torch.Tensor:
        """logits (B, V) float32 on the device."""
        t = self._ids(ids)
        B = t.shape[0]
        self._check(ms.ms_mlp_forward(self.shape, self.params.data_ptr(),
                                      t.data_ptr(), B,
                                      self.logits.data_ptr(),
                                      self.ws.data_ptr(), self.ws_bytes,
                                      self._stream()), "ms_mlp_forward")
        return self.logits[:B * self.vocab].view(B, self.vocab)

    def backward(self, ids, targets) -> torch.Tensor:
        """Gradients (blob) of the mean loss; returns the loss tensor."""
        t = self._ids(ids)
        y = torch.as_tensor(targets, dtype=torch.int32).to(self.device)
        y = y.contiguous()
        self._check(ms.ms_mlp_backward(self.shape, self.params.data_ptr(),
                                       t.data_ptr(), y.data_ptr(),
                                       t.shape[0], self.grads.data_ptr(),
                                       self.loss.data_ptr(),
                                       self.ws.data_ptr(), self.ws_bytes,
                                       self._stream()), "ms_mlp_backward")
        return self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        self.step += 1
        self._check(ms.ms_mlp_adam(self.shape, self.master.data_ptr(),
                                   self.m.data_ptr(), self.v.data_ptr(),
                                   self.grads.data_ptr(),
                                   self.params.data_ptr(), lr, beta1, beta2,
                                   eps, self.step, self._stream()),
                    "ms_mlp_adam")

    def train_step(self, ids, targets, lr=1e-3) -> torch.Tensor:
        loss = self.backward(ids, targets)
        self.adam(lr=lr)
        return loss

    def topk(self, logits: torch.Tensor, k: int, exclude: int,
             with_prob: bool = False):
        B = logits.shape[0]
        self._check(ms.ms_mlp_topk(logits.data_ptr(), B, self.vocab, k,
                                   exclude, self.topk_out.data_ptr(),
                                   self.topk_prob.data_ptr() if with_prob
                                   else None, self._stream()), "ms_mlp_topk")
        ids = self.topk_out[:B * k].view(B, k)
        if with_prob:
            return ids, self.topk_prob[:B * k].view(B, k)
        return ids

    def predict(self, ids, k: int, exclude: int, with_prob: bool = False):
        return self.topk(self.forward(ids), k, exclude, with_prob)

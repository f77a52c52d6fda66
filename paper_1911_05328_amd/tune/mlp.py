"""The learned schedule proposal: an MLP cost model trained on the GPU by the
library's own kernels (mm_mlp_* in the C ABI).

Network: 7 inputs (log2 m, n, k; dtype one-hot; log2 budget / |C|) ->
3 hidden layers of 64 ReLU units -> one output per schedule, the predicted (standardised)
log-time of every schedule of the space.  Loss: mean-squared error over the
schedules that were measured and fit the budget (masked).  Update: Adam.
torch provides only device buffers and the stream; every arithmetic step of
training and inference is a library kernel.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from .. import _lib
from . import space

SIZES = (space.NFEAT, 64, 64, 64, space.NSCHED)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check(st, what):
    if st != 0:
        raise _lib.StarmmError(st, what)


class CostModel:
    def __init__(self, seed: int = 1911, sizes=SIZES):
        import torch
        self.torch = torch
        self.sizes = tuple(sizes)
        g = np.random.Generator(np.random.PCG64(seed))
        self.params = []  # (W out x in, b out) device float32
        for i, o in zip(self.sizes, self.sizes[1:]):
            bound = math.sqrt(6.0 / i)  # He-uniform for ReLU layers
            W = g.uniform(-bound, bound, (o, i)).astype(np.float32)
            b = np.zeros(o, np.float32)
            self.params.append((torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda()))
        self.adam_m = [(torch.zeros_like(W), torch.zeros_like(b)) for W, b in self.params]
        self.adam_v = [(torch.zeros_like(W), torch.zeros_like(b)) for W, b in self.params]
        self.step_count = 0
        self.t_mean, self.t_std = 0.0, 1.0

    # ---------------------------------------------------------------- kernels
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def forward(self, X):
        """Layer outputs [X, H1, ..., HL] as device tensors."""
        torch, L = self.torch, _lib.lib()
        H = [X]
        for l, (W, b) in enumerate(self.params):
            out = torch.empty((X.shape[0], W.shape[0]), dtype=torch.float32, device="cuda")
            relu = 1 if l + 1 < len(self.params) else 0
            _check(L.mm_mlp_linear_forward(X.shape[0], W.shape[1], W.shape[0], _p(H[-1]), _p(W), _p(b), _p(out),
                                           relu, self._stream()), "mm_mlp_linear_forward")
            H.append(out)
        return H

    def loss_and_grads(self, X, T, M):
        """(loss device scalar, [(dW, db)]) of the masked MSE."""
        torch, L = self.torch, _lib.lib()
        H = self.forward(X)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        dY = torch.empty_like(H[-1])
        _check(L.mm_mlp_masked_mse(H[-1].numel(), _p(H[-1]), _p(T), _p(M), _p(loss), _p(dY), self._stream()),
               "mm_mlp_masked_mse")
        grads = [None] * len(self.params)
        for l in range(len(self.params) - 1, -1, -1):
            W, b = self.params[l]
            relu = 1 if l + 1 < len(self.params) else 0
            dZ = torch.empty_like(H[l + 1])
            dX = torch.empty_like(H[l]) if l > 0 else None
            dW = torch.empty_like(W)
            db = torch.empty_like(b)
            _check(L.mm_mlp_linear_backward(X.shape[0], W.shape[1], W.shape[0], _p(H[l]), _p(W), _p(H[l + 1]),
                                            _p(dY), _p(dZ), _p(dX), _p(dW), _p(db), relu, self._stream()),
                   "mm_mlp_linear_backward")
            grads[l] = (dW, db)
            dY = dX
        return loss, grads

    def adam_step(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        L = _lib.lib()
        self.step_count += 1
        for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(self.params, grads, self.adam_m, self.adam_v):
            for p, g, m, v in ((W, gW, mW, vW), (b, gb, mb, vb)):
                _check(L.mm_mlp_adam(p.numel(), _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, self.step_count,
                                     self._stream()), "mm_mlp_adam")

    # --------------------------------------------------------------- training
    def fit(self, X, T, M, steps=2000, lr=3e-3, lr_final=2e-4, log_every=0):
        """Full-batch Adam on standardised log-time targets.  X, T, M numpy."""
        torch = self.torch
        meas = M > 0
        self.t_mean = float(T[meas].mean())
        self.t_std = float(T[meas].std() + 1e-6)
        Tn = np.where(meas, (T - self.t_mean) / self.t_std, 0.0)
        dX = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
        dT = torch.from_numpy(np.ascontiguousarray(Tn, np.float32)).cuda()
        dM = torch.from_numpy(np.ascontiguousarray(M, np.float32)).cuda()
        hist = []
        for s in range(steps):
            frac = s / max(steps - 1, 1)
            cur = lr * (lr_final / lr) ** frac  # geometric decay
            loss, grads = self.loss_and_grads(dX, dT, dM)
            self.adam_step(grads, lr=cur)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
        return hist

    def predict(self, X):
        """Predicted log-time (natural log, ms) of every schedule, numpy N x NSCHED."""
        torch = self.torch
        dX = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
        out = self.forward(dX)[-1].cpu().numpy().astype(np.float64)
        return out * self.t_std + self.t_mean

    # ------------------------------------------------------------------- I/O
    def state(self):
        d = {"t_mean": self.t_mean, "t_std": self.t_std, "sizes": np.array(self.sizes)}
        if getattr(self, "accurate", None) is not None:
            d["accurate"] = np.asarray(self.accurate, np.float32)
        for l, (W, b) in enumerate(self.params):
            d[f"W{l}"] = W.cpu().numpy()
            d[f"b{l}"] = b.cpu().numpy()
        return d

    def save(self, path):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path):
        z = np.load(path)  # plain arrays only (no pickles)
        m = cls(sizes=tuple(int(x) for x in z["sizes"]))
        m.t_mean, m.t_std = float(z["t_mean"]), float(z["t_std"])
        m.params = [(m.torch.from_numpy(z[f"W{l}"]).cuda(), m.torch.from_numpy(z[f"b{l}"]).cuda())
                    for l in range(len(m.sizes) - 1)]
        m.accurate = np.asarray(z["accurate"]) if "accurate" in z.files else None
        return m

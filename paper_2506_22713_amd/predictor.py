"""Learned warm start of the basis size (binding and training loop).

The network, its loss, gradient and Adam update run in the library's
kernels (eodabe_mlp_forward / _grad / _adam); this module holds the
parameters on the device, feeds batches and reads and writes checkpoints.

Checkpoint format: one JSON header line (UTF-8, ending in a newline) with
keys format ("eodabe-mlp-1"), nparam, step, dtype ("float32"), order
(["params", "m", "v"]) and free-form meta, followed by the three arrays of
nparam little-endian FP32 values in that order.
"""
from __future__ import annotations

import ctypes
import json

import numpy as np
import torch

from . import _lib, Context, EodAbeError, EODABE_EINVAL

NPARAM = int(_lib.eodabe_mlp_param_count())
NIN, NH, NOUT = 67, 256, 2
FORMAT = "eodabe-mlp-1"


def features(diag: np.ndarray, m: int, n: int, eps: float) -> np.ndarray:
    """eodabe_mlp_features: the 67 inputs from the stopping-test values d_0..d_63
    and the threshold eps = tol ||A||_F."""
    d = np.ascontiguousarray(np.asarray(diag, dtype=np.float64)[:64])
    if d.size < 64:
        raise EodAbeError(EODABE_EINVAL, "features: 64 stopping-test values needed")
    out = np.zeros(NIN, dtype=np.float32)
    st = _lib.eodabe_mlp_features(d.ctypes.data_as(ctypes.c_void_p), int(m), int(n), float(eps),
                                  out.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise EodAbeError(st, "eodabe_mlp_features")
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights (fan-in), zero biases, in the flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for nout, nin in ((NH, NIN), (NH, NH), (NH, NH), (NOUT, NH)):
        lim = np.sqrt(6.0 / nin)
        parts.append(rng.uniform(-lim, lim, size=nout * nin))
        parts.append(np.zeros(nout))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == NPARAM
    return p


class Predictor:
    """MLP parameters and Adam state on the device."""

    def __init__(self, params: np.ndarray | None = None, seed: int = 0, device: str = "cuda"):
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.size != NPARAM:
            raise EodAbeError(EODABE_EINVAL, "predictor: wrong parameter count")
        self.params = torch.from_numpy(p.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step = 0
        self.meta: dict = {}
        self._ws, self._wsb = None, 0

    def _workspace(self, batch: int):
        need = int(_lib.eodabe_mlp_workspace_size(batch))
        if self._ws is None or self._wsb < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.params.device)
            self._wsb = need
        return self._ws

    def forward(self, ctx: Context, X: torch.Tensor) -> torch.Tensor:
        X = X.contiguous().float()
        B = X.shape[0]
        Y = torch.empty((B, NOUT), dtype=torch.float32, device=self.params.device)
        ws = self._workspace(B)
        ctx._check(_lib.eodabe_mlp_forward(ctx.h, self.params.data_ptr(), X.data_ptr(), B, Y.data_ptr(),
                                           ws.data_ptr(), self._wsb), "eodabe_mlp_forward")
        return Y

    def grad(self, ctx: Context, X: torch.Tensor, T: torch.Tensor) -> float:
        """Loss of the batch; the gradient lands in self.grads."""
        X = X.contiguous().float()
        T = T.contiguous().float()
        B = X.shape[0]
        ws = self._workspace(B)
        loss = ctypes.c_double()
        ctx._check(_lib.eodabe_mlp_grad(ctx.h, self.params.data_ptr(), X.data_ptr(), T.data_ptr(), B,
                                        self.grads.data_ptr(), ws.data_ptr(), self._wsb, ctypes.byref(loss)),
                   "eodabe_mlp_grad")
        return float(loss.value)

    def adam(self, ctx: Context, lr: float):
        self.step += 1
        ctx._check(_lib.eodabe_mlp_adam(ctx.h, self.params.data_ptr(), self.grads.data_ptr(), self.m.data_ptr(),
                                        self.v.data_ptr(), float(lr), self.step), "eodabe_mlp_adam")

    def train_step(self, ctx: Context, X: torch.Tensor, T: torch.Tensor, lr: float) -> float:
        loss = self.grad(ctx, X, T)
        self.adam(ctx, lr)
        return loss

    def attach(self, ctx: Context, margin: float = 0.1):
        ctx.set_predictor(self.params, margin)

    def save(self, path: str, meta: dict | None = None):
        head = dict(format=FORMAT, nparam=NPARAM, step=self.step, dtype="float32", order=["params", "m", "v"],
                    meta={**self.meta, **(meta or {})})
        with open(path, "wb") as fh:
            fh.write((json.dumps(head, sort_keys=True) + "\n").encode("utf-8"))
            for t in (self.params, self.m, self.v):
                fh.write(t.detach().cpu().numpy().astype("<f4").tobytes())

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "Predictor":
        with open(path, "rb") as fh:
            head = json.loads(fh.readline().decode("utf-8"))
            if head.get("format") != FORMAT or head.get("nparam") != NPARAM:
                raise EodAbeError(EODABE_EINVAL, f"predictor checkpoint {path}: unknown format")
            arr = np.frombuffer(fh.read(), dtype="<f4")
        if arr.size != 3 * NPARAM:
            raise EodAbeError(EODABE_EINVAL, f"predictor checkpoint {path}: truncated")
        pr = cls(arr[:NPARAM], device=device)
        pr.m.copy_(torch.from_numpy(arr[NPARAM:2 * NPARAM].copy()))
        pr.v.copy_(torch.from_numpy(arr[2 * NPARAM:].copy()))
        pr.step = int(head.get("step", 0))
        pr.meta = dict(head.get("meta", {}))
        return pr

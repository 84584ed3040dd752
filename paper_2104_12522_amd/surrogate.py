"""Learned surrogate of the binned transmission spectrum for delayed-acceptance MCMC.

A multilayer perceptron (parameters scaled to the prior box -> standardised binned
depths), trained on spectra that the library's own forward model generates from prior
draws, with the library's BF16 matrix-core kernels for the forward pass, the
back-propagation and Adam. Argument marshalling only: every arithmetic step runs in
libbartmi; torch allocates device memory and provides streams.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import BartmiError, Forward, _check, _ptr, _stream, lib
from ._abi import BM_MLP_MAX_LAYERS, BmMlp


class MLP:
    """Device state of one network (the bm_mlp struct plus the tensors it borrows)."""

    def __init__(self, dims, max_batch: int, seed: int = 0, device="cuda"):
        dims = [int(d) for d in dims]
        n = len(dims) - 1
        if not 1 <= n <= BM_MLP_MAX_LAYERS:
            raise BartmiError(f"1..{BM_MLP_MAX_LAYERS} layers")
        self.dims, self.n_layers, self.max_batch = dims, n, max_batch
        f32 = dict(dtype=torch.float32, device=device)
        bf = dict(dtype=torch.int16, device=device)   # raw BF16 bit patterns
        g = np.random.default_rng(seed)
        self.w32, self.w16, self.b32 = [], [], []
        self.gw, self.gb, self.mw, self.vw, self.mb, self.vb = [], [], [], [], [], []
        self.z, self.h = [], []
        for i in range(n):
            fan_in, fan_out = dims[i], dims[i + 1]
            # He-uniform for SiLU layers, Glorot-uniform for the linear output layer
            lim = math.sqrt(6.0 / fan_in) if i < n - 1 else math.sqrt(6.0 / (fan_in + fan_out))
            w = g.uniform(-lim, lim, (fan_out, fan_in)).astype(np.float32)
            self.w32.append(torch.as_tensor(w, **f32))
            self.w16.append(torch.empty(fan_out, fan_in, **bf))
            self.b32.append(torch.zeros(fan_out, **f32))
            for lst, shape in ((self.gw, (fan_out, fan_in)), (self.gb, (fan_out,)),
                               (self.mw, (fan_out, fan_in)), (self.vw, (fan_out, fan_in)),
                               (self.mb, (fan_out,)), (self.vb, (fan_out,))):
                lst.append(torch.zeros(*shape, **f32))
            self.h.append(torch.empty(max_batch, fan_in, **bf))
            self.z.append(torch.empty(max_batch, fan_out, **f32) if i < n - 1 else None)
        wmax = max(dims[1:])
        self.dz = [torch.empty(max_batch, wmax, **bf) for _ in range(2)]
        st = BmMlp()
        st.n_layers, st.max_batch = n, max_batch
        for i, d in enumerate(dims):
            st.dims[i] = d
        for name in ("w32", "w16", "b32", "gw", "gb", "mw", "vw", "mb", "vb", "z", "h"):
            arr = getattr(st, name)
            for i, t in enumerate(getattr(self, name)):
                arr[i] = _ptr(t).value
        for i in range(2):
            st.dz[i] = _ptr(self.dz[i]).value
        self.struct = st
        self.step = 0
        self.sync_bf16()

    def _r(self, fn, *args, stream=None):
        _check(getattr(lib(), fn)(C.byref(self.struct), *args, _stream(stream)), fn)

    def sync_bf16(self, stream=None):
        self._r("bm_mlp_sync_bf16", stream=stream)

    def set_input(self, params, lo, hi, rows=None, B=None, stream=None):
        B = params.shape[0] if B is None else B
        self._r("bm_mlp_set_input", _ptr(params), params.shape[1], _ptr(rows), B, lo.numel(),
                _ptr(lo), _ptr(hi), stream=stream)

    def forward(self, B: int, out: torch.Tensor, stream=None):
        self._r("bm_mlp_forward", B, _ptr(out), stream=stream)

    def loss_grad(self, B, out, target, rows=None, mean=None, scale=None, row_loss=None,
                  stream=None):
        self._r("bm_mlp_loss_grad", B, _ptr(out), _ptr(target), _ptr(rows), _ptr(mean),
                _ptr(scale), _ptr(row_loss), stream=stream)

    def backward(self, B: int, stream=None):
        self._r("bm_mlp_backward", B, stream=stream)

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        self._r("bm_adam_step", C.c_float(lr), C.c_float(beta1), C.c_float(beta2),
                C.c_float(eps), self.step, stream=stream)

    @property
    def n_weights(self) -> int:
        return sum(self.dims[i] * self.dims[i + 1] + self.dims[i + 1] for i in range(self.n_layers))


class Trainer:
    """Minibatch Adam on (params, binned spectra) pairs resident on the GPU."""

    def __init__(self, net: MLP, lo, hi, params: torch.Tensor, targets: torch.Tensor,
                 mean: torch.Tensor, scale: torch.Tensor, batch: int, seed: int = 0):
        if batch > net.max_batch:
            raise BartmiError("batch exceeds the network's max_batch")
        self.net, self.lo, self.hi = net, lo, hi
        self.params, self.targets, self.mean, self.scale = params, targets, mean, scale
        self.batch = batch
        self.out = torch.empty(batch, net.dims[-1], dtype=torch.float32, device=params.device)
        self.row_loss = torch.empty(batch, dtype=torch.float32, device=params.device)
        self.gen = np.random.default_rng(seed)

    def epoch(self, lr: float, stream=None) -> torch.Tensor:
        """One pass over the data in a fresh random order; returns the per-row losses of
        every minibatch, concatenated (device), for monitoring."""
        n = self.params.shape[0]
        perm = torch.as_tensor(self.gen.permutation(n).astype(np.int32), device=self.params.device)
        losses = []
        for s in range(0, n - self.batch + 1, self.batch):
            rows = perm[s:s + self.batch]
            self.step(rows, lr, stream)
            losses.append(self.row_loss.clone())
        return torch.cat(losses)

    def step(self, rows: torch.Tensor, lr: float, stream=None):
        B = rows.numel()
        net = self.net
        net.set_input(self.params, self.lo, self.hi, rows=rows, B=B, stream=stream)
        net.forward(B, self.out, stream=stream)
        net.loss_grad(B, self.out, self.targets, rows=rows, mean=self.mean, scale=self.scale,
                      row_loss=self.row_loss, stream=stream)
        net.backward(B, stream=stream)
        net.adam(lr, stream=stream)


class Surrogate:
    """Callable for Retrieval(surrogate=...): [C][d] parameters -> [C] surrogate chi^2 of
    the model's observation, all on the library's kernels."""

    def __init__(self, net: MLP, lo: torch.Tensor, hi: torch.Tensor, mean: torch.Tensor,
                 scale: torch.Tensor, data: torch.Tensor, err: torch.Tensor, n_chains: int):
        self.net, self.lo, self.hi, self.mean, self.scale = net, lo, hi, mean, scale
        self.data, self.err = data, err
        dev = lo.device
        self.out = torch.empty(n_chains, net.dims[-1], dtype=torch.float32, device=dev)
        self.chi2 = torch.empty(n_chains, dtype=torch.float64, device=dev)

    def predict(self, params: torch.Tensor, stream=None) -> torch.Tensor:
        """Standardised surrogate outputs [B][N] (FP32) for B <= n_chains parameter rows."""
        B = params.shape[0]
        self.net.set_input(params, self.lo, self.hi, stream=stream)
        self.net.forward(B, self.out, stream=stream)
        return self.out[:B]

    def __call__(self, params: torch.Tensor, stream=None) -> torch.Tensor:
        B = params.shape[0]
        self.predict(params, stream)
        N = self.net.dims[-1]
        _check(lib().bm_surrogate_chi2(_ptr(self.out), B, N, _ptr(self.mean), _ptr(self.scale),
                                       _ptr(self.data), _ptr(self.err), _ptr(self.chi2),
                                       _stream(stream)), "bm_surrogate_chi2")
        return self.chi2[:B]


def training_set(model, prior, n: int, seed: int, batch: int = 4096, device="cuda"):
    """n prior draws and their binned spectra from the library's batched forward model.
    Draws flagged by the forward model (clamped temperatures, invalid radii...) are
    dropped. Returns (params [m][d] double, binned [m][nb] double), m <= n."""
    if model.n_bins == 0:
        raise BartmiError("the model needs a bin width for binned training targets")
    theta = torch.as_tensor(prior.draw(n, seed=seed), device=device)
    fwd = Forward(model, batch, binned=True)
    keep_p, keep_y = [], []
    nb = model.n_bins
    for s in range(0, n, batch):
        chunk = theta[s:s + batch]
        m = chunk.shape[0]
        if m < batch:
            fwd = Forward(model, m, binned=True)
        fwd(chunk.contiguous())
        ok = fwd.flags == 0
        keep_p.append(chunk[ok])
        keep_y.append(fwd.binned.view(m, nb)[ok])
    return torch.cat(keep_p).contiguous(), torch.cat(keep_y).contiguous()


def standardisation(targets: torch.Tensor):
    """Per-bin mean and scale of the training targets (host statistics in double)."""
    y = targets.cpu().numpy()
    mean = y.mean(0)
    scale = y.std(0)
    scale[scale == 0] = 1.0
    dev = targets.device
    return torch.as_tensor(mean, device=dev), torch.as_tensor(scale, device=dev)

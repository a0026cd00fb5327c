"""Learned warm start for batched Newton-Raphson power flow.

A fully connected network (GELU hidden layers) maps each scenario's specified injections
-- (P, Q) at PQ buses, (P, |V| set-point) at PV buses -- to initial voltages (|V|, angle)
of every non-REF bus.  Newton still iterates to the same tolerance from that start, so
the network changes only the iteration count; instances that do not converge from the
predicted start are solved again from flat start.

This module only marshals arguments: every arithmetic step of training and inference
(matrix-core GEMMs with fused bias/GELU, activation backward, MSE gradient, Adam, feature
extraction, start-vector assembly) runs in the HIP library through its C ABI.  Device
memory comes from PyTorch; host-side work is limited to seeded initialisation, the
normalisation statistics of the training targets and minibatch index shuffling.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import (PF_BUS_PQ, PF_BUS_PV, PF_BUS_REF, PF_FP64, Plan, PfError, Result, _check, lib,
               solve_batch)

_vp = ctypes.c_void_p


def _p(t):
    return _vp(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


@dataclass
class TrainReport:
    epochs: int
    steps: int
    seconds: float
    train_loss: List[float] = field(default_factory=list)
    val_loss: List[float] = field(default_factory=list)


class WarmStartNet:
    """Network state on the device: FP32 master weights, BF16 copies for the GEMMs,
    FP32 biases, Adam moments and the normalisation constants."""

    def __init__(self, bus_type, hidden=(512, 512, 512), seed: int = 0, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        bt = np.asarray(bus_type, dtype=np.int8)
        self.n = int(bt.shape[0])
        self.feat_bus = np.flatnonzero(bt != PF_BUS_REF).astype(np.int32)
        self.nf = int(self.feat_bus.shape[0])
        self.dims = [2 * self.nf, *hidden, 2 * self.nf]
        rng = np.random.default_rng(seed)
        self.W, self.Wb, self.b, self.mW, self.vW, self.mb, self.vb = [], [], [], [], [], [], []
        for din, dout in zip(self.dims[:-1], self.dims[1:]):
            lim = math.sqrt(6.0 / (din + dout))
            w = torch.from_numpy(rng.uniform(-lim, lim, (din, dout)).astype(np.float32)).to(self.device)
            self.W.append(w)
            self.Wb.append(torch.empty((din, dout), dtype=torch.int16, device=self.device))
            self.b.append(torch.zeros(dout, dtype=torch.float32, device=self.device))
            self.mW.append(torch.zeros_like(w)); self.vW.append(torch.zeros_like(w))
            self.mb.append(torch.zeros(dout, dtype=torch.float32, device=self.device))
            self.vb.append(torch.zeros(dout, dtype=torch.float32, device=self.device))
        self._refresh_bf16()
        self.step = 0
        self.bus_type_d = torch.from_numpy(bt).to(self.device)
        self.feat_bus_d = torch.from_numpy(self.feat_bus).to(self.device)
        one = np.ones(2 * self.nf, np.float32)
        self.set_normalization(np.zeros_like(one), one, np.zeros_like(one), one)

    # ------------------------------------------------------------------ plumbing
    def _refresh_bf16(self):
        for w, wb in zip(self.W, self.Wb):
            _check(lib().pf_mlp_to_bf16(w.numel(), _p(w), _p(wb), _stream()), "pf_mlp_to_bf16")

    def set_normalization(self, mu_x, sd_x, mu_y, sd_y):
        t = self.torch
        f = lambda a: t.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)
        self.mu_x, self.sd_x, self.mu_y, self.sd_y = f(mu_x), f(sd_x), f(mu_y), f(sd_y)

    @property
    def n_params(self) -> int:
        return sum(w.numel() + b.numel() for w, b in zip(self.W, self.b))

    def features(self, sbus, v0):
        """BF16 z-scored features [B][2 nf] from device sbus (complex128 [B][n]) and v0."""
        t = self.torch
        B = int(v0.shape[0])
        s2 = t.view_as_real(sbus) if sbus.dtype == t.complex128 else sbus
        x = t.empty((B, 2 * self.nf), dtype=t.int16, device=self.device)
        for b0 in range(0, B, 65535):
            b1 = min(B, b0 + 65535)
            _check(lib().pf_mlp_features(b1 - b0, self.n, _vp(s2[b0:b1].data_ptr()), _vp(v0[b0:b1].data_ptr()),
                                         _p(self.bus_type_d), _p(self.feat_bus_d), self.nf, _p(self.mu_x),
                                         _p(self.sd_x), _vp(x[b0:b1].data_ptr()), _stream()), "pf_mlp_features")
        return x

    def forward(self, x_bf16, keep: bool = False):
        """Network output (FP32, normalised units).  With keep=True also returns the
        per-layer (input BF16, pre-activation FP32) needed by the backward pass."""
        t = self.torch
        B = int(x_bf16.shape[0])
        a = x_bf16
        cache = []
        L = len(self.W)
        out = None
        for l in range(L):
            din, dout = self.dims[l], self.dims[l + 1]
            z = t.empty((B, dout), dtype=t.float32, device=self.device) if (keep or l == L - 1) else None
            last = l == L - 1
            a_next = None if last else t.empty((B, dout), dtype=t.int16, device=self.device)
            _check(lib().pf_mlp_gemm(B, dout, din, 0, 0, _p(a), _p(self.Wb[l]), _p(self.b[l]), 0 if last else 1,
                                     _p(z), _p(a_next), None, _stream()), "pf_mlp_gemm")
            cache.append((a, z))
            if last:
                out = z
            a = a_next
        return (out, cache) if keep else out

    def _backward_and_update(self, cache, dout, lr):
        t = self.torch
        L = len(self.W)
        g = dout
        self.step += 1
        for l in range(L - 1, -1, -1):
            a, z = cache[l]
            B = int(a.shape[0])
            din, dn = self.dims[l], self.dims[l + 1]
            dz = t.empty((B, dn), dtype=t.int16, device=self.device)
            db = t.empty(dn, dtype=t.float32, device=self.device)
            _check(lib().pf_mlp_act_backward(B, dn, _p(g), _p(z), 0 if l == L - 1 else 1, _p(dz), _p(db), _stream()),
                   "pf_mlp_act_backward")
            dW = t.empty((din, dn), dtype=t.float32, device=self.device)
            _check(lib().pf_mlp_gemm(din, dn, B, 1, 0, _p(a), _p(dz), None, 0, _p(dW), None, None, _stream()),
                   "pf_mlp_gemm")
            if l > 0:
                g = t.empty((B, din), dtype=t.float32, device=self.device)
                _check(lib().pf_mlp_gemm(B, din, dn, 0, 1, _p(dz), _p(self.Wb[l]), None, 0, _p(g), None, None,
                                         _stream()), "pf_mlp_gemm")
            self.last_grads = getattr(self, "last_grads", {})
            self.last_grads[l] = (dW, db)
            _check(lib().pf_mlp_adam(dW.numel(), _p(self.W[l]), _p(self.Wb[l]), _p(dW), _p(self.mW[l]),
                                     _p(self.vW[l]), lr, 0.9, 0.999, 1e-8, self.step, _stream()), "pf_mlp_adam")
            _check(lib().pf_mlp_adam(db.numel(), _p(self.b[l]), None, _p(db), _p(self.mb[l]), _p(self.vb[l]), lr,
                                     0.9, 0.999, 1e-8, self.step, _stream()), "pf_mlp_adam")

    def loss_and_grad(self, out, target):
        t = self.torch
        grad = t.empty_like(out)
        parts = t.empty(256, dtype=t.float32, device=self.device)
        _check(lib().pf_mlp_mse(out.numel(), _p(out), _p(target), _p(grad), _p(parts), 256, _stream()), "pf_mlp_mse")
        return parts, grad

    def train_step(self, x_bf16, y_norm, lr=1e-3, update=True):
        out, cache = self.forward(x_bf16, keep=True)
        parts, grad = self.loss_and_grad(out, y_norm)
        if update:
            self._backward_and_update(cache, grad, lr)
        return parts

    # ------------------------------------------------------------------ training
    def fit(self, x_all, y_all, n_train: int, epochs: int = 20, batch: int = 256, lr: float = 1e-3,
            seed: int = 0, log=None, lr_final: float | None = None) -> TrainReport:
        """x_all BF16 [S][2nf], y_all FP32 normalised [S][2nf] on the device; the first
        n_train rows train, the rest validate.  With lr_final the learning rate follows a
        cosine from lr down to lr_final over all steps."""
        t = self.torch
        rng = np.random.default_rng(seed)
        rep = TrainReport(epochs=epochs, steps=0, seconds=0.0)
        t0 = time.perf_counter()
        S = int(x_all.shape[0])
        total = max(1, epochs * max(0, (n_train - batch) // batch + 1))
        for ep in range(epochs):
            perm = t.from_numpy(rng.permutation(n_train)).to(self.device)
            acc = []
            for s0 in range(0, n_train - batch + 1, batch):
                idx = perm[s0:s0 + batch]
                xb = x_all.index_select(0, idx)
                yb = y_all.index_select(0, idx)
                step_lr = lr
                if lr_final is not None:
                    step_lr = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * rep.steps / total))
                acc.append(self.train_step(xb, yb, lr=step_lr))
                rep.steps += 1
            tl = float(t.stack(acc).sum(dim=1).mean().item()) if acc else float("nan")
            vl = float("nan")
            if S > n_train:
                vparts = []
                for v0 in range(n_train, S, 4096):
                    v1 = min(S, v0 + 4096)
                    out = self.forward(x_all[v0:v1])
                    parts, _ = self.loss_and_grad(out, y_all[v0:v1])
                    vparts.append(float(parts.sum().item()) * (v1 - v0))
                vl = sum(vparts) / (S - n_train)
            rep.train_loss.append(tl)
            rep.val_loss.append(vl)
            if log:
                log(f"[warmstart] epoch {ep + 1}/{epochs}: train mse {tl:.3e}  val mse {vl:.3e}")
        t.cuda.synchronize()
        rep.seconds = time.perf_counter() - t0
        return rep

    # ------------------------------------------------------------------ inference
    def warm_v0(self, sbus, v_set):
        """Initial voltages [B][n][2] (device, FP64) from the network; v_set supplies the
        PV |V| and REF set-points (a flat-start array)."""
        t = self.torch
        B = int(v_set.shape[0])
        out = t.empty((B, 2 * self.nf), dtype=t.float32, device=self.device)
        for b0 in range(0, B, 65535):
            b1 = min(B, b0 + 65535)
            x = self.features(sbus[b0:b1], v_set[b0:b1])
            out[b0:b1] = self.forward(x)
        v0 = t.empty_like(v_set)
        for b0 in range(0, B, 65535):
            b1 = min(B, b0 + 65535)
            _check(lib().pf_mlp_warm_v0(b1 - b0, self.n, _vp(out[b0:b1].data_ptr()), _p(self.feat_bus_d), self.nf,
                                        _p(self.mu_y), _p(self.sd_y), _p(self.bus_type_d),
                                        _vp(v_set[b0:b1].data_ptr()), _vp(v0[b0:b1].data_ptr()), _stream()),
                   "pf_mlp_warm_v0")
        return v0

    def save(self, path):
        """Checkpoint: FP32 master weights and biases, the Adam moments and step count (so
        training resumes where it stopped), and the normalisation constants."""
        arrs = {}
        for l in range(len(self.W)):
            arrs[f"W{l}"] = self.W[l].cpu().numpy()
            arrs[f"b{l}"] = self.b[l].cpu().numpy()
            arrs[f"mW{l}"] = self.mW[l].cpu().numpy()
            arrs[f"vW{l}"] = self.vW[l].cpu().numpy()
            arrs[f"mb{l}"] = self.mb[l].cpu().numpy()
            arrs[f"vb{l}"] = self.vb[l].cpu().numpy()
        np.savez(path, dims=np.array(self.dims), feat_bus=self.feat_bus, adam_step=np.array(self.step),
                 mu_x=self.mu_x.cpu().numpy(), sd_x=self.sd_x.cpu().numpy(),
                 mu_y=self.mu_y.cpu().numpy(), sd_y=self.sd_y.cpu().numpy(), **arrs)

    def load(self, path):
        """Restores a checkpoint written by save() into a network of the same shape; plain
        arrays only (no pickled objects are read)."""
        d = np.load(path, allow_pickle=False)
        if list(d["dims"]) != list(self.dims):
            raise PfError(f"checkpoint dims {list(d['dims'])} differ from the network's {self.dims}")
        t = self.torch
        for l in range(len(self.W)):
            self.W[l].copy_(t.from_numpy(d[f"W{l}"]))
            self.b[l].copy_(t.from_numpy(d[f"b{l}"]))
            if f"mW{l}" in d:
                self.mW[l].copy_(t.from_numpy(d[f"mW{l}"]))
                self.vW[l].copy_(t.from_numpy(d[f"vW{l}"]))
                self.mb[l].copy_(t.from_numpy(d[f"mb{l}"]))
                self.vb[l].copy_(t.from_numpy(d[f"vb{l}"]))
        self.step = int(d["adam_step"]) if "adam_step" in d else 0
        self._refresh_bf16()
        self.set_normalization(d["mu_x"], d["sd_x"], d["mu_y"], d["sd_y"])


def targets_from_solution(net: WarmStartNet, v_sol: np.ndarray) -> np.ndarray:
    """(|V|, angle) of every feature bus from solved voltages [S][n][2] (host)."""
    return np.ascontiguousarray(v_sol[:, net.feat_bus, :].reshape(v_sol.shape[0], 2 * net.nf), dtype=np.float32)


def feature_stats(net: WarmStartNet, sbus: np.ndarray, v0: np.ndarray):
    """Mean and standard deviation of the raw features over a training set (host); a
    feature that never varies (PV set-points) gets sigma 1."""
    bt = net.bus_type_d.cpu().numpy()
    fb = net.feat_bus
    p = sbus[:, fb].real
    second = np.where(bt[fb][None, :] == PF_BUS_PV, v0[:, fb, 0], sbus[:, fb].imag)
    raw = np.stack([p, second], axis=2).reshape(sbus.shape[0], 2 * net.nf)
    mu = raw.mean(axis=0)
    sd = raw.std(axis=0)
    sd = np.where(sd > 1e-12, sd, 1.0)
    return mu.astype(np.float32), sd.astype(np.float32)


def target_stats(y: np.ndarray):
    mu = y.mean(axis=0)
    sd = y.std(axis=0)
    sd = np.where(sd > 1e-12, sd, 1.0)
    return mu.astype(np.float32), sd.astype(np.float32)


def solve_with_warm_start(plan: Plan, net: WarmStartNet, ybus, sbus, v_flat, tol=1e-8, max_iter=10,
                          precision=PF_FP64, workspace=None, fallback=True, **kw):
    """Warm-started solve: the network predicts the start, and with fallback an instance that
    fails from it restarts from the flat start inside the same kernel launch
    (pf_solve_batch_warm).  Returns the result."""
    v0 = net.warm_v0(sbus, v_flat)
    return solve_batch(plan, ybus, sbus, v0, tol=tol, max_iter=max_iter, precision=precision,
                       workspace=workspace, v_fallback=v_flat if fallback else None, **kw)

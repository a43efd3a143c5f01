"""Learned screen: training and screening on the device.

Orchestration only: every computation runs in libtt's kernels (features,
labels, the BF16 forward/backward GEMMs, loss, Adam, the reduced
enumeration with its exact check and fallback, support and histogram).
PyTorch supplies device memory, the batch shuffle and the stream.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import (  # noqa: F401
    AdamGroup,
    adam_step,
    cast_bf16,
    descriptors,
    device_descriptors,
    enumerate_device,
    layout,
    mlp_backward,
    mlp_forward,
    mlp_infer,
    mlp_loss,
    mlp_scratch_floats,
    screen_expand,
    screen_features,
    screen_labels,
    screen_infer,
    screen_infer_work_bytes,
    screen_run,
    screen_work_bytes,
    support_device,
)

DIMS = (32, 256, 256, 256, 12)


def _torch():
    import torch
    return torch


class ScreenNet:
    """The screening MLP: fp32 master weights with bf16 copies for the GEMMs."""

    def __init__(self, params, max_batch: int, device: str = "cuda"):
        torch = _torch()
        self.max_batch = int(max_batch)
        self.W32 = [torch.from_numpy(np.ascontiguousarray(W, np.float32)).to(device) for W, _ in params]
        self.b32 = [torch.from_numpy(np.ascontiguousarray(b, np.float32)).to(device) for _, b in params]
        self.Wb = [torch.empty(w.shape, dtype=torch.int16, device=device) for w in self.W32]
        for w32, wb in zip(self.W32, self.Wb):
            cast_bf16(w32, wb)
        self.gW = [torch.zeros_like(w) for w in self.W32]
        self.gb = [torch.zeros_like(b) for b in self.b32]
        self.mW = [torch.zeros_like(w) for w in self.W32]
        self.vW = [torch.zeros_like(w) for w in self.W32]
        self.mb = [torch.zeros_like(b) for b in self.b32]
        self.vb = [torch.zeros_like(b) for b in self.b32]
        B = self.max_batch
        self.acts = [torch.empty((B, d), dtype=torch.int16, device=device) for d in DIMS[1:-1]]
        self.z = torch.empty((B, DIMS[-1]), dtype=torch.float32, device=device)
        self.dz = torch.empty((B, DIMS[-1]), dtype=torch.int16, device=device)
        self.dh = [torch.empty((B, d), dtype=torch.int16, device=device) for d in DIMS[1:-1]]
        self.scratch = torch.empty(max(mlp_scratch_floats(B, max(DIMS)), 64), dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.steps = 0
        self.infer_work = None  # the gated inference's candidate list
        # one Adam launch for all eight parameter tensors
        self.adam = AdamGroup(self.W32 + self.b32, self.gW + self.gb, self.mW + self.mb, self.vW + self.vb,
                              self.Wb + [None] * 4)

    def forward(self, X, B: int):
        """Logits [B, 12] (fp32) for bf16 features X [B, 32]."""
        assert B <= self.max_batch
        h = X
        for l in range(4):
            if l < 3:
                mlp_forward(h, B, self.Wb[l], self.b32[l], relu=True, y_bf16=self.acts[l])
                h = self.acts[l]
            else:
                mlp_forward(h, B, self.Wb[l], self.b32[l], relu=False, y_f32=self.z)
        return self.z[:B]

    def infer(self, X, n: int, out=None):
        """Logits [n, 12] (fp32) for bf16 features X [n, 32] from one fused
        launch (tt_mlp_infer); any n."""
        torch = _torch()
        if out is None:
            out = torch.empty((n, DIMS[-1]), dtype=torch.float32, device="cuda")
        mlp_infer(X, n, self.Wb, self.b32, out)
        return out[:n]

    def infer_desc(self, d_desc, n: int, gated: bool, out, stream=None):
        """Logits of candidates straight from device descriptors (features
        computed in the kernel, tt_screen_infer); gated: only the candidates
        the screen's wave pass takes (their rows of out are written)."""
        work = None
        if gated:
            torch = _torch()
            need = screen_infer_work_bytes(n)
            if need and (self.infer_work is None or self.infer_work.numel() < need):
                self.infer_work = torch.empty(need, dtype=torch.uint8, device=out.device)
            work = self.infer_work if need else None
        screen_infer(d_desc, n, gated, self.Wb, self.b32, out, work=work, stream=stream)
        return out[:n]

    def backward(self, X, B: int):
        """Gradients of the loss whose dL/dz is in self.dz."""
        ins = [X] + self.acts
        g = self.dz
        for l in (3, 2, 1, 0):
            dx = self.dh[l - 1] if l > 0 else None
            mlp_backward(g, B, self.Wb[l], ins[l], relu_mask=l > 0, dx=dx, dw=self.gW[l], db=self.gb[l],
                         scratch=self.scratch)
            g = dx

    def train_step(self, X, y, m, h, B: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.forward(X, B)
        mlp_loss(self.z, B, y, m, h, self.dz, self.loss, self.scratch)
        self.backward(X, B)
        self.steps += 1
        self.adam.step(lr, beta1, beta2, eps, self.steps)
        return self.loss


@dataclass
class Candidates:
    """Device-resident candidate neurons with their table layout."""
    ns: object
    desc: np.ndarray
    d_desc: object
    total_words: int

    @property
    def n(self) -> int:
        return len(self.desc)


def candidates(ns) -> Candidates:
    desc = descriptors(ns)
    total = layout(desc)
    return Candidates(ns=ns, desc=desc, d_desc=device_descriptors(desc), total_words=total)


def exact_labels(c: Candidates):
    """Exact support / histogram by full enumeration, plus the training
    targets and features, all on the device."""
    torch = _torch()
    n = c.n
    tables = torch.empty(c.total_words, dtype=torch.int64, device="cuda")
    sup = torch.zeros(n, dtype=torch.uint8, device="cuda")
    hist = torch.zeros(n * 8, dtype=torch.int32, device="cuda")
    work = torch.empty(max(1, screen_work_bytes(n)), dtype=torch.uint8, device="cuda")
    screen_run(c.d_desc, n, None, 0.5, tables, sup, hist, work)
    X = torch.empty((n, 32), dtype=torch.int16, device="cuda")
    y = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    m = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    h = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    screen_features(c.d_desc, n, X)
    screen_labels(c.d_desc, n, sup, hist, y, m, h)
    return {"X": X, "y": y, "m": m, "h": h, "support": sup, "hist": hist, "tables": tables}


def train(net: ScreenNet, data, epochs: int, batch: int, lr: float, seed: int = 0, log=None):
    """Minibatch Adam with a cosine learning-rate decay; returns per-epoch
    mean loss."""
    torch = _torch()
    n = data["X"].shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        X, y, m, h = (data[key].index_select(0, perm) for key in ("X", "y", "m", "h"))
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        for s in range(steps_per_epoch):
            sl = slice(s * batch, (s + 1) * batch)
            cur = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * k / total)))
            acc += net.train_step(X[sl].contiguous(), y[sl].contiguous(), m[sl].contiguous(), h[sl].contiguous(),
                                  batch, cur)
            k += 1
        hist.append(float(acc.item()) / max(1, steps_per_epoch))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def predict(net: ScreenNet, X, n: int):
    """Logits [n, 12] from the fused inference kernel (one launch)."""
    return net.infer(X.contiguous(), n)


def support_accuracy(logits, y, m, tau: float):
    """Per-input accuracy of the predicted support over valid inputs, the
    fraction of neurons predicted exactly, and the fraction whose true
    support the prediction covers (those pass the exact check)."""
    torch = _torch()
    pred = (logits[:, :8] > math.log(tau / (1 - tau))).float()
    valid = m > 0
    correct = ((pred == y) | ~valid).all(1)
    bits = ((pred == y) & valid).sum().item() / max(1, valid.sum().item())
    covers = (((pred >= y) | ~valid).all(1)).float().mean().item()
    return {"bit_accuracy": bits, "exact_neurons": correct.float().mean().item(), "covers_support": covers}


class ScreenRunner:
    """Buffers for screening a fixed candidate set."""

    def __init__(self, c: Candidates):
        torch = _torch()
        n = c.n
        self.c = c
        self.tables = torch.empty(c.total_words, dtype=torch.int64, device="cuda")
        self.support = torch.zeros(n, dtype=torch.uint8, device="cuda")
        self.hist = torch.zeros(n * 8, dtype=torch.int32, device="cuda")
        self.mask = torch.zeros(n, dtype=torch.uint8, device="cuda")
        self.accept = torch.zeros(n, dtype=torch.uint8, device="cuda")
        self.status = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.work = torch.empty(max(1, screen_work_bytes(n)), dtype=torch.uint8, device="cuda")

    def plain(self):
        """Full enumeration + support/histogram (the method without the screen)."""
        screen_run(self.c.d_desc, self.c.n, None, 0.5, self.tables, self.support, self.hist, self.work,
                   status=self.status)

    def screened(self, logits=None, tau=0.5, force_mask=None):
        screen_run(self.c.d_desc, self.c.n, logits, tau, self.tables, self.support, self.hist, self.work,
                   force_mask=force_mask, mask=self.mask, accept=self.accept, status=self.status)

    def expand(self, out):
        screen_expand(self.c.d_desc, self.c.n, self.work, self.tables, out)


class LearnedScreen:
    """The learned screen end to end on a fixed candidate set: the network,
    fed straight from the descriptors, runs only for the candidates the wave
    pass takes (the lane pass settles the others under the zero-weight rule
    and never reads their logits), then the exact screen."""

    def __init__(self, net: ScreenNet, runner: ScreenRunner, tau: float):
        torch = _torch()
        self.net, self.runner, self.tau = net, runner, float(tau)
        self.logits = torch.zeros((runner.c.n, DIMS[-1]), dtype=torch.float32, device="cuda")

    def __call__(self):
        c = self.runner.c
        self.net.infer_desc(c.d_desc, c.n, True, self.logits)
        self.runner.screened(logits=self.logits, tau=self.tau)


def wave_pass_candidates(desc) -> np.ndarray:
    """Host mirror of the gate: candidates whose table reduced to the inputs of
    nonzero weight (full when every weight is nonzero) exceeds 64 rows."""
    F = desc["F"].astype(np.int64)
    b = desc["b"].astype(np.int64)
    live = (desc["w"] != 0) & (np.arange(8)[None, :] < F[:, None])
    k = live.sum(1)
    LF = np.where(k == F, F, np.maximum(k, 1))
    return LF * b > 6


def nonzero_weight_mask(c: Candidates):
    """The trivial screen: every input with a nonzero weight may matter."""
    torch = _torch()
    w = c.desc["w"].astype(np.int16)
    F = c.desc["F"].astype(np.int64)
    live = (w != 0) & (np.arange(8)[None, :] < F[:, None])
    bits = (live.astype(np.uint8) << np.arange(8, dtype=np.uint8)[None, :]).sum(1).astype(np.uint8)
    return torch.from_numpy(bits).cuda()


def row_cost(c: Candidates, mask: np.ndarray, accept: np.ndarray) -> int:
    """Row-evaluations of a screened pass: 2 * 2^(|S| b) per reduced
    candidate, plus 2^(F b) for every candidate enumerated in full."""
    total = 0
    for i in range(c.n):
        F, b = int(c.desc["F"][i]), int(c.desc["b"][i])
        k = bin(int(mask[i]) & ((1 << F) - 1)).count("1")
        if k == F:
            total += 1 << (F * b)
            continue
        total += 2 * (1 << (max(k, 1) * b))
        if not accept[i]:
            total += 1 << (F * b)
    return total


def timed(fn, reps: int = 5):
    torch = _torch()
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def timed_queued(fn, reps: int = 5):
    """GPU time alone: the launches are queued behind a ~20 ms spin, so the
    host's issue rate does not pace them."""
    torch = _torch()
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(50_000_000)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def wall(fn):
    torch = _torch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t

"""Helpers for the GPU parity tests (device buffers, poisoning, canaries)."""
from __future__ import annotations

import sys

import numpy as np

POISON = np.uint64(0xA5A5A5A5A5A5A5A5).view(np.int64)
CANARY = np.uint64(0x5EEDC0DE5EEDC0DE).view(np.int64)
N_CANARY = 64


def note(msg: str) -> None:
    """Name the case before a GPU step, so a fault can be traced to it."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def device_tables(total: int):
    """A poisoned table buffer followed by canary words."""
    import torch

    t = torch.empty(total + N_CANARY, dtype=torch.int64, device="cuda")
    t[:total].fill_(int(POISON))
    t[total:].fill_(int(CANARY))
    return t


def check_canary(t, total: int) -> None:
    tail = t[total:].cpu().numpy()
    assert (tail == CANARY).all(), "a kernel wrote past the table buffer"


def host_u64(t, lo: int = 0, hi=None) -> np.ndarray:
    x = t[lo:hi].cpu().numpy() if hi is not None else t[lo:].cpu().numpy()
    return x.view(np.uint64)


def neuron_planes(planes: np.ndarray, word_off: int, o: int, W: int):
    return [planes[word_off + p * W: word_off + (p + 1) * W] for p in range(o)]

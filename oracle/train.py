"""Training machinery: Adam and progressive tap pruning (Sec. IV-B, IV-C).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Adam (Sec. IV-B, Table I: learning rate 0.001) with the moment constants of
Kingma & Ba (beta1 = 0.9, beta2 = 0.999, eps = 1e-8; the paper is silent on them),
applied to real parameters -- the real and imaginary parts of every tap and the
per-step Kerr coefficients.

Pruning (Sec. IV-C): filters start at lengths T'_i and are shortened to T_i by
masking; every pruning event removes the two outermost taps of one filter.  The
paper only says that pruning more at the beginning works better.  Reading:
events go round-robin over the layers (each round shortens every filter still
above its target by one pair), and event e of E (e = 1..E) happens at iteration
floor(I_p (e/E)^2), I_p = frac * I_total (front-loaded).  Example 2 pins the event
count: five filters 11 -> 7 give 10 events.  Event timing: parity unpinned
(no schedule is printed).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


class Adam:
    """Plain Adam on a flat float64 parameter vector."""

    def __init__(self, nparam: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = np.zeros(nparam)
        self.v = np.zeros(nparam)
        self.t = 0

    def step(self, theta: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def pruning_events(t_init: Sequence[int], t_final: Sequence[int]) -> list[int]:
    """Ordered list of layer indices, one per pruning event (each removes one symmetric pair)."""
    cur = [int(t) for t in t_init]
    tgt = [int(t) for t in t_final]
    for a, b in zip(cur, tgt):
        assert a % 2 == 1 and b % 2 == 1 and a >= b >= 1
    events = []
    while any(a > b for a, b in zip(cur, tgt)):
        for i in range(len(cur)):
            if cur[i] > tgt[i]:
                cur[i] -= 2
                events.append(i)
    return events


def pruning_iterations(n_events: int, total_iters: int, frac: float = 0.2) -> list[int]:
    """Iteration at which each event fires: floor(I_p (e/E)^2), e = 1..E, I_p = frac * total_iters."""
    ip = frac * total_iters
    return [int(np.floor(ip * (e / n_events) ** 2)) for e in range(1, n_events + 1)]


def active_lengths(t_init: Sequence[int], events: Sequence[int], n_done: int) -> list[int]:
    """Current filter lengths after the first ``n_done`` events."""
    cur = [int(t) for t in t_init]
    for i in events[:n_done]:
        cur[i] -= 2
    return cur


def mask_taps(taps, lengths: Sequence[int]):
    """Zero all taps outside the centred window of the given active length."""
    out = []
    for h, t in zip(taps, lengths):
        h = np.array(h, dtype=np.complex128)
        K = (h.shape[0] - 1) // 2
        k = (int(t) - 1) // 2
        m = np.zeros_like(h)
        m[K - k:K + k + 1] = 1.0
        out.append(h * m)
    return out

"""Brute-force references for pinning the VATE oracle (test infrastructure).

* ``window_truth``: the exact quantity VATE estimates, |OP(aip, t-k'+1, k')|
  (Def. 1), by hash sets of distinct (aip, bip) pairs over the window.
* ``TSPool``: the plain 64-bit timestamp counter of Sec. 1 (the "TS" prior
  art): one last-set slice per pool slot.  Thm. 1 / Cor. 1 say the AT pool's
  CheckAT must agree with it exactly for every k' <= k, which makes it an
  independent check of the oracle's AT state machine (ACT clock, blocks,
  preservation schedule and Algorithm 3).
* ``virtual_std_error``: the delta-method standard error of the pool-shared
  (virtual) estimator, after linear counting's (Whang et al., cited in
  Sec. 2.1).  Used as an accuracy bound.
"""
from __future__ import annotations

import math

import numpy as np


def window_truth(slices: list[np.ndarray], t: int, kprime: int) -> dict[int, int]:
    """Distinct opposite hosts of every aip in W(t-k'+1, k') (Def. 1).

    slices[s] is the (P, 2) uint32 array of (aip, bip) pairs of slice s.
    """
    seen: dict[int, set[int]] = {}
    for s in range(max(0, t - kprime + 1), t + 1):
        for aip, bip in slices[s].reshape(-1, 2).tolist():
            seen.setdefault(aip, set()).add(bip)
    return {aip: len(b) for aip, b in seen.items()}


class TSPool:
    """64-bit last-set timestamp per pool slot (no expiry arithmetic at all)."""

    NEVER = np.iinfo(np.int64).min // 2

    def __init__(self, n_slots: int):
        self.last = np.full(n_slots, self.NEVER, dtype=np.int64)

    def set(self, pids: np.ndarray, t: int) -> None:
        self.last[np.asarray(pids, dtype=np.int64)] = t

    def active(self, t: int, kprime: int) -> np.ndarray:
        """Slot was set in one of the slices t-k'+1 .. t."""
        return (t - self.last) < kprime

    def age(self, t: int) -> np.ndarray:
        """t - last-set slice (huge for never-set slots)."""
        return t - self.last


def virtual_std_error(n: float, g: int, zp: float) -> float:
    """Delta-method standard error of n_hat/n for the virtual estimator
    g ln Z_p - g ln Z_v when each of the host's g VATs is independently
    inactive with probability q = Z_p e^{-n/g}: sd(n_hat) ~ sqrt(g(1-q)/q)."""
    q = zp * math.exp(-n / g)
    return math.sqrt(g * (1.0 - q) / q) / n


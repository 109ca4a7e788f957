"""CPU oracle of the learned estimator's network (test infrastructure only).

Plain numpy in float64 with the GPU kernels' BF16 rounding points written
out, so that the HIP forward/backward/Adam kernels can be compared with it:

  features x (64; see features()) -> z1 = W1 x + b1 -> a1 = GELU(z1) -> z2 = W2 a1 + b2
  -> a2 = GELU(z2) -> o = w3 . a2 + b3 + r,     n_hat = exp(o)

r is the log of the closed-form estimate (clamped below at 1), a fixed
residual branch, so that zero output weights reproduce the closed form.
BF16 rounding (round-to-nearest-even) is applied to x, W1, W2, a1 and a2 in
the forward pass and to the pre-activation gradients dz2, dz1 before the
products that use them, exactly where the GPU rounds operands for its
matrix-core instructions; everything else stays in float64 here.
GELU is the erf form 0.5 z (1 + erf(z / sqrt 2)) (Hendrycks & Gimpel).
Loss: mean relative error |exp(o - y) - 1|, y = ln(true cardinality).
Adam: Kingma & Ba (2015), bias-corrected, on float32 master weights.

The module itself is pinned in tests/test_mlp_oracle.py (GELU values from
the normal CDF, BF16 rounding cases, finite differences of the unrounded
network, the first Adam step).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

F = 64   # input features (k-bin histogram, live fraction, pool occupancy, zero pad)
HID = 64


def bf16_round(x) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  Works on the float32 bit pattern: add 0x7FFF plus the lowest kept
    bit, then clear the low 16 bits."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


@dataclass
class Params:
    W1: np.ndarray   # (HID, F)
    b1: np.ndarray   # (HID,)
    W2: np.ndarray   # (HID, HID)
    b2: np.ndarray   # (HID,)
    w3: np.ndarray   # (HID,)
    b3: float

    def copy(self) -> "Params":
        return Params(self.W1.copy(), self.b1.copy(), self.W2.copy(), self.b2.copy(),
                      self.w3.copy(), float(self.b3))

    def flat(self) -> dict:
        return {"W1": self.W1, "b1": self.b1, "W2": self.W2, "b2": self.b2,
                "w3": self.w3, "b3": np.array([self.b3])}


def init_params(seed: int, zero_out: bool = True) -> Params:
    """He-style init of the hidden layers; the output layer starts at zero so
    that the network starts equal to the closed form."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((HID, F)) * math.sqrt(2.0 / F)
    W2 = rng.standard_normal((HID, HID)) * math.sqrt(2.0 / HID)
    w3 = np.zeros(HID) if zero_out else rng.standard_normal(HID) * 0.05
    return Params(W1.astype(np.float32).astype(np.float64), np.zeros(HID),
                  W2.astype(np.float32).astype(np.float64), np.zeros(HID),
                  w3, 0.0)


def forward(p: Params, x, r, rounding: bool = True):
    """x: (B, F) features, r: (B,) residual.  Returns o and the cache."""
    rd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    xb = rd(x)
    W1b, W2b = rd(p.W1), rd(p.W2)
    z1 = xb @ W1b.T + p.b1
    a1 = rd(gelu(z1))
    z2 = a1 @ W2b.T + p.b2
    a2 = rd(gelu(z2))
    o = a2 @ p.w3 + p.b3 + np.asarray(r, dtype=np.float64)
    cache = dict(xb=xb, W1b=W1b, W2b=W2b, z1=z1, a1=a1, z2=z2, a2=a2)
    return o, cache


def loss_grad(o, y):
    """Mean relative error |exp(o - y) - 1| and its gradient w.r.t. o."""
    e = np.exp(np.asarray(o, dtype=np.float64) - np.asarray(y, dtype=np.float64))
    B = e.size
    loss = np.mean(np.abs(e - 1.0))
    do = np.sign(e - 1.0) * e / B
    return loss, do


def backward(p: Params, cache, do, rounding: bool = True) -> Params:
    rd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    do = np.asarray(do, dtype=np.float64)
    dw3 = cache["a2"].T @ do
    db3 = float(do.sum())
    da2 = np.outer(do, p.w3)
    dz2 = da2 * gelu_grad(cache["z2"])
    dz2b = rd(dz2)
    dW2 = dz2b.T @ cache["a1"]
    db2 = dz2.sum(axis=0)
    da1 = dz2b @ cache["W2b"]
    dz1 = da1 * gelu_grad(cache["z1"])
    dz1b = rd(dz1)
    dW1 = dz1b.T @ cache["xb"]
    db1 = dz1.sum(axis=0)
    return Params(dW1, db1, dW2, db2, dw3, db3)


@dataclass
class AdamState:
    m: Params
    v: Params
    t: int = 0


def adam_init(p: Params) -> AdamState:
    z = lambda a: np.zeros_like(a)
    zp = Params(z(p.W1), z(p.b1), z(p.W2), z(p.b2), z(p.w3), 0.0)
    return AdamState(zp, zp.copy(), 0)


def adam_step(p: Params, g: Params, st: AdamState, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8) -> None:
    """In-place Adam update of p (float64 arithmetic on float32-valued state)."""
    st.t += 1
    c1 = 1.0 - beta1 ** st.t
    c2 = 1.0 - beta2 ** st.t
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        gp = np.asarray(getattr(g, name), dtype=np.float64)
        m = beta1 * np.asarray(getattr(st.m, name)) + (1 - beta1) * gp
        v = beta2 * np.asarray(getattr(st.v, name)) + (1 - beta2) * gp * gp
        theta = np.asarray(getattr(p, name)) - lr * (m / c1) / (np.sqrt(v / c2) + eps)
        if name == "b3":
            setattr(st.m, name, float(m)); setattr(st.v, name, float(v)); setattr(p, name, float(theta))
        else:
            setattr(st.m, name, m); setattr(st.v, name, v); setattr(p, name, theta)


def features(hist: np.ndarray, live_k: np.ndarray, g: int, k: int, pool_occupancy: float,
             r: np.ndarray) -> np.ndarray:
    """(B, F) feature matrix from per-host distance histograms (B, k+1), live
    counts at window k, the pool's active fraction at window k, and
    r = ln(max(closed-form estimate, 1)) (entered as r / 16)."""
    B = hist.shape[0]
    x = np.zeros((B, F), dtype=np.float64)
    x[:, :k] = hist[:, :k] / g
    x[:, k] = np.asarray(live_k, dtype=np.float64) / g
    x[:, k + 1] = pool_occupancy
    x[:, k + 2] = np.asarray(r, dtype=np.float64) / 16.0
    return x

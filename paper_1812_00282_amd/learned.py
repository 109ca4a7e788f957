"""Python face of the learned estimator kernels (include/vate_mlp.h).

theta is a float32 tensor of MLP_PARAMS values laid out as
W1[64][64], b1[64], W2[64][64], b2[64], w3[64], b3; feature matrices are
int16 tensors holding bf16 bit patterns, [n][64].
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import MLP_FEATURES, MLP_PARAMS, MLP_WEIGHT_BYTES, VateMlpEnvelope, check, lib
from .sketch import Sketch, _stream_handle, as_u32_tensor

OFFSETS = {"W1": (0, (64, 64)), "b1": (4096, (64,)), "W2": (4160, (64, 64)),
           "b2": (8256, (64,)), "w3": (8320, (64,)), "b3": (8384, ())}


def theta_from(params: dict) -> np.ndarray:
    """Flatten {W1, b1, W2, b2, w3, b3} into the float32 theta layout."""
    th = np.zeros(MLP_PARAMS, dtype=np.float32)
    for k, (off, shape) in OFFSETS.items():
        v = np.asarray(params[k], dtype=np.float32).reshape(-1)
        th[off:off + v.size] = v
    return th


def params_from(theta) -> dict:
    th = theta.detach().cpu().numpy() if isinstance(theta, torch.Tensor) else np.asarray(theta)
    out = {}
    for k, (off, shape) in OFFSETS.items():
        n = int(np.prod(shape)) if shape else 1
        v = th[off:off + n].astype(np.float64)
        out[k] = v.reshape(shape) if shape else float(v[0])
    return out


def new_weights(device="cuda") -> torch.Tensor:
    # the caching allocator returns >= 512-byte aligned blocks
    return torch.empty(MLP_WEIGHT_BYTES, dtype=torch.uint8, device=device)


def pack(theta: torch.Tensor, weights: torch.Tensor, stream=None) -> torch.Tensor:
    check(lib().vate_mlp_pack(theta.data_ptr(), weights.data_ptr(), _stream_handle(stream)))
    return weights


def set_envelope(weights: torch.Tensor, env: dict | None, stream=None) -> torch.Tensor:
    """Set the network's training envelope on packed weights (None clears it):
    env = {"k", "g", "log2_pool", "width", "lo": 64 floats, "hi": 64 floats}.
    Zeroes the fallback counter."""
    if env is None:
        check(lib().vate_mlp_set_envelope(weights.data_ptr(), None, _stream_handle(stream)))
        return weights
    e = VateMlpEnvelope(int(env["k"]), int(env["g"]), int(env["log2_pool"]), int(env["width"]),
                        (ctypes.c_float * 64)(*np.asarray(env["lo"], dtype=np.float32).tolist()),
                        (ctypes.c_float * 64)(*np.asarray(env["hi"], dtype=np.float32).tolist()))
    check(lib().vate_mlp_set_envelope(weights.data_ptr(), ctypes.byref(e), _stream_handle(stream)))
    return weights


def fallbacks(weights: torch.Tensor, reset: bool = False, stream=None) -> int:
    """Hosts the envelope (or a non-finite output) sent to the closed form."""
    c = ctypes.c_uint64()
    check(lib().vate_mlp_fallbacks(weights.data_ptr(), ctypes.byref(c), int(reset), _stream_handle(stream)))
    return c.value


def forward(weights, x: torch.Tensor, r: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    n = x.shape[0]
    o = out if out is not None else torch.empty(n, dtype=torch.float32, device=x.device)
    check(lib().vate_mlp_forward(weights.data_ptr(), x.data_ptr(), r.data_ptr(), n,
                                 o.data_ptr(), _stream_handle(stream)))
    return o


def train_step(weights, x, r, y, grad, loss, stream=None) -> None:
    check(lib().vate_mlp_train_step(weights.data_ptr(), x.data_ptr(), r.data_ptr(), y.data_ptr(),
                                    x.shape[0], grad.data_ptr(), loss.data_ptr(),
                                    _stream_handle(stream)))


def adam(theta, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
         stream=None) -> None:
    check(lib().vate_mlp_adam(theta.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                              step, lr, beta1, beta2, eps, _stream_handle(stream)))


def fill(t: torch.Tensor, value: float = 0.0, stream=None) -> None:
    check(lib().vate_mlp_fill(t.data_ptr(), t.numel(), value, _stream_handle(stream)))


def features(hist: torch.Tensor, est: torch.Tensor, k: int, g: int, occupancy: float,
             stream=None):
    n = hist.shape[0]
    x = torch.empty((n, MLP_FEATURES), dtype=torch.int16, device=hist.device)
    r = torch.empty(n, dtype=torch.float32, device=hist.device)
    check(lib().vate_mlp_features(hist.data_ptr(), est.data_ptr(), n, k, g, occupancy,
                                  x.data_ptr(), r.data_ptr(), _stream_handle(stream)))
    return x, r


def learned_workspace(sk: Sketch, n_hosts: int) -> torch.Tensor:
    b = ctypes.c_size_t()
    check(lib().vate_estimate_learned_workspace_bytes(sk.handle, n_hosts, ctypes.byref(b)), sk.handle)
    ws = getattr(sk, "_lws", None)
    if ws is None or ws.numel() < b.value:
        ws = torch.empty(b.value, dtype=torch.uint8, device=sk.device)
        sk._lws = ws
    return ws


def estimate_learned(sk: Sketch, hosts, weights, stream=None, out=None, partitioned=False):
    """(learned estimates, closed-form estimates) at window k for all hosts.

    partitioned=True uses vate_estimate_learned_ws (locality-ordered lookups)
    with a workspace cached on the sketch."""
    ht = as_u32_tensor(hosts, sk.device)
    n = ht.numel()
    if out is None:
        est = torch.empty(n, dtype=torch.float32, device=sk.device)
        cf = torch.empty(n, dtype=torch.float32, device=sk.device)
    else:
        est, cf = out
    args = (sk.handle, ht.data_ptr() if n else None, n, weights.data_ptr(),
            est.data_ptr() if n else None, cf.data_ptr() if n else None)
    if partitioned and n:
        ws = learned_workspace(sk, n)
        check(lib().vate_estimate_learned_ws(*args, ws.data_ptr(), ws.numel(),
                                             _stream_handle(stream)), sk.handle)
    else:
        check(lib().vate_estimate_learned(*args, _stream_handle(stream)), sk.handle)
    sk._keep_h = ht
    return est, cf


def estimate_learned_run(sk: Sketch, weights, stream=None, out=None):
    """estimate_learned for the hosts planned with sk.plan(...)
    (vate_estimate_learned_run)."""
    n = sk._plan_n
    if out is None:
        est = torch.empty(n, dtype=torch.float32, device=sk.device)
        cf = torch.empty(n, dtype=torch.float32, device=sk.device)
    else:
        est, cf = out
    check(lib().vate_estimate_learned_run(sk.handle, n, weights.data_ptr(), est.data_ptr(), cf.data_ptr(),
                                          sk._pws.data_ptr(), sk._pws.numel(), _stream_handle(stream)),
          sk.handle)
    return est, cf


def mfma_selftest(a_bf16: torch.Tensor, b_bf16: torch.Tensor) -> torch.Tensor:
    d = torch.empty((16, 16), dtype=torch.float32, device=a_bf16.device)
    check(lib().vate_mlp_mfma_selftest(a_bf16.data_ptr(), b_bf16.data_ptr(), d.data_ptr(),
                                       _stream_handle(None)))
    return d

"""Python face of one VATE sketch on the GPU.

PyTorch provides the device memory (pool, state, inputs, outputs) and the
stream; the library's kernels do the work.  Tensors holding 32-bit IDs are
int32 tensors whose bits are the unsigned values.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import VateParams, check, lib


def _stream_handle(stream: torch.cuda.Stream | None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def as_u32_tensor(x, device) -> torch.Tensor:
    """uint32 numpy array / int32 tensor -> contiguous int32 tensor on device."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint32).view(np.int32))
    if x.dtype != torch.int32:
        raise TypeError("expected uint32 numpy data or an int32 tensor")
    return x.to(device, non_blocking=True).contiguous()


@dataclass(frozen=True)
class Config:
    log2_pool: int
    width: int
    k: int
    g: int
    partition: int = 0
    seed_a: int = 0
    seed_b: int = 0
    counter: int = 0      # 0: asynchronous timestamps (VATE); 1: distance recorders (VDRE)
    block_log2: int = 0   # 0: independent VATs (the paper's H); b > 0: locality-blocked H

    def params(self) -> VateParams:
        return VateParams(self.log2_pool, self.width, self.k, self.g, self.partition,
                          self.seed_a & 0xFFFFFFFF, self.seed_b & 0xFFFFFFFF, self.counter,
                          self.block_log2)


def state_bytes(cfg: Config) -> tuple[int, int]:
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    p = cfg.params()
    check(lib().vate_state_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(sb)))
    return pb.value, sb.value


class Sketch:
    """One VATE sketch: ingest* -> close_slice -> estimate* per time slice."""

    def __init__(self, cfg: Config, device="cuda", stream: torch.cuda.Stream | None = None):
        self.cfg = cfg
        self.device = torch.device(device)
        self.pool_bytes, self.state_bytes = state_bytes(cfg)
        self.pool = torch.empty(self.pool_bytes, dtype=torch.uint8, device=self.device)
        self.state = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        self._p = cfg.params()
        h = ctypes.c_void_p()
        check(lib().vate_create(ctypes.byref(self._p), self.pool.data_ptr(), self.state.data_ptr(),
                                _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().vate_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def ingest(self, pairs, stream=None) -> None:
        """pairs: (n, 2) uint32 (aip, bip) as numpy or int32 tensor."""
        t = as_u32_tensor(pairs, self.device).reshape(-1)
        n = t.numel() // 2
        check(lib().vate_ingest(self._h, t.data_ptr() if n else None, n, _stream_handle(stream)),
              self._h)
        self._keep = t          # keep the input alive until the stream reaches it

    def close_slice(self, stream=None) -> None:
        check(lib().vate_close_slice(self._h, _stream_handle(stream)), self._h)

    def workspace_bytes(self, n_hosts: int) -> int:
        b = ctypes.c_size_t()
        check(lib().vate_estimate_workspace_bytes(self._h, n_hosts, ctypes.byref(b)), self._h)
        return b.value

    def _workspace(self, n_hosts: int) -> torch.Tensor:
        need = self.workspace_bytes(n_hosts)
        ws = getattr(self, "_ws", None)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws = ws
        return ws

    def estimate(self, hosts, kprime: int | None = None, want_live: bool = True,
                 want_hist: bool = False, stream=None, out=None, partitioned: bool = False):
        """Returns (est float32, live int32 or None, hist int32 (n, k+1) or None).

        partitioned=True uses vate_estimate_ws (locality-ordered lookups) with a
        workspace cached on the sketch; otherwise vate_estimate."""
        ht = as_u32_tensor(hosts, self.device)
        n = ht.numel()
        kp = self.cfg.k if kprime is None else kprime
        if out is not None:
            est, live, hist = out
        else:
            est = torch.empty(n, dtype=torch.float32, device=self.device)
            live = torch.empty(n, dtype=torch.int32, device=self.device) if want_live else None
            hist = (torch.empty((n, self.cfg.k + 1), dtype=torch.int32, device=self.device)
                    if want_hist else None)
        args = (self._h, ht.data_ptr() if n else None, n, kp,
                est.data_ptr() if n else None,
                live.data_ptr() if (live is not None and n) else None,
                hist.data_ptr() if (hist is not None and n) else None)
        if partitioned and n:
            ws = self._workspace(n)
            check(lib().vate_estimate_ws(*args, ws.data_ptr(), ws.numel(), _stream_handle(stream)),
                  self._h)
        else:
            check(lib().vate_estimate(*args, _stream_handle(stream)), self._h)
        self._keep_h = ht
        return est, live, hist

    def plan(self, hosts, stream=None) -> None:
        """Hash and sort the VATs of a host list that stays the same across
        slices (vate_estimate_plan); estimate_run / learned.estimate_learned_run
        then answer each closed slice from the plan.  The plan lives in a
        workspace owned by the sketch, sized for the learned estimate too."""
        ht = as_u32_tensor(hosts, self.device)
        n = ht.numel()
        b = ctypes.c_size_t()
        check(lib().vate_estimate_learned_workspace_bytes(self._h, n, ctypes.byref(b)), self._h)
        if getattr(self, "_pws", None) is None or self._pws.numel() < b.value:
            self._pws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        check(lib().vate_estimate_plan(self._h, ht.data_ptr(), n, self._pws.data_ptr(), self._pws.numel(),
                                       _stream_handle(stream)), self._h)
        self._plan_n = n
        self._keep_plan_hosts = ht

    def estimate_run(self, kprime: int | None = None, want_live: bool = True, want_hist: bool = False,
                     stream=None, out=None):
        """vate_estimate_run: the outputs of estimate(...) for the planned hosts."""
        n = self._plan_n
        kp = self.cfg.k if kprime is None else kprime
        if out is not None:
            est, live, hist = out
        else:
            est = torch.empty(n, dtype=torch.float32, device=self.device)
            live = torch.empty(n, dtype=torch.int32, device=self.device) if want_live else None
            hist = (torch.empty((n, self.cfg.k + 1), dtype=torch.int32, device=self.device)
                    if want_hist else None)
        check(lib().vate_estimate_run(self._h, n, kp, est.data_ptr(),
                                      live.data_ptr() if live is not None else None,
                                      hist.data_ptr() if hist is not None else None,
                                      self._pws.data_ptr(), self._pws.numel(), _stream_handle(stream)), self._h)
        return est, live, hist

    def estimate_windows(self, hosts, kprimes, stream=None) -> torch.Tensor:
        """Estimates for several windows (ascending k' values) from one pass:
        float32 tensor [hosts][windows]."""
        ht = as_u32_tensor(hosts, self.device)
        n = ht.numel()
        kp = np.ascontiguousarray(kprimes, dtype=np.uint32)
        est = torch.empty((n, kp.size), dtype=torch.float32, device=self.device)
        if n == 0:
            return est
        b = ctypes.c_size_t()
        check(lib().vate_estimate_multi_workspace_bytes(self._h, n, ctypes.byref(b)), self._h)
        ws = getattr(self, "_mws", None)
        if ws is None or ws.numel() < b.value:
            ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
            self._mws = ws
        check(lib().vate_estimate_multi_ws(self._h, ht.data_ptr(), n, kp.ctypes.data, kp.size,
                                           est.data_ptr(), ws.data_ptr(), ws.numel(),
                                           _stream_handle(stream)), self._h)
        self._keep_h = ht
        return est

    def census(self, stream=None) -> np.ndarray:
        out = np.zeros(self.cfg.k + 1, dtype=np.uint64)
        check(lib().vate_read_census(self._h, out.ctypes.data, _stream_handle(stream)), self._h)
        return out

    def read_state(self, stream=None):
        """(pool bytes as numpy uint8, t, bact0, closed)."""
        pool = np.empty(self.pool_bytes, dtype=np.uint8)
        t, b, c = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_int()
        check(lib().vate_read_state(self._h, pool.ctypes.data, ctypes.byref(t), ctypes.byref(b),
                                    ctypes.byref(c), _stream_handle(stream)), self._h)
        return pool, t.value, b.value, bool(c.value)

    def load_state(self, pool: np.ndarray, t: int, bact0: int, closed: bool, stream=None) -> None:
        src = torch.from_numpy(np.ascontiguousarray(pool, dtype=np.uint8)).to(self.device)
        check(lib().vate_load_state(self._h, src.data_ptr(), t, bact0, int(closed),
                                    _stream_handle(stream)), self._h)
        self._keep_pool = src


def host_hash(cfg: Config, which: int, x: int, i: int = 0) -> int:
    p = cfg.params()
    return lib().vate_host_hash(ctypes.byref(p), which, x & 0xFFFFFFFF, i)


def host_block(cfg: Config, pid: int) -> int:
    p = cfg.params()
    return lib().vate_host_block(ctypes.byref(p), pid)

"""Python face of the batched VATE path (include/vate_batch.h).

A Batch drives several Sketch objects through each time slice with one
persistent launch per phase, optionally replaying a captured hipGraph, with
launch shapes from the library's autotuner.  All of a batch's work runs on
its own (default-priority) stream.
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

from ._lib import VateBatchTune, VateError, lib
from .sketch import Sketch, as_u32_tensor


def _check(rc: int, handle) -> None:
    if rc != 0:
        msg = (lib().vate_batch_last_error(handle) or b"").decode() if handle else ""
        raise VateError(rc, msg or lib().vate_status_string(rc).decode())


class Batch:
    def __init__(self, sketches: list[Sketch], pair_capacity: list[int], hosts: list,
                 kprime: list[int] | None = None, want_live: bool = True):
        S = len(sketches)
        self.sketches = sketches
        self.device = sketches[0].device
        self.stream = torch.cuda.Stream(device=self.device)
        b = ctypes.c_size_t()
        _check(lib().vate_batch_bytes(S, ctypes.byref(b)), None)
        self.block = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self.n_pairs = torch.zeros(S, dtype=torch.int64, device=self.device)
        self.pairs = [torch.empty((max(int(c), 1), 2), dtype=torch.int32, device=self.device)
                      for c in pair_capacity]
        self.hosts = [as_u32_tensor(h, self.device) for h in hosts]
        self.est = [torch.zeros(h.numel(), dtype=torch.float32, device=self.device) for h in self.hosts]
        self.live = [torch.zeros(h.numel(), dtype=torch.int32, device=self.device) if want_live else None
                     for h in self.hosts]
        handles = (ctypes.c_void_p * S)(*[s.handle.value for s in sketches])
        h = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        _check(lib().vate_batch_create(handles, S, self.block.data_ptr(), self.n_pairs.data_ptr(),
                                       ctypes.byref(h)), None)
        self._h = h
        self.kprime = [s.cfg.k if kprime is None else kprime[i] for i, s in enumerate(sketches)]
        for i, s in enumerate(sketches):
            kp = self.kprime[i]
            lv = self.live[i]
            _check(lib().vate_batch_set_io(h, i, self.pairs[i].data_ptr(), self.pairs[i].shape[0],
                                           self.hosts[i].data_ptr(),
                                           self.hosts[i].numel(), kp, self.est[i].data_ptr(),
                                           lv.data_ptr() if lv is not None else None), h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().vate_batch_destroy(h)
            self._h = None

    def load(self, slices: list) -> None:
        """Copy this slice's packets ((n_i, 2) uint32 / int32 each) into the
        fixed pair buffers and set the counts (on the batch's stream)."""
        counts = []
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            for buf, sl in zip(self.pairs, slices):
                t = as_u32_tensor(sl, self.device).reshape(-1, 2)
                if t.shape[0] > buf.shape[0]:
                    raise ValueError("slice larger than the pair buffer")
                buf[: t.shape[0]].copy_(t, non_blocking=True)
                counts.append(t.shape[0])
            self.n_pairs.copy_(torch.tensor(counts, dtype=torch.int64), non_blocking=False)

    def slice(self) -> None:
        _check(lib().vate_batch_slice(self._h, self.stream.cuda_stream), self._h)

    def capture(self) -> None:
        _check(lib().vate_batch_capture(self._h, self.stream.cuda_stream), self._h)

    def replay(self) -> None:
        _check(lib().vate_batch_replay(self._h, self.stream.cuda_stream), self._h)

    def synchronize(self) -> None:
        self.stream.synchronize()

    def get_tune(self) -> dict:
        t = VateBatchTune()
        _check(lib().vate_batch_get_tune(self._h, ctypes.byref(t)), self._h)
        return {n: getattr(t, n) for n, _ in VateBatchTune._fields_}

    def set_tune(self, tune: dict) -> None:
        """Set launch shapes; fields missing from `tune` keep their values."""
        cur = self.get_tune()
        cur.update(tune)
        t = VateBatchTune(**cur)
        _check(lib().vate_batch_set_tune(self._h, ctypes.byref(t)), self._h)

    def geometry_key(self) -> str:
        """What a tuned launch shape depends on: the device (name, CUs) and,
        per member, pool size, width, window, g, counter kind, hosts, window
        estimated and pair capacity."""
        props = torch.cuda.get_device_properties(self.device)
        parts = [f"{props.name}/{props.multi_processor_count}cu"]
        for s, h, buf, kp in zip(self.sketches, self.hosts, self.pairs, self.kprime):
            c = s.cfg
            parts.append(f"c{c.log2_pool}w{c.width}k{c.k}g{c.g}x{c.counter}b{c.block_log2}"
                         f"h{h.numel()}kp{kp}p{buf.shape[0]}")
        return "|".join(parts)

    def autotune(self, cache: str | None = None, key: str | None = None) -> dict:
        """Run the library's autotuner on the current slice and return its
        report ("candidates", "best", "tune").  With a JSON file `cache`, a
        choice stored there under `key` (default: geometry_key()) is set
        instead ({"cached": True, "tune": ...}); a new choice is stored."""
        if cache and key is None:
            key = self.geometry_key()
        if cache and os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
            if key in known:
                self.set_tune(known[key])
                return {"cached": True, "key": key, "tune": self.get_tune()}
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().vate_batch_autotune(self._h, self.stream.cuda_stream, buf, len(buf)), self._h)
        rep = json.loads(buf.value.decode())
        rep["tune"] = self.get_tune()
        rep["cached"] = False
        if cache:
            rep["key"] = key
            known = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    known = json.load(f)
            known[key] = rep["tune"]
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(known, f, indent=1)
            os.replace(tmp, cache)
        return rep

"""ctypes wrapper around the plain-C VATE oracle (``oracle/vate_oracle.c``).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to check the HIP path.  It shares no code with the
HIP library (``paper_1812_00282_amd``) and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vate_oracle.c")
_LIB = os.path.join(_HERE, "libvate_oracle.so")

_u32, _u64, _i32, _dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
_vp = ctypes.c_void_p


def build_lib() -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation pragmas)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", _SRC,
                           "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_lib()
        L = ctypes.CDLL(_LIB)
        sig = {
            "o_fmix32": (_u32, [_u32]),
            "o_hash_BH": (_u32, [_u32, _u32, _u32]),
            "o_hash_H": (_u32, [_u32, _u32, _u32, _u32]),
            "o_hash_H_blocked": (_u32, [_u32, _u32, _u32, _u32, _u32]),
            "o_BH": (_u32, [_vp, _u32]),
            "o_H": (_u32, [_vp, _u32, _u32]),
            "o_block_of": (_u32, [_vp, _u64]),
            "o_block_act": (_u32, [_vp, _u32]),
            "o_act_of": (_u32, [_vp, _u64]),
            "o_checkAT": (_i32, [_u32, _u32, _u32, _u32]),
            "o_preserve_general": (_u32, [_u32, _u32, _u32]),
            "o_preserve_fast": (_u32, [_u32, _u32, _u32]),
            "o_create": (_vp, [_u32, _u32, _u32, _u32, _u32, _u32, _u32, _u32, _u32]),
            "o_checkDR": (_i32, [_u32, _u32]),
            "o_destroy": (None, [_vp]),
            "o_ingest": (None, [_vp, _vp, _u64]),
            "o_close": (None, [_vp]),
            "o_packet_pids": (None, [_vp, _vp, _u64, _vp]),
            "o_census": (None, [_vp, _vp]),
            "o_pool_inactive": (_u64, [_vp, _u32]),
            "o_estimate_counts": (_dbl, [_u64, _u64, _u32, _u64]),
            "o_estimate": (_i32, [_vp, _vp, _u64, _u32, _vp, _vp, _vp]),
            "o_N": (_u64, [_vp]),
            "o_t": (_u64, [_vp]),
            "o_bact0": (_u32, [_vp]),
            "o_closed": (_i32, [_vp]),
            "o_blk_start": (_u64, [_vp, _u32]),
            "o_values": (None, [_vp, _vp]),
            "o_set_values": (None, [_vp, _vp, _u64, _u32, _i32]),
            "o_pack_pool": (None, [_vp, _vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def fmix32(x: int) -> int:
    return lib().o_fmix32(x & 0xFFFFFFFF)


def hash_BH(g: int, seed_b: int, bip: int) -> int:
    return lib().o_hash_BH(g, seed_b & 0xFFFFFFFF, bip & 0xFFFFFFFF)


def hash_H(c: int, seed_a: int, aip: int, i: int) -> int:
    return lib().o_hash_H(c, seed_a & 0xFFFFFFFF, aip & 0xFFFFFFFF, i)


def hash_H_blocked(c: int, b: int, seed_a: int, aip: int, i: int) -> int:
    return lib().o_hash_H_blocked(c, b, seed_a & 0xFFFFFFFF, aip & 0xFFFFFFFF, i)


def check_at(value: int, act: int, k: int, kprime: int) -> bool:
    return bool(lib().o_checkAT(value, act, k, kprime))


def preserve_fast(value: int, act: int, k: int) -> int:
    return lib().o_preserve_fast(value, act, k)


def preserve_general(value: int, act: int, k: int) -> int:
    return lib().o_preserve_general(value, act, k)


def estimate_counts(u_v: int, u_p: int, g: int, N: int) -> float:
    return lib().o_estimate_counts(u_v, u_p, g, N)


class OracleSketch:
    """One VATE sketch on the CPU; same call sequence as the C-ABI library."""

    def __init__(self, log2_pool: int, width: int, k: int, g: int,
                 seed_a: int = 0, seed_b: int = 0, partition: int = 0, counter: int = 0,
                 block_log2: int = 0):
        """counter 0: asynchronous timestamps (VATE); 1: distance recorders
        (VDRE, full-pool maintenance every slice).  block_log2 > 0 selects
        the locality-blocked H (blocks of 2^block_log2 consecutive VATs)."""
        self.c, self.w, self.k, self.g = log2_pool, width, k, g
        self.partition, self.counter, self.block_log2 = partition, counter, block_log2
        self._s = lib().o_create(log2_pool, width, k, g, seed_a & 0xFFFFFFFF,
                                 seed_b & 0xFFFFFFFF, partition, counter, block_log2)
        if not self._s:
            raise ValueError("invalid oracle sketch parameters")
        self.N = lib().o_N(self._s)

    def __del__(self):
        s = getattr(self, "_s", None)
        if s:
            lib().o_destroy(s)
            self._s = None

    # --- the method's steps ---
    def ingest(self, pairs: np.ndarray) -> None:
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1)
        assert pairs.size % 2 == 0
        lib().o_ingest(self._s, _ptr(pairs), pairs.size // 2)

    def close_slice(self) -> None:
        lib().o_close(self._s)

    def estimate(self, hosts: np.ndarray, kprime: int | None = None,
                 want_live: bool = True, want_hist: bool = False):
        hosts = np.ascontiguousarray(hosts, dtype=np.uint32)
        kp = self.k if kprime is None else kprime
        est = np.zeros(hosts.size, dtype=np.float64)
        live = np.zeros(hosts.size, dtype=np.uint32) if want_live else None
        hist = np.zeros((hosts.size, self.k + 1), dtype=np.uint32) if want_hist else None
        rc = lib().o_estimate(self._s, _ptr(hosts), hosts.size, kp, _ptr(est),
                              _ptr(live) if live is not None else None,
                              _ptr(hist) if hist is not None else None)
        if rc != 0:
            raise RuntimeError("oracle estimate: slice not closed or k' out of range")
        return est, live, hist

    def census(self) -> np.ndarray:
        h = np.zeros(self.k + 1, dtype=np.uint64)
        lib().o_census(self._s, _ptr(h))
        return h

    def pool_inactive(self, kprime: int) -> int:
        return lib().o_pool_inactive(self._s, kprime)

    # --- hashing / blocks (exported for the pins) ---
    def BH(self, bip: int) -> int:
        return lib().o_BH(self._s, bip & 0xFFFFFFFF)

    def H(self, aip: int, i: int) -> int:
        return lib().o_H(self._s, aip & 0xFFFFFFFF, i)

    def packet_pids(self, pairs: np.ndarray) -> np.ndarray:
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1)
        out = np.zeros(pairs.size // 2, dtype=np.uint32)
        lib().o_packet_pids(self._s, _ptr(pairs), pairs.size // 2, _ptr(out))
        return out

    def block_of(self, pid: int) -> int:
        return lib().o_block_of(self._s, pid)

    def block_act(self, i: int) -> int:
        return lib().o_block_act(self._s, i)

    def act_of(self, pid: int) -> int:
        return lib().o_act_of(self._s, pid)

    def blk_start(self, i: int) -> int:
        return lib().o_blk_start(self._s, i)

    # --- state ---
    @property
    def t(self) -> int:
        return lib().o_t(self._s)

    @property
    def bact0(self) -> int:
        return lib().o_bact0(self._s)

    @property
    def closed(self) -> bool:
        return bool(lib().o_closed(self._s))

    def values(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.uint16)
        lib().o_values(self._s, _ptr(out))
        return out

    def set_values(self, vals: np.ndarray, t: int, bact0: int, closed: bool) -> None:
        vals = np.ascontiguousarray(vals, dtype=np.uint16)
        assert vals.size == self.N
        lib().o_set_values(self._s, _ptr(vals), t, bact0, int(closed))

    def packed_pool(self) -> np.ndarray:
        out = np.zeros(self.N * self.w // 8, dtype=np.uint8)
        lib().o_pack_pool(self._s, _ptr(out))
        return out

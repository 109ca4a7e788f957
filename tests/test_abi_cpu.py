"""Host-side checks of libvate.so (no GPU compute): exported symbols, parameter
validation, and the library's hash and block functions (the same inline code
its kernels run) against the CPU oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import vate_ref
from oracle.vate_ref import OracleSketch
from paper_1812_00282_amd import _lib
from paper_1812_00282_amd.sketch import Config, host_block, host_hash, state_bytes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(vate_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    # the binding declares a signature for each one
    assert declared <= set(_lib.exported_symbols())


@pytest.mark.parametrize("bad", [
    dict(log2_pool=0), dict(log2_pool=33), dict(width=0), dict(width=17), dict(k=0),
    dict(width=3, k=4),                                   # 2^3 < 2k+1
    dict(log2_pool=4, width=5, k=2),                      # exact packing needs >= 32 counters
    dict(width=4, k=8), dict(width=8, k=128), dict(g=0), dict(g=65536),
    dict(partition=2), dict(log2_pool=3, k=3, width=4),   # 2^3 < 2k
    dict(log2_pool=4, width=4, k=1),                      # pool of 8 bytes < 16
    dict(width=4, k=16, counter=1),                       # DR needs 2^w >= k+1
])
def test_invalid_params_rejected(bad):
    base = dict(log2_pool=16, width=8, k=4, g=128)
    base.update(bad)
    cfg = Config(**base)
    with pytest.raises(_lib.VateError) as e:
        state_bytes(cfg)
    assert e.value.code == _lib.VATE_E_INVAL


def test_counter_kind_validated():
    p = Config(16, 8, 4, 128).params()
    p.counter = 2
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    assert _lib.lib().vate_state_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(sb)) == _lib.VATE_E_INVAL


def test_exact_widths_accepted():
    """Any width of 1..16 bits that holds the counter's range is accepted;
    widths other than 4/8/16 pack the counters exactly (the paper's pool:
    ceil(log2(2k+1)) bits per AT, Sec. 3)."""
    for k in (1, 2, 3, 60, 300, 1000):
        w = (2 * k).bit_length()            # ceil(log2(2k+1))
        assert state_bytes(Config(16, w, k, 64))[0] == (1 << 16) * w // 8
        wd = k.bit_length()                 # ceil(log2(k+1)) for a DR
        assert state_bytes(Config(16, wd, k, 64, counter=1))[0] == (1 << 16) * wd // 8


def test_dr_width_rule():
    """A DR needs ceil(log2(k+1)) bits (Sec. 1), one fewer than an AT: k = 8 fits
    4-bit DRs but not 4-bit ATs."""
    assert state_bytes(Config(16, 4, 8, 64, counter=1))[0] == (1 << 16) // 2
    with pytest.raises(_lib.VateError):
        state_bytes(Config(16, 4, 8, 64, counter=0))


@pytest.mark.parametrize("c,w,k", [(16, 8, 4), (5, 4, 2), (28, 8, 60), (29, 16, 256), (32, 16, 300),
                                   (28, 7, 60), (32, 10, 300), (5, 3, 2), (20, 13, 4000)])
def test_state_bytes(c, w, k):
    pb, sb = state_bytes(Config(c, w, k, 64))
    assert pb == (1 << c) * w // 8
    assert sb % 256 == 0 and sb >= 32 + 8 * k


def test_null_handles_are_rejected():
    L = _lib.lib()
    assert L.vate_ingest(None, None, 0, None) == _lib.VATE_E_INVAL
    assert L.vate_close_slice(None, None) == _lib.VATE_E_INVAL
    assert L.vate_estimate(None, None, 0, 1, None, None, None, None) == _lib.VATE_E_INVAL
    assert L.vate_last_error(None) == b""
    L.vate_destroy(None)
    p = Config(16, 8, 4, 128).params()
    out = ctypes.c_void_p()
    assert L.vate_create(ctypes.byref(p), None, None, None, ctypes.byref(out)) == _lib.VATE_E_INVAL
    assert L.vate_create(ctypes.byref(p), 0x1000 + 8, 0x2000, None, ctypes.byref(out)) == _lib.VATE_E_INVAL


@pytest.mark.parametrize("g", [1, 7, 128, 1000, 1024, 4096, 65535])
def test_host_bh_matches_oracle(g):
    cfg = Config(20, 8, 4, g, seed_a=0x1234, seed_b=0xABCDEF)
    ref = OracleSketch(20, 8, 4, g, 0x1234, 0xABCDEF)
    rng = np.random.default_rng(g)
    for bip in list(rng.integers(0, 2**32, size=300)) + [0, 1, 2**32 - 1]:
        assert host_hash(cfg, 0, int(bip)) == ref.BH(int(bip))


@pytest.mark.parametrize("c", [5, 16, 28, 31, 32])
def test_host_h_matches_oracle(c):
    cfg = Config(c, 16, 4, 64, seed_a=0x77, seed_b=0x99)
    rng = np.random.default_rng(c)
    for aip in list(rng.integers(0, 2**32, size=40)) + [0, 2**32 - 1]:
        for i in (0, 1, 2, 63, 1000, 65534):
            assert host_hash(cfg, 1, int(aip), i) == vate_ref.hash_H(c, 0x77, int(aip), i)


@pytest.mark.parametrize("c,b", [(5, 1), (16, 3), (28, 6), (32, 10), (10, 10)])
def test_host_h_blocked_matches_oracle(c, b):
    """The locality-blocked H of the library equals the oracle's."""
    cfg = Config(c, 16, 4, 64, seed_a=0x51, seed_b=0x99, block_log2=b)
    rng = np.random.default_rng(c + b)
    for aip in list(rng.integers(0, 2**32, size=40)) + [0, 2**32 - 1]:
        for i in (0, 1, 2, 63, 64, 1000, 65534):
            assert host_hash(cfg, 1, int(aip), i) == vate_ref.hash_H_blocked(c, b, 0x51, int(aip), i)


def test_block_log2_validated():
    for bad in (dict(block_log2=11), dict(log2_pool=5, block_log2=6)):
        base = dict(log2_pool=16, width=8, k=4, g=128)
        base.update(bad)
        with pytest.raises(_lib.VateError):
            state_bytes(Config(**base))


@pytest.mark.parametrize("partition", [0, 1])
@pytest.mark.parametrize("c,k", [(6, 1), (6, 2), (7, 3), (8, 9), (10, 16), (16, 4),
                                 (16, 60), (20, 127), (28, 60), (29, 256), (31, 1),
                                 (32, 1), (32, 2), (32, 300), (32, 32767)])
def test_host_block_matches_oracle(c, k, partition):
    """Magic-number division and block clamping equal the oracle's plain
    integer division (Eq. 9-10 / Fig. 5) at block edges and random pids."""
    w = 4 if 2 * k + 1 <= 16 else 8 if 2 * k + 1 <= 256 else 16
    if (1 << c) * w // 8 < 16:
        w = 16
    cfg = Config(c, w, k, 16, partition=partition)
    ref = OracleSketch(c, w, k, 16, partition=partition) if c <= 20 else None
    N = 1 << c
    rng = np.random.default_rng(c * 1000 + k)
    pids = set(int(x) for x in rng.integers(0, N, size=2000))
    pids |= {0, 1, N - 1, N - 2}
    # block edges under both readings
    twok = 2 * k
    for i in range(min(twok + 1, 600)):
        for base in (i * (N // (twok - 1)) if twok > 1 else 0, i * (N // twok)):
            for d in (-1, 0, 1):
                if 0 <= base + d < N:
                    pids.add(base + d)
    for pid in sorted(pids):
        got = host_block(cfg, pid)
        if ref is not None:
            want = ref.block_of(pid)
        elif partition == 0:
            want = min(pid // (N // (twok - 1)), twok - 1)
        else:
            ap, bp = N // twok, N % twok
            want = pid // ap if pid < ap * (twok - bp) else (pid + twok - bp) // (ap + 1)
        assert got == want, (pid, got, want)


def test_kernel_source_hash_ignores_comments(tmp_path, monkeypatch):
    """The hash that ties a committed traffic summary to the kernel sources
    changes with the code and not with its comments or spacing."""
    import shutil

    import bench

    src = os.path.join(bench.ROOT, "paper_1812_00282_amd", "csrc")
    dst = tmp_path / "paper_1812_00282_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    f = dst / "vate_part.h"
    text = f.read_text()
    f.write_text("// another comment\n" + text.replace("\n", "\n\n", 3) + "/* trailing */\n")
    assert bench.kernel_source_hash() == h0
    f.write_text(text.replace("kLookU = 8", "kLookU = 4", 1))
    assert bench.kernel_source_hash() != h0

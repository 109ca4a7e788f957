"""vate_estimate_noalloc (the estimate with its workspace in a fixed device
array) against vate_estimate_ws, through the C ABI: two calls in a row on
one sketch, the second with fewer hosts and a shorter window, must give the
same estimates, live counts and histograms bit for bit; a host count whose
workspace exceeds the fixed array is refused before any work is enqueued."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1812_00282_amd import _lib  # noqa: E402
from paper_1812_00282_amd.sketch import Config, Sketch, _stream_handle  # noqa: E402

pytestmark = pytest.mark.gpu


def _ptr(t):
    return t.data_ptr() if t is not None else None


def _outputs(n, k, dev):
    return (torch.empty(n, dtype=torch.float32, device=dev),
            torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty((n, k + 1), dtype=torch.int32, device=dev))


def _call_ws(sk, hosts, kprime):
    n = hosts.numel()
    est, live, hist = _outputs(n, sk.cfg.k, hosts.device)
    need = ctypes.c_size_t()
    _lib.check(_lib.lib().vate_estimate_workspace_bytes(sk.handle, n, ctypes.byref(need)), sk.handle)
    ws = torch.empty(need.value, dtype=torch.uint8, device=hosts.device)
    _lib.check(_lib.lib().vate_estimate_ws(sk.handle, hosts.data_ptr(), n, kprime, _ptr(est), _ptr(live),
                                           _ptr(hist), ws.data_ptr(), ws.numel(), _stream_handle(None)),
               sk.handle)
    torch.cuda.synchronize()
    return est, live, hist


def _call_noalloc(sk, hosts, kprime):
    n = hosts.numel()
    est, live, hist = _outputs(n, sk.cfg.k, hosts.device)
    # poison the outputs so that a launch that writes nothing cannot pass
    est.fill_(float("nan"))
    live.fill_(-1)
    hist.fill_(-1)
    _lib.check(_lib.lib().vate_estimate_noalloc(sk.handle, hosts.data_ptr(), n, kprime, _ptr(est), _ptr(live),
                                                _ptr(hist), _stream_handle(None)), sk.handle)
    torch.cuda.synchronize()
    return est, live, hist


def _same(a, b, what):
    for x, y, name in zip(a, b, ("est", "live", "hist")):
        assert torch.equal(x, y), f"{what}: {name} differs from vate_estimate_ws"


@pytest.mark.parametrize("log2_pool,width,k,g,n1,n2", [
    (20, 8, 8, 1024, 7000, 1537),     # 8 pool slices, scratch about three quarters full
    (16, 8, 4, 128, 1000, 313),       # the small workload's geometry
    (18, 4, 6, 256, 3000, 77),        # nibble ATs
])
def test_noalloc_matches_ws_two_calls(log2_pool, width, k, g, n1, n2):
    dev = torch.device("cuda")
    print(f"noalloc vs ws: c={log2_pool} w={width} k={k} g={g} hosts {n1} then {n2}", flush=True)
    cfg = Config(log2_pool, width, k, g, seed_a=0x1234, seed_b=0x4321)
    sk = Sketch(cfg, device=dev)
    need = ctypes.c_size_t()
    _lib.check(_lib.lib().vate_estimate_workspace_bytes(sk.handle, n1, ctypes.byref(need)), sk.handle)
    assert 0 < need.value <= _lib.NOALLOC_SCRATCH_BYTES
    rng = np.random.default_rng(7)
    aips = rng.choice(2**32, size=n1, replace=False).astype(np.uint32)
    for t in range(k + 2):
        m = 60_000
        pairs = np.empty((m, 2), dtype=np.uint32)
        pairs[:, 0] = aips[rng.integers(0, n1 // 2, size=m)]
        pairs[:, 1] = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
        sk.ingest(pairs)
        sk.close_slice()
    hosts1 = torch.from_numpy(aips.view(np.int32)).to(dev)
    hosts2 = torch.from_numpy(aips[n1 - n2:].copy().view(np.int32)).to(dev)
    a = _call_noalloc(sk, hosts1, k)
    _same(a, _call_ws(sk, hosts1, k), "first call")
    assert int(a[1].max()) > 0
    b = _call_noalloc(sk, hosts2, max(1, k // 2))
    _same(b, _call_ws(sk, hosts2, max(1, k // 2)), "second, smaller call")


def test_noalloc_refuses_beyond_scratch():
    cfg = Config(20, 8, 8, 1024, seed_a=1, seed_b=2)
    sk = Sketch(cfg, device="cuda")
    sk.ingest(np.zeros((1, 2), dtype=np.uint32))
    sk.close_slice()
    n = 20_000
    need = ctypes.c_size_t()
    _lib.check(_lib.lib().vate_estimate_workspace_bytes(sk.handle, n, ctypes.byref(need)), sk.handle)
    assert need.value > _lib.NOALLOC_SCRATCH_BYTES
    hosts = torch.zeros(n, dtype=torch.int32, device="cuda")
    est = torch.empty(n, dtype=torch.float32, device="cuda")
    rc = _lib.lib().vate_estimate_noalloc(sk.handle, hosts.data_ptr(), n, 8, est.data_ptr(), None, None,
                                          _stream_handle(None))
    assert rc == _lib.VATE_E_INVAL
    assert b"fixed scratch" in _lib.lib().vate_last_error(sk.handle)
    torch.cuda.synchronize()

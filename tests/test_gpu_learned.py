"""Parity of the learned-estimator kernels (BF16 matrix cores, FP32
accumulation) with the FP64 CPU oracle that mirrors their BF16 rounding
points (oracle/mlp_ref.py).

Bar: forward outputs and every gradient tensor within a relative L2 error of
1e-3 (an occasional BF16 rounding of an activation may land on the other side
of a rounding boundary in FP32 vs FP64, moving that activation by one BF16
step, 2^-8 relative); the fragment-layout self-test and the features exact;
Adam within 1e-6 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_ref as M  # noqa: E402
from oracle.vate_ref import OracleSketch  # noqa: E402
from paper_1812_00282_amd import learned as L  # noqa: E402
from paper_1812_00282_amd import streams  # noqa: E402
from paper_1812_00282_amd.sketch import Config, Sketch  # noqa: E402

pytestmark = pytest.mark.gpu


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    return (M.bf16_round(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def _rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    p = M.init_params(seed, zero_out=False)
    p.w3 = rng.standard_normal(64) * 0.3
    p.b1 = rng.standard_normal(64) * 0.1
    p.b2 = rng.standard_normal(64) * 0.1
    p.b3 = 0.2
    x = rng.random((n, 64)) * rng.choice([0.0, 1.0], size=(n, 64), p=[0.3, 0.7])
    r = rng.standard_normal(n) * 2
    y = r + rng.standard_normal(n) * 0.5
    return p, x, r, y


def _to_dev(p, x, r, y=None):
    theta = torch.from_numpy(L.theta_from(p.flat() | {"b3": p.b3})).cuda()
    w = L.pack(theta, L.new_weights())
    xd = torch.from_numpy(_bf16_bits(x).view(np.int16)).cuda()
    rd = torch.from_numpy(r.astype(np.float32)).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda() if y is not None else None
    return theta, w, xd, rd, yd


def test_mfma_fragment_layout():
    rng = np.random.default_rng(0)
    A = M.bf16_round(rng.standard_normal((16, 32)))
    B = M.bf16_round(rng.standard_normal((32, 16)))
    d = L.mfma_selftest(torch.from_numpy(_bf16_bits(A).view(np.int16)).cuda(),
                        torch.from_numpy(_bf16_bits(B).view(np.int16)).cuda())
    torch.cuda.synchronize()
    np.testing.assert_allclose(d.cpu().numpy(), A @ B, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("n", [1, 16, 63, 64, 1000, 4097])
def test_forward_parity(n):
    p, x, r, _ = _problem(n, n)
    _, w, xd, rd, _ = _to_dev(p, x, r)
    o = L.forward(w, xd, rd)
    torch.cuda.synchronize()
    ref, _ = M.forward(p, x, r)
    got = o.cpu().numpy()
    assert _rel_l2(got, ref) < 1e-3
    assert np.max(np.abs(got - ref)) < 2e-2


@pytest.mark.parametrize("n", [64, 200, 4096])
def test_gradient_parity(n):
    p, x, r, y = _problem(100 + n, n)
    _, w, xd, rd, yd = _to_dev(p, x, r, y)
    grad = torch.zeros(L.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    L.train_step(w, xd, rd, yd, grad, loss)
    torch.cuda.synchronize()
    o, cache = M.forward(p, x, r)
    ref_loss, do = M.loss_grad(o, y)
    g = M.backward(p, cache, do)
    got = L.params_from(grad)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-3)
    for name in ("W1", "b1", "W2", "b2", "w3"):
        assert _rel_l2(got[name], getattr(g, name)) < 1e-3, name
    assert got["b3"] == pytest.approx(g.b3, rel=1e-3, abs=1e-6)


def test_adam_parity():
    rng = np.random.default_rng(9)
    p = M.init_params(9, zero_out=False)
    theta = torch.from_numpy(L.theta_from(p.flat() | {"b3": p.b3})).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    st = M.adam_init(p)
    for step in range(1, 4):
        gnp = rng.standard_normal(L.MLP_PARAMS).astype(np.float32)
        g = M.Params(**{k: (val if isinstance(val, float) else val)
                        for k, val in L.params_from(gnp).items()})
        L.adam(theta, torch.from_numpy(gnp).cuda(), m, v, step, lr=1e-2)
        M.adam_step(p, g, st, lr=1e-2)
    torch.cuda.synchronize()
    got = L.params_from(theta)
    for name in ("W1", "b1", "W2", "b2", "w3"):
        np.testing.assert_allclose(got[name], getattr(p, name), rtol=1e-6, atol=1e-7)


def _small_sketch():
    wl = streams.SMALL
    pop = wl.population()
    cfg = Config(wl.log2_pool, wl.width, wl.k, wl.g, seed_a=31, seed_b=32)
    gpu = Sketch(cfg)
    ref = OracleSketch(wl.log2_pool, wl.width, wl.k, wl.g, 31, 32)
    for t in range(wl.n_slices):
        pairs = wl.slice(pop, t)
        gpu.ingest(pairs)
        ref.ingest(pairs)
        gpu.close_slice()
        ref.close_slice()
    return wl, pop, gpu, ref


def test_features_and_fused_learned_estimate():
    """Features from the estimate's histogram match the oracle bit for bit;
    the fused gather+network kernel equals estimate -> features -> forward on
    the GPU exactly, and the oracle's network within tolerance."""
    wl, pop, gpu, ref = _small_sketch()
    hosts = pop.aips
    est, live, hist = gpu.estimate(hosts, want_hist=True)
    cen = gpu.census()
    occ = (2**wl.log2_pool - int(cen[wl.k])) / 2**wl.log2_pool
    x, r = L.features(hist, est, wl.k, wl.g, occ)
    torch.cuda.synchronize()
    r_est, r_live, r_hist = ref.estimate(hosts, want_hist=True)
    r_o = np.log(np.maximum(r_est, 1.0))
    xo = M.features(r_hist, r_hist[:, :wl.k].sum(1), wl.g, wl.k,
                    (ref.N - ref.pool_inactive(wl.k)) / ref.N, r_o)
    xg = x.cpu().numpy().view(np.uint16)
    xb = _bf16_bits(xo)
    # histogram, live and occupancy columns exact; the log column within one
    # BF16 step (FP32 logf vs FP64 log may round to neighbouring values)
    assert np.array_equal(np.delete(xg, wl.k + 2, 1), np.delete(xb, wl.k + 2, 1))
    assert np.all(np.abs(xg[:, wl.k + 2].astype(np.int32) - xb[:, wl.k + 2].astype(np.int32)) <= 1)
    np.testing.assert_allclose(r.cpu().numpy(), np.log(np.maximum(r_est, 1.0)), rtol=1e-6, atol=1e-6)

    p, _, _, _ = _problem(5, 1)
    p.w3 = np.random.default_rng(6).standard_normal(64) * 0.05
    theta = torch.from_numpy(L.theta_from(p.flat() | {"b3": p.b3})).cuda()
    w = L.pack(theta, L.new_weights())
    o = L.forward(w, x, r)
    e_learn, e_cf = L.estimate_learned(gpu, hosts, w)
    p_learn, p_cf = L.estimate_learned(gpu, hosts, w, partitioned=True)
    torch.cuda.synchronize()
    assert torch.equal(e_cf, est)
    assert torch.equal(p_cf, est) and torch.equal(p_learn, e_learn)
    np.testing.assert_allclose(e_learn.cpu().numpy(), np.exp(o.cpu().numpy().astype(np.float64)), rtol=1e-6)
    ref_o, _ = M.forward(p, xo, r_o)
    assert _rel_l2(e_learn.cpu().numpy(), np.exp(ref_o)) < 1e-3


def test_zero_output_layer_gives_closed_form():
    """Before training (w3 = 0, b3 = 0) the learned estimate is the closed
    form clamped below at 1."""
    wl, pop, gpu, ref = _small_sketch()
    p = M.init_params(3, zero_out=True)
    theta = torch.from_numpy(L.theta_from(p.flat() | {"b3": 0.0})).cuda()
    w = L.pack(theta, L.new_weights())
    e_learn, e_cf = L.estimate_learned(gpu, pop.aips, w)
    torch.cuda.synchronize()
    cf = e_cf.cpu().numpy()
    np.testing.assert_allclose(e_learn.cpu().numpy(), np.maximum(cf, 1.0), rtol=2e-6)


# ------------------------------------------------------------------------------
# The trained network at the geometry the benchmark runs (k = 60, g = 1024),
# host by host against the FP64 oracle, and the training envelope.

def _trained_params():
    from paper_1812_00282_amd import train as T
    th = np.load(T.WEIGHTS, allow_pickle=False)["theta"].astype(np.float64)
    d = L.params_from(th)
    return M.Params(d["W1"], d["b1"], d["W2"], d["b2"], d["w3"], float(d["b3"]))


def _k60_sketch(log2_pool=21, n_hosts=3000, slices=64, seed=60):
    """k = 60, g = 1024 sketch and its oracle twin after `slices` slices of a
    heavy-tailed stream (per-host universes of 1..3000 opposite hosts)."""
    rng = np.random.default_rng(seed)
    cfg = Config(log2_pool, 8, 60, 1024, seed_a=0xA5A5, seed_b=0x5A5A)
    gpu = Sketch(cfg)
    ref = OracleSketch(log2_pool, 8, 60, 1024, 0xA5A5, 0x5A5A)
    hosts = rng.choice(2**32, size=n_hosts, replace=False).astype(np.uint32)
    card = np.minimum(np.floor(rng.pareto(1.1, n_hosts) + 1), 3000).astype(np.int64)
    w = card / card.sum()
    for t in range(slices):
        h = rng.choice(n_hosts, size=20_000, p=w)
        j = rng.integers(0, card[h]).astype(np.uint64)
        bip = (hosts[h].astype(np.uint64) * np.uint64(0x9E37) + j * np.uint64(0x85EBCA6B)) % np.uint64(2**32)
        pairs = np.stack([hosts[h], bip.astype(np.uint32)], 1)
        gpu.ingest(pairs)
        ref.ingest(pairs)
        gpu.close_slice()
        ref.close_slice()
    return cfg, gpu, ref, hosts


def test_trained_network_per_host_at_k60():
    """The committed network on a k = 60, g = 1024 sketch after more than k
    slices: features built by the FP64 oracle from its own histograms, its
    forward pass with the GPU's BF16 rounding points, and, per host,
    |ln(learned estimate) - o_ref| <= 2e-2 on the fused and the partitioned
    paths (an activation rounded to the other BF16 neighbour moves o by at
    most |w3_i| 2^-8 |a2_i|); the closed-form outputs within 1e-6 of Eq. 11."""
    cfg, gpu, ref, hosts = _k60_sketch()
    r_est, r_live, r_hist = ref.estimate(hosts, want_hist=True)
    occ = (ref.N - ref.pool_inactive(cfg.k)) / ref.N
    r_o = np.log(np.maximum(r_est, 1.0))
    xo = M.features(r_hist, r_live, cfg.g, cfg.k, occ, r_o)
    o_ref, _ = M.forward(_trained_params(), xo, r_o)
    from paper_1812_00282_amd import train as T
    w = L.pack(T.load(), L.new_weights())
    tol_cf = 1e-6 * np.abs(r_est) + cfg.g * 64 * 2.0**-52
    for part in (False, True):
        learn, cf = L.estimate_learned(gpu, hosts, w, partitioned=part)
        torch.cuda.synchronize()
        cfv = cf.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(cfv - r_est) <= tol_cf), part
        lo = np.log(learn.cpu().numpy().astype(np.float64))
        err = np.abs(lo - o_ref)
        assert np.all(err <= 2e-2), (part, float(err.max()), int(np.argmax(err)))
        assert float(err.mean()) < 2e-3, part
    assert L.fallbacks(w) == 0       # no envelope set: the network runs for every host


def test_envelope_other_geometry_gives_closed_form():
    """Weights whose envelope names another geometry (k = 60, 2^28 x 8-bit,
    g = 1024) on a k = 4 sketch: every learned estimate is exactly the closed
    form, on both paths, and every host is counted."""
    from paper_1812_00282_amd import train as T
    wl, pop, gpu, ref = _small_sketch()
    env = {"k": 60, "g": 1024, "log2_pool": 28, "width": 8,
           "lo": np.full(64, -1e30, np.float32), "hi": np.full(64, 1e30, np.float32)}
    w = L.set_envelope(L.pack(T.load(), L.new_weights()), env)
    hosts = pop.aips
    for part in (False, True):
        learn, cf = L.estimate_learned(gpu, hosts, w, partitioned=part)
        torch.cuda.synchronize()
        assert torch.equal(learn, cf), part
        assert L.fallbacks(w, reset=True) == hosts.size, part
    r_est, _, _ = ref.estimate(hosts)
    assert np.all(np.abs(cf.cpu().numpy() - r_est) <= 1e-6 * np.abs(r_est) + wl.g * 64 * 2.0**-52)


def test_envelope_per_host_ranges():
    """An envelope with the sketch's own geometry whose live-fraction range
    stops at the median: hosts above it get exactly the closed form, the
    others exactly the network's estimate without an envelope; the counter
    holds the number of hosts above it.  Both paths."""
    from paper_1812_00282_amd import train as T
    cfg, gpu, ref, hosts = _k60_sketch(log2_pool=20, n_hosts=2000, slices=62, seed=61)
    _, live, _ = gpu.estimate(hosts)
    torch.cuda.synchronize()
    xl = M.bf16_round(live.cpu().numpy().astype(np.float64) / cfg.g)   # feature k as the network reads it
    hi_live = float(np.median(xl))
    lo = np.full(64, -1e30, np.float32)
    hi = np.full(64, 1e30, np.float32)
    hi[cfg.k] = hi_live
    outside = xl > hi_live
    assert 0 < outside.sum() < hosts.size
    env = {"k": cfg.k, "g": cfg.g, "log2_pool": cfg.log2_pool, "width": cfg.width, "lo": lo, "hi": hi}
    theta = T.load()
    plain = L.pack(theta, L.new_weights())
    guarded = L.set_envelope(L.pack(theta, L.new_weights()), env)
    for part in (False, True):
        free, cf = L.estimate_learned(gpu, hosts, plain, partitioned=part)
        got, cf2 = L.estimate_learned(gpu, hosts, guarded, partitioned=part)
        torch.cuda.synchronize()
        assert torch.equal(cf, cf2)
        out = torch.from_numpy(outside).cuda()
        assert torch.equal(got[out], cf[out]), part
        assert torch.equal(got[~out], free[~out]), part
        assert L.fallbacks(guarded, reset=True) == int(outside.sum()), part


def test_envelope_counts_across_many_workgroups():
    """Every host of a 60,000-host estimate falls back (an envelope of another
    pool size): the fallback counters, kept in slots per workgroup, sum to the
    host count on both paths, and every estimate is the closed form."""
    from paper_1812_00282_amd import train as T
    cfg, gpu, ref, _ = _k60_sketch(log2_pool=21, n_hosts=3000, slices=8, seed=62)
    hosts = np.random.default_rng(63).choice(2**32, size=60_000, replace=False).astype(np.uint32)
    env = {"k": cfg.k, "g": cfg.g, "log2_pool": cfg.log2_pool + 1, "width": cfg.width,
           "lo": np.full(64, -1e30, np.float32), "hi": np.full(64, 1e30, np.float32)}
    w = L.set_envelope(L.pack(T.load(), L.new_weights()), env)
    assert L.fallbacks(w) == 0
    for part in (False, True):
        learn, cf = L.estimate_learned(gpu, hosts, w, partitioned=part)
        torch.cuda.synchronize()
        assert torch.equal(learn, cf), part
        assert L.fallbacks(w, reset=True) == hosts.size, part
    assert L.fallbacks(w) == 0

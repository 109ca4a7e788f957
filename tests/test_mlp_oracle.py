"""Pins of the learned-estimator CPU oracle (oracle/mlp_ref.py).  CPU only."""

import numpy as np
import pytest

from oracle import mlp_ref as M


def test_gelu_matches_normal_cdf_table():
    """GELU(z) = z * Phi(z); standard normal CDF values Phi(1) = 0.8413447461,
    Phi(2) = 0.9772498681, Phi(-1) = 0.1586552539 (normal tables)."""
    assert M.gelu(0.0) == 0.0
    assert M.gelu(1.0) == pytest.approx(0.8413447460685429, abs=1e-15)
    assert M.gelu(2.0) == pytest.approx(2 * 0.9772498680518208, abs=1e-15)
    assert M.gelu(-1.0) == pytest.approx(-0.15865525393145707, abs=1e-15)


def test_gelu_grad_by_finite_differences():
    z = np.linspace(-6, 6, 121)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(z), fd, atol=1e-8)


def test_bf16_round_to_nearest_even():
    e = 2.0 ** -7            # bf16 spacing at 1.0
    cases = {1.0: 1.0, 1.0 + e / 2: 1.0, 1.0 + 1.5 * e: 1.0 + 2 * e,
             1.0 + e / 2 + 2.0 ** -20: 1.0 + e, -(1.0 + 1.5 * e): -(1.0 + 2 * e),
             65536.0: 65536.0, 0.0: 0.0, 3.0: 3.0}
    for x, want in cases.items():
        assert M.bf16_round(np.float32(x)) == want, x
    # every result is representable in 8 significant bits
    r = M.bf16_round(np.random.default_rng(0).standard_normal(1000))
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)


def _rand_problem(seed, B=37):
    rng = np.random.default_rng(seed)
    p = M.init_params(seed, zero_out=False)
    p.b1 = rng.standard_normal(M.HID) * 0.1
    p.b2 = rng.standard_normal(M.HID) * 0.1
    p.b3 = 0.3
    x = rng.random((B, M.F))
    r = rng.standard_normal(B)
    return p, x, r


def test_backward_matches_finite_differences_unrounded():
    """With the BF16 rounding points switched off the network is smooth; the
    analytic gradient of sum(c * o) must match central differences for every
    parameter tensor."""
    p, x, r = _rand_problem(1)
    c = np.random.default_rng(2).standard_normal(x.shape[0])
    o, cache = M.forward(p, x, r, rounding=False)
    g = M.backward(p, cache, c, rounding=False)
    h = 1e-6
    rng = np.random.default_rng(3)
    for name in ("W1", "b1", "W2", "b2", "w3"):
        arr = getattr(p, name)
        idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(12)]
        for ix in idx:
            q = p.copy()
            getattr(q, name)[ix] += h
            op, _ = M.forward(q, x, r, rounding=False)
            q2 = p.copy()
            getattr(q2, name)[ix] -= h
            om, _ = M.forward(q2, x, r, rounding=False)
            fd = (c @ op - c @ om) / (2 * h)
            assert getattr(g, name)[ix] == pytest.approx(fd, rel=1e-5, abs=1e-7), (name, ix)
    q = p.copy(); q.b3 += h
    op, _ = M.forward(q, x, r, rounding=False)
    assert g.b3 == pytest.approx((c @ op - c @ o) / h, rel=1e-4)


def test_loss_gradient_by_finite_differences():
    rng = np.random.default_rng(4)
    o = rng.standard_normal(50)
    y = o + rng.choice([-1, 1], 50) * (0.1 + rng.random(50))    # away from the kink
    _, do = M.loss_grad(o, y)
    h = 1e-7
    for i in range(50):
        op = o.copy(); op[i] += h
        om = o.copy(); om[i] -= h
        fd = (M.loss_grad(op, y)[0] - M.loss_grad(om, y)[0]) / (2 * h)
        assert do[i] == pytest.approx(fd, rel=1e-5)


def test_zero_output_layer_reproduces_residual():
    """With w3 = 0 and b3 = 0 the network returns r exactly, i.e. the learned
    estimate equals the (clamped) closed form before any training."""
    p = M.init_params(7, zero_out=True)
    x = np.random.default_rng(5).random((10, M.F))
    r = np.log(np.arange(1, 11, dtype=np.float64))
    o, _ = M.forward(p, x, r)
    assert np.array_equal(o, r)


def test_adam_first_step_is_signed_lr():
    """Kingma & Ba: after bias correction the first step is
    -lr * g / (|g| + eps) for every parameter."""
    p, x, r = _rand_problem(6)
    g = p.copy()
    rng = np.random.default_rng(8)
    for name in ("W1", "b1", "W2", "b2", "w3"):
        setattr(g, name, rng.standard_normal(getattr(p, name).shape))
    g.b3 = -0.25
    st = M.adam_init(p)
    q = p.copy()
    M.adam_step(q, g, st, lr=0.01, eps=1e-8)
    for name in ("W1", "b1", "W2", "b2", "w3"):
        gp = getattr(g, name)
        want = getattr(p, name) - 0.01 * gp / (np.abs(gp) + 1e-8)
        assert np.allclose(getattr(q, name), want, rtol=0, atol=1e-12)
    assert q.b3 == pytest.approx(p.b3 + 0.01 * 0.25 / (0.25 + 1e-8))


def test_features_layout():
    hist = np.array([[3, 1, 0, 124], [0, 0, 0, 128]], dtype=np.uint32)
    x = M.features(hist, np.array([4, 0]), 128, 3, 0.25, np.array([1.6, 0.0]))
    assert x.shape == (2, M.F)
    assert np.allclose(x[0, :6], [3 / 128, 1 / 128, 0, 4 / 128, 0.25, 0.1])
    assert np.all(x[:, 6:] == 0)

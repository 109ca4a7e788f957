"""Pins of the CPU oracle against facts fixed by the paper and the mathematics,
not against the oracle itself.  CPU only.

Each test names the passage it pins and a plausible mistake it would catch.
"""
import math
import os

import numpy as np
import pytest

from oracle import brute, vate_ref
from oracle.vate_ref import OracleSketch
from paper_1812_00282_amd import streams

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ranges(spec: str) -> list[int]:
    out = []
    for part in spec.split(","):
        if "-" in part:
            lo, hi = part.split("-")
            out.extend(range(int(lo), int(hi) + 1))
        else:
            out.append(int(part))
    return out


# ---------------------------------------------------------------- hashing --

def test_fmix32_published_vectors():
    """mix = MurmurHash3's finalizer; the empty-input MurmurHash3_x86_32
    verification values equal fmix32(seed).  Catches a wrong constant or
    shift in the finalizer."""
    with open(os.path.join(GOLDEN, "fmix32_vectors.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for x, y in rows:
        assert vate_ref.fmix32(int(x, 16)) == int(y, 16)


def test_bh_is_top_bits_for_power_of_two_g():
    """Multiply-high range reduction floor(m*g/2^32) equals the top log2(g)
    bits of m when g is a power of two (Lemire).  BH(bip) must therefore be
    mix(bip ^ seed_b) >> (32 - log2 g); catches a modulo or wrong shift."""
    seed_b = 0x1234567
    for g in (1, 2, 128, 1024, 65536):
        s = OracleSketch(16, 8, 4, g, seed_a=7, seed_b=seed_b)
        m = int(math.log2(g))
        for bip in (0, 1, 2, 0xDEADBEEF, 0xFFFFFFFF, 12345678):
            mixed = vate_ref.fmix32(bip ^ seed_b)
            want = mixed >> (32 - m) if m > 0 else 0
            assert s.BH(bip) == want


def test_bh_range_and_balance():
    """BH lands in [0, g) and spreads bips evenly (chi-square at 1e-6)."""
    for g in (100, 1000):
        s = OracleSketch(16, 8, 4, g, seed_a=1, seed_b=2)
        vals = np.array([s.BH(b) for b in range(20000)])
        assert vals.min() >= 0 and vals.max() < g
        cnt = np.bincount(vals, minlength=g)
        exp = vals.size / g
        chi2 = ((cnt - exp) ** 2 / exp).sum()
        # mean g-1, sd sqrt(2(g-1)); 6 sd is far beyond chance
        assert chi2 < (g - 1) + 6 * math.sqrt(2 * (g - 1))


def test_h_range_and_balance():
    """H(aip, i) lands in [0, 2^c) and a host's g VATs spread evenly over the
    pool (a host-independent offset or a constant i-term would fail)."""
    c = 10
    s = OracleSketch(c, 8, 4, 64, seed_a=99, seed_b=3)
    pids = np.array([s.H(aip, i) for aip in range(300) for i in range(64)])
    assert pids.min() >= 0 and pids.max() < 2**c
    cnt = np.bincount(pids, minlength=2**c)
    exp = pids.size / 2**c
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    dof = 2**c - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    # different i of one host give different slots most of the time
    one = [s.H(0xABCDEF, i) for i in range(64)]
    assert len(set(one)) >= 60


# ------------------------------------------------------------- partition --

@pytest.mark.parametrize("c,k", [(6, 1), (6, 2), (6, 3), (8, 4), (8, 9), (10, 16),
                                 (7, 31), (12, 60), (5, 16)])
def test_partition_eq9_block_sizes(c, k):
    """Eq. 9-10, Fig. 4: blocks 0..2k-2 hold a = floor(2^c/(2k-1)) ATs each,
    the last block holds b = 2^c mod (2k-1); blocks are contiguous and
    ordered.  Catches using Algorithm 4's 2^c/k or an unclamped last block."""
    s = OracleSketch(c, 16, k, 4, partition=0)
    N = 2**c
    bids = np.array([s.block_of(p) for p in range(N)])
    assert np.all(np.diff(bids) >= 0) and bids[0] == 0 and bids.max() <= 2 * k - 1
    sizes = np.bincount(bids, minlength=2 * k)
    a, b = N // (2 * k - 1), N % (2 * k - 1)
    assert np.all(sizes[: 2 * k - 1] == a)
    assert sizes[2 * k - 1] == b
    for i in range(2 * k):
        assert s.blk_start(i) == int(np.searchsorted(bids, i, side="left"))


@pytest.mark.parametrize("c,k", [(6, 1), (6, 3), (8, 9), (10, 16), (7, 31), (12, 60)])
def test_partition_lowdev_block_sizes(c, k):
    """Fig. 5: with a' = 2^c/(2k), b' = 2^c mod 2k, the first 2k-b' blocks
    hold a' ATs and the last b' hold a'+1; sizes differ by at most one."""
    s = OracleSketch(c, 16, k, 4, partition=1)
    N = 2**c
    bids = np.array([s.block_of(p) for p in range(N)])
    assert np.all(np.diff(bids) >= 0) and bids.max() == 2 * k - 1
    sizes = np.bincount(bids, minlength=2 * k)
    ap, bp = N // (2 * k), N % (2 * k)
    assert np.all(sizes[: 2 * k - bp] == ap)
    assert np.all(sizes[2 * k - bp:] == ap + 1)


# ------------------------------------------------------------ preserveAT --

def test_preserve_k9_worked_example():
    """The k = 9 example of Sec. 3 (golden fixture)."""
    with open(os.path.join(GOLDEN, "preserve_k9.txt")) as f:
        lines = [l.split() for l in f if l.strip() and not l.startswith("#")]
    k = int(lines[0][1])
    assert k == 9
    for row in lines[1:]:
        act = int(row[1])
        mark, keep = _ranges(row[3]), _ranges(row[5])
        assert sorted(mark + keep) == list(range(2 * k + 1))
        for v in mark:
            assert vate_ref.preserve_fast(v, act, k) == 2 * k, (act, v)
        for v in keep:
            assert vate_ref.preserve_fast(v, act, k) == v, (act, v)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 9, 16, 60, 127])
def test_alg3_equals_alg2_on_reachable_states(k):
    """Algorithm 3 is the fast form of Algorithm 2 at ACT in {0, k}.  The two
    agree for every value except Value == ACT, which cannot occur at the start
    of a slice (it would mean a distance of exactly 2k, which the previous
    preservation k slices earlier already removed)."""
    for act in (0, k):
        for v in range(2 * k + 1):
            f = vate_ref.preserve_fast(v, act, k)
            g = vate_ref.preserve_general(v, act, k)
            if v == act:
                assert f == 2 * k and g == v
            else:
                assert f == g, (act, v)


def test_check_at_k9_distances():
    """Algorithm 1 at k=9: an AT set d slices ago (value = ACT - d mod 2k) is
    active for k' iff d < k'; the inactive value 2k is never active."""
    k = 9
    for act in range(2 * k):
        for d in range(2 * k):
            v = (act - d) % (2 * k)
            for kp in range(1, k + 1):
                assert vate_ref.check_at(v, act, k, kp) == (d < kp)
        for kp in range(1, k + 1):
            assert not vate_ref.check_at(2 * k, act, k, kp)


# ------------------------------------------- AT state vs 64-bit timestamps --

def _ts_run(c, k, partition, seed, n_slices, per_slice, n_hosts=40, g=16,
            empty_every=0, block_log2=0):
    """Drive the oracle and a TS pool with the same random stream and compare
    at every slice end: CheckAT of every slot for every k' (Thm. 1, Cor. 1),
    the census, and each host's live count and distance histogram."""
    rng = np.random.default_rng(seed)
    s = OracleSketch(c, 16, k, g, seed_a=seed, seed_b=seed + 1, partition=partition,
                     block_log2=block_log2)
    N = s.N
    ts = brute.TSPool(N)
    hosts = rng.integers(0, 2**32, size=n_hosts, dtype=np.uint64).astype(np.uint32)
    vat_pids = np.array([[s.H(int(a), i) for i in range(g)] for a in hosts])
    for t in range(n_slices):
        if empty_every and t % empty_every == empty_every - 1:
            pairs = np.zeros((0, 2), dtype=np.uint32)
        else:
            n = int(rng.integers(0, per_slice + 1))
            pairs = np.stack([hosts[rng.integers(0, n_hosts, size=n)],
                              rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)],
                             axis=1)
        if pairs.size:
            s.ingest(pairs)
            ts.set(s.packet_pids(pairs), t)
        s.close_slice()
        assert s.t == t and s.bact0 == t % (2 * k)
        vals = s.values().astype(np.int64)
        acts = np.array([s.act_of(p) for p in range(N)])
        age = ts.age(t)
        # distance histogram of the pool
        cen = s.census()
        for d in range(k):
            assert cen[d] == np.count_nonzero(age == d), (t, d)
        assert cen[k] == N - np.count_nonzero(age < k)
        for kp in range(1, k + 1):
            truth = ts.active(t, kp)
            got = np.array([vate_ref.check_at(int(v), int(a), k, kp)
                            for v, a in zip(vals, acts)])
            assert np.array_equal(got, truth), (t, kp)
            assert s.pool_inactive(kp) == N - truth.sum()
        est, live, hist = s.estimate(hosts, kprime=k, want_hist=True)
        host_age = age[vat_pids]
        assert np.array_equal(live, (host_age < k).sum(axis=1))
        for d in range(k):
            assert np.array_equal(hist[:, d], (host_age == d).sum(axis=1))
        assert np.array_equal(hist[:, k], g - (host_age < k).sum(axis=1))
    return s


@pytest.mark.parametrize("k", [1, 2, 3, 4, 9, 16])
@pytest.mark.parametrize("partition", [0, 1])
def test_at_state_matches_timestamps(k, partition):
    """Thm. 1 / Cor. 1: with preservation at ACT in {0, k}, CheckAT equals
    the exact timestamp test for every slot, slice and k' <= k.  Catches a
    wrong preserve range, a wrong ACT offset, a missed block, preserving
    before estimating, or an off-by-one in the distance."""
    c = 6 if k <= 4 else 8
    _ts_run(c, k, partition, seed=10 * k + partition, n_slices=4 * k + 6,
            per_slice=3 * 2**c // (2 * k + 2), empty_every=5)


def test_at_state_matches_timestamps_long_sparse():
    """Long run with sparse traffic so ATs age through several ACT wraps."""
    _ts_run(8, 5, 0, seed=77, n_slices=60, per_slice=20, n_hosts=10, g=8)


@pytest.mark.parametrize("k,b", [(4, 2), (9, 3)])
def test_at_state_matches_timestamps_blocked_h(k, b):
    """The AT state machine does not depend on where H puts the VATs: with
    the locality-blocked H the pool still equals the timestamp pool."""
    _ts_run(8, k, 0, seed=31 * k + b, n_slices=3 * k + 4, per_slice=150, block_log2=b)


def test_blocked_h_structure():
    """Locality-blocked H with blocks of 2^b VATs: VAT i lands in slot i mod 2^b
    of a block whose index is the independent H of a pool of 2^(c-b) ATs
    evaluated at VAT index floor(i / 2^b); b = 0 is the independent H."""
    rng = np.random.default_rng(8)
    for b in range(0, 7):
        for _ in range(300):
            c = int(rng.integers(max(b, 1), 33))
            seed, aip = int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))
            i = int(rng.integers(0, 1 << 14))
            got = vate_ref.hash_H_blocked(c, b, seed, aip, i)
            if b == 0:
                assert got == vate_ref.hash_H(c, seed, aip, i)
            else:
                base = vate_ref.hash_H(c - b, seed, aip, i >> b)
                assert got == (base << b) | (i & ((1 << b) - 1))


# -------------------------------------------------------------- estimate --

def test_estimate_reduces_to_linear_counting():
    """Eq. 11 with an empty pool (Z_p = 1) is the linear estimator of Eq. 1,
    -g ln(g0/g).  Catches the printed sign of Eq. 11 and a mis-scaled Z."""
    for g in (16, 128, 1024):
        for u_v in (1, 3, g // 2, g - 1, g):
            N = 2**20
            le = -g * math.log(u_v / g)
            assert vate_ref.estimate_counts(u_v, N, g, N) == pytest.approx(le, rel=1e-15, abs=1e-12)
    # saturation: no inactive VAT is treated as one
    assert vate_ref.estimate_counts(0, 2**20, 64, 2**20) == pytest.approx(64 * math.log(64))


def test_estimate_accuracy_on_loaded_pool():
    """Def. 1 truth vs the oracle for probe hosts in a pool that traffic keeps
    about 40% active.  With g = 1024 the mean estimate must sit
    within 4 standard errors of the true cardinality.  Dropping the pool term
    g ln Z_p would bias every estimate by ~g*0.36 = 370 and fail."""
    c, k, g = 18, 4, 1024
    s = OracleSketch(c, 8, k, g, seed_a=5, seed_b=6)
    rng = np.random.default_rng(123)
    # background: 70k distinct pairs over many hosts; the 180 probes add 63k
    bg_hosts = rng.integers(0, 2**32, size=3000, dtype=np.uint64).astype(np.uint32)
    bg = np.stack([bg_hosts[rng.integers(0, 3000, size=70000)],
                   rng.integers(0, 2**32, size=70000, dtype=np.uint64).astype(np.uint32)], 1)
    probes = rng.integers(0, 2**32, size=180, dtype=np.uint64).astype(np.uint32)
    truths = np.array([50, 200, 800] * 60)
    pp = [np.stack([np.full(n, h, dtype=np.uint32),
                    rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)], 1)
          for h, n in zip(probes, truths)]
    slice_pairs = np.concatenate([bg] + pp)
    s.ingest(slice_pairs)
    s.close_slice()
    zp = s.pool_inactive(k) / s.N
    assert 0.55 < zp < 0.8
    truth = brute.window_truth([slice_pairs], 0, k)
    est, live, _ = s.estimate(probes)
    for n in (50, 200, 800):
        sel = truths == n
        tr = np.array([truth[int(h)] for h in probes[sel]])
        assert np.all(tr == n)
        rel = est[sel] / tr
        se = brute.virtual_std_error(n, g, zp)
        assert abs(rel.mean() - 1.0) < 4 * se / math.sqrt(sel.sum()) + 0.01, (n, rel.mean())
        # without the pool term the mean would be off by g ln(1/Z_p) / n
        assert g * math.log(1 / zp) / n > 8 * se / math.sqrt(sel.sum())


def test_blocked_h_accuracy_cost():
    """The locality-blocked H keeps the estimate unbiased but spreads it: the
    VATs of a block share their neighbours' traffic, so the noise of Z_v is
    no longer averaged over g independent slots.  Same loaded pool as above;
    the mean stays within 6 observed standard errors of the truth for 64-VAT
    blocks, and the spread at n = 200 exceeds the independent H's."""
    c, k, g = 18, 4, 1024
    rng0 = np.random.default_rng(123)
    bg_hosts = rng0.integers(0, 2**32, size=3000, dtype=np.uint64).astype(np.uint32)
    bg = np.stack([bg_hosts[rng0.integers(0, 3000, size=70000)],
                   rng0.integers(0, 2**32, size=70000, dtype=np.uint64).astype(np.uint32)], 1)
    probes = rng0.integers(0, 2**32, size=300, dtype=np.uint64).astype(np.uint32)
    truths = np.array([50, 200, 800] * 100)
    pp = [np.stack([np.full(n, h, dtype=np.uint32),
                    rng0.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)], 1)
          for h, n in zip(probes, truths)]
    pairs = np.concatenate([bg] + pp)
    spread = {}
    for b in (0, 6):
        s = OracleSketch(c, 8, k, g, seed_a=5, seed_b=6, block_log2=b)
        s.ingest(pairs)
        s.close_slice()
        est, _, _ = s.estimate(probes)
        for n in (50, 200, 800):
            rel = est[truths == n] / n
            assert abs(rel.mean() - 1.0) < 6 * rel.std() / math.sqrt(rel.size) + 0.02, (b, n)
            spread[b, n] = rel.std()
    assert spread[6, 200] > 1.5 * spread[0, 200]


def test_estimate_accuracy_small_workload():
    """The small 2^16 x 8-bit workload: hosts with window truth in [10, 300]
    (well below g ln g saturation for g = 128) are estimated with mean
    relative error under 15%."""
    wl = streams.SMALL
    pop = wl.population()
    s = OracleSketch(wl.log2_pool, wl.width, wl.k, wl.g, seed_a=11, seed_b=12)
    slices = []
    for t in range(wl.n_slices):
        pairs = wl.slice(pop, t)
        slices.append(pairs)
        s.ingest(pairs)
        s.close_slice()
    t = wl.n_slices - 1
    truth = brute.window_truth(slices, t, wl.k)
    hosts = np.array([h for h, n in truth.items() if 10 <= n <= 300], dtype=np.uint32)
    assert hosts.size > 50
    est, _, _ = s.estimate(hosts)
    tr = np.array([truth[int(h)] for h in hosts], dtype=np.float64)
    mre = np.mean(np.abs(est - tr) / tr)
    assert mre < 0.15, mre


# --------------------------------------------------------- ingest / state --

def test_order_and_duplicate_invariance():
    """Sec. 4.2's race argument: every SetAT of one AT within a slice writes
    the same value, so packet order, duplicates, and padding the last batch
    with its last pair (Sec. 4.2 buffers) do not change the pool."""
    rng = np.random.default_rng(4)
    pairs = rng.integers(0, 2**32, size=(5000, 2), dtype=np.uint64).astype(np.uint32)
    pairs[:, 0] = pairs[rng.integers(0, 50, size=5000), 0]
    a = OracleSketch(10, 8, 3, 32, 1, 2)
    b = OracleSketch(10, 8, 3, 32, 1, 2)
    for t in range(7):
        chunk = pairs[t * 700:(t + 1) * 700]
        a.ingest(chunk)
        shuffled = chunk[rng.permutation(len(chunk))]
        dup = np.concatenate([shuffled, shuffled[:100], np.repeat(shuffled[-1:], 37, 0)])
        b.ingest(dup[:300])
        b.ingest(dup[300:])
        a.close_slice()
        b.close_slice()
        assert np.array_equal(a.values(), b.values())


def test_state_machine_and_clock():
    s = OracleSketch(8, 8, 3, 16)
    with pytest.raises(RuntimeError):
        s.estimate(np.array([1], dtype=np.uint32))          # slice 0 still open
    for t in range(20):
        s.close_slice()                                      # empty slices
        assert s.t == t and s.bact0 == t % 6 and s.closed
    with pytest.raises(RuntimeError):
        s.estimate(np.array([1], dtype=np.uint32), kprime=4)  # k' > k
    with pytest.raises(ValueError):
        OracleSketch(8, 4, 8, 16)                            # 2k+1 = 17 > 2^4
    with pytest.raises(ValueError):
        OracleSketch(2, 8, 3, 16)                            # 2^c < 2k


@pytest.mark.parametrize("w", [4, 8, 16, 2, 3, 7, 10, 13])
def test_packed_layout(w):
    """Pool layout: AT p occupies bits [p*w, (p+1)*w) of a little-endian bit
    stream, for the 4/8/16-bit containers and for exact widths (the paper's
    ceil(log2(2k+1))-bit ATs).  Unpacked here bit by bit with numpy."""
    k = {4: 3, 8: 60, 16: 300}.get(w, min((2**w - 1) // 2, 400))
    s = OracleSketch(10, w, k, 8)
    rng = np.random.default_rng(w)
    vals = rng.integers(0, 2 * k + 1, size=s.N).astype(np.uint16)
    s.set_values(vals, 0, 0, False)
    packed = s.packed_pool()
    bits = np.unpackbits(packed, bitorder="little").reshape(s.N, w)
    back = (bits.astype(np.uint32) << np.arange(w, dtype=np.uint32)).sum(1)
    assert np.array_equal(back, vals)


# ---------------------------------------------------------- VDRE (DR) ----

@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_dr_state_matches_timestamps(k):
    """DR counters (Sec. 1): reset to 0 on a hit, +1 per slide (saturating at
    k); active for k' iff the value is below k' -- i.e. exactly the 64-bit
    timestamp test for every slot, slice and k' <= k."""
    rng = np.random.default_rng(100 + k)
    c, g = 8, 16
    s = OracleSketch(c, 8, k, g, seed_a=3, seed_b=4, counter=1)
    ts = brute.TSPool(s.N)
    hosts = rng.integers(0, 2**32, size=30, dtype=np.uint64).astype(np.uint32)
    for t in range(4 * k + 8):
        n = int(rng.integers(0, 200))
        pairs = np.stack([hosts[rng.integers(0, 30, size=n)],
                          rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)], 1)
        s.ingest(pairs)
        ts.set(s.packet_pids(pairs), t)
        s.close_slice()
        vals = s.values().astype(np.int64)
        assert np.array_equal(vals, np.minimum(ts.age(t), k))
        for kp in range(1, k + 1):
            assert s.pool_inactive(kp) == s.N - ts.active(t, kp).sum()


@pytest.mark.parametrize("k,partition", [(3, 0), (9, 1), (16, 0)])
def test_vate_equals_vdre(k, partition):
    """The paper (Sec. 5): with the same hashing, VATE and VDRE give the same
    estimates.  Live counts, histograms, census and estimates must be equal
    at every slice for every window."""
    rng = np.random.default_rng(k)
    a = OracleSketch(10, 16, k, 64, seed_a=5, seed_b=6, partition=partition, counter=0)
    d = OracleSketch(10, 16, k, 64, seed_a=5, seed_b=6, partition=partition, counter=1)
    hosts = rng.integers(0, 2**32, size=40, dtype=np.uint64).astype(np.uint32)
    for t in range(3 * k + 5):
        n = int(rng.integers(0, 600))
        pairs = np.stack([hosts[rng.integers(0, 40, size=n)],
                          rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)], 1)
        a.ingest(pairs)
        d.ingest(pairs)
        a.close_slice()
        d.close_slice()
        assert np.array_equal(a.census(), d.census())
        for kp in range(1, k + 1):
            ea, la, ha = a.estimate(hosts, kprime=kp, want_hist=True)
            ed, ld, hd = d.estimate(hosts, kprime=kp, want_hist=True)
            assert np.array_equal(la, ld) and np.array_equal(ha, hd)
            assert np.array_equal(ea, ed)

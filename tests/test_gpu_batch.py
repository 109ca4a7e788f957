"""Batched sketches (one persistent launch per phase, hipGraph replay,
autotuned launch shapes): every member sketch bit-exact with its oracle twin
(eager, under graph replay, after the autotuner and under two hand-set
launch shapes) and with the same sketch driven alone through the
single-sketch calls."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.vate_ref import OracleSketch  # noqa: E402
from paper_1812_00282_amd import streams  # noqa: E402
from paper_1812_00282_amd.batch import Batch  # noqa: E402
from paper_1812_00282_amd.sketch import Config, Sketch  # noqa: E402

pytestmark = pytest.mark.gpu

REL_TOL = 1e-6


def _tol(ref_est, g):
    return REL_TOL * np.abs(ref_est) + g * 64 * 2.0**-52


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _rand_slice(rng, hosts, n):
    return np.stack([hosts[rng.integers(0, hosts.size, size=n)],
                     rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)], 1)


SMALL = [Config(12, 8, 4, 64, 0, 1, 2), Config(10, 4, 3, 32, 0, 3, 4), Config(14, 8, 16, 128, 0, 5, 6),
         Config(11, 16, 7, 64, 1, 7, 8), Config(12, 8, 1, 16, 0, 9, 10), Config(9, 4, 2, 16, 1, 11, 12),
         Config(15, 16, 40, 256, 0, 13, 14)]


def test_batch_matches_oracle():
    rng = np.random.default_rng(0)
    hosts = [rng.integers(0, 2**32, size=int(rng.integers(50, 600)), dtype=np.uint64).astype(np.uint32)
             for _ in SMALL]
    caps = [20000] * len(SMALL)
    sks = [Sketch(c) for c in SMALL]
    refs = [OracleSketch(c.log2_pool, c.width, c.k, c.g, c.seed_a, c.seed_b, c.partition) for c in SMALL]
    b = Batch(sks, caps, hosts)
    for t in range(30):
        slices = [_rand_slice(rng, h, 0 if (t + i) % 9 == 8 else int(rng.integers(1, 20000)))
                  for i, h in enumerate(hosts)]
        b.load(slices)
        b.slice()
        for r, sl in zip(refs, slices):
            r.ingest(sl)
            r.close_slice()
        if t % 3 == 2 or t == 29:
            b.synchronize()
            for i, (s, r) in enumerate(zip(sks, refs)):
                pool, tt, bact0, closed = s.read_state()
                assert (tt, bact0, closed) == (r.t, r.bact0, True), (t, i)
                assert np.array_equal(pool, r.packed_pool()), (t, i)
                assert np.array_equal(s.census(), r.census()), (t, i)
                r_est, r_live, _ = r.estimate(hosts[i])
                assert np.array_equal(_u32(b.live[i]), r_live), (t, i)
                e = b.est[i].cpu().numpy().astype(np.float64)
                assert np.all(np.abs(e - r_est) <= _tol(r_est, r.g)), (t, i)


EXACT = [Config(12, 3, 3, 64, 0, 21, 22), Config(13, 7, 60, 128, 0, 23, 24), Config(11, 5, 12, 32, 1, 25, 26),
         Config(14, 10, 300, 256, 0, 27, 28), Config(12, 6, 60, 64, 0, 29, 30, counter=1),
         Config(13, 8, 20, 64, 0, 31, 32), Config(10, 9, 9, 16, 0, 33, 34, counter=1)]


def test_batch_exact_widths_match_oracle():
    """Exact-width pools (3, 5, 6, 7, 9 and 10 bits; AT and DR counters; both
    block partitions) batched with a byte pool: every member's pool, clock,
    census, live counts and estimates against its oracle twin after every
    third slice, over more than 2k slices for the k = 3..60 members."""
    rng = np.random.default_rng(5)
    hosts = [rng.integers(0, 2**32, size=int(rng.integers(50, 400)), dtype=np.uint64).astype(np.uint32)
             for _ in EXACT]
    sks = [Sketch(c) for c in EXACT]
    refs = [OracleSketch(c.log2_pool, c.width, c.k, c.g, c.seed_a, c.seed_b, c.partition, c.counter)
            for c in EXACT]
    b = Batch(sks, [6000] * len(EXACT), hosts)
    n_slices = 125
    for t in range(n_slices):
        slices = [_rand_slice(rng, h, 0 if (t + i) % 11 == 10 else int(rng.integers(1, 6000)))
                  for i, h in enumerate(hosts)]
        b.load(slices)
        b.slice()
        for r, sl in zip(refs, slices):
            r.ingest(sl)
            r.close_slice()
        if t % 3 == 2 or t == n_slices - 1:
            b.synchronize()
            for i, (sk, r) in enumerate(zip(sks, refs)):
                _check_oracle(sk, b.est[i], b.live[i], r, hosts[i], np.arange(hosts[i].size), (t, i))


def test_batch_exact_widths_graph_replay():
    """Exact-width members under graph replay: every slice bit-exact with the
    oracle twins and the standalone GPU twins."""
    members = [streams.BatchMember(c.log2_pool, c.width, c.k, c.g, 200 + 37 * i, 700 + i)
               for i, c in enumerate(EXACT) if c.counter == 0]
    counts = lambda s: streams.batch_packet_counts(8, len(members), s, lo=3.0, hi=3.7)
    timing, _ = _run_pair(members, 10, counts, graph=True)
    assert len(timing["replay"]) == 9


def _members_small():
    ms = streams.batch_members(seed=4, pool_range=(14, 18), host_shift=6)
    return ms


def _check_oracle(sk, est, live, ref, hosts_np, idx, what):
    """A batch member against its oracle twin: pool bytes, clock and census
    bit-exact; live counts exact and estimates within the bar on hosts idx."""
    pool, t, bact0, closed = sk.read_state()
    assert (t, bact0, closed) == (ref.t, ref.bact0, True), what
    assert np.array_equal(pool, ref.packed_pool()), what
    assert np.array_equal(sk.census(), ref.census()), what
    r_est, r_live, _ = ref.estimate(hosts_np[idx])
    assert np.array_equal(_u32(live)[idx], r_live), what
    e = est.cpu().numpy().astype(np.float64)[idx]
    assert np.all(np.abs(e - r_est) <= _tol(r_est, ref.g)), what


def _run_pair(members, n_slices, counts_fn, graph=True, tune_at=None, check_every=1, oracle=True,
              oracle_hosts=None, oracle_every=1, tunes=None):
    """Drive the members through a batch (eager first slice, then graph
    replays) and the same configs through standalone sketches and through
    oracle twins (Alg. 4's per-slice loop on the CPU); compare.  oracle_hosts
    caps the hosts per member whose estimates the oracle recomputes (a seeded
    sample); tunes maps a slice to launch shapes set before it."""
    dev = torch.device("cuda")
    cfgs = [Config(m.log2_pool, m.width, m.k, m.g, 0, m.seed, m.seed + 1) for m in members]
    hosts = []
    for m in members:
        g = torch.Generator(device=dev)
        g.manual_seed(m.seed)
        hosts.append(torch.randint(-2**31, 2**31, (m.n_hosts,), generator=g, device=dev, dtype=torch.int64)
                     .to(torch.int32))
    counts = [counts_fn(s) for s in range(n_slices)]
    caps = [int(max(c[i] for c in counts)) for i in range(len(members))]
    A = [Sketch(c) for c in cfgs]
    B = [Sketch(c) for c in cfgs]
    batch = Batch(A, caps, hosts)
    O = [OracleSketch(c.log2_pool, c.width, c.k, c.g, c.seed_a, c.seed_b, c.partition) for c in cfgs] \
        if oracle else []
    hosts_np = [h.cpu().numpy().view(np.uint32) for h in hosts]
    pick = np.random.default_rng(17)
    idx = [np.arange(h.size) if oracle_hosts is None or h.size <= oracle_hosts
           else np.sort(pick.choice(h.size, oracle_hosts, replace=False)) for h in hosts_np]
    timing = {"eager": [], "replay": []}
    report = None
    for s in range(n_slices):
        slices = [streams.member_slice_torch(m, hosts[i], s, int(counts[s][i]), dev)
                  for i, m in enumerate(members)]
        torch.cuda.synchronize()
        if tunes and s in tunes:
            batch.set_tune(tunes[s])
            if graph and s > 0:
                batch.capture()      # the graph holds the launch shapes it was captured with
        batch.load(slices)
        batch.synchronize()
        t0 = time.perf_counter()
        if s == 0 or not graph:
            batch.slice()
            kind = "eager"
        else:
            batch.replay()
            kind = "replay"
        batch.synchronize()
        timing[kind].append(time.perf_counter() - t0)
        if s == 0 and graph:
            batch.capture()
        if tune_at is not None and s == tune_at:
            before = [e.clone() for e in batch.est]
            report = batch.autotune()
            batch.synchronize()
            assert all(torch.equal(x, y) for x, y in zip(before, batch.est))
            if graph:
                batch.capture()
        # eager torch work between replays
        torch.randn(1 << 20, device=dev).sum().item()
        refs = []
        for i, sk in enumerate(B):
            sk.ingest(slices[i])
            sk.close_slice()
            refs.append(sk.estimate(hosts[i]))
        torch.cuda.synchronize()
        for i, ref in enumerate(O):
            ref.ingest(slices[i].cpu().numpy().view(np.uint32))
            ref.close_slice()
        if O and (s % oracle_every == 0 or s == n_slices - 1):
            batch.synchronize()
            for i, ref in enumerate(O):
                _check_oracle(A[i], batch.est[i], batch.live[i], ref, hosts_np[i], idx[i],
                              f"slice {s} member {i} ({'replay' if kind == 'replay' else 'eager'})")
        if s % check_every == 0 or s == n_slices - 1:
            for i in range(len(members)):
                pa, ta, ba, ca = A[i].read_state()
                pb, tb, bb, cb = B[i].read_state()
                assert (ta, ba, ca) == (tb, bb, cb), (s, i)
                assert np.array_equal(pa, pb), (s, i)
                assert torch.equal(batch.est[i], refs[i][0]), (s, i)
                assert torch.equal(batch.live[i], refs[i][1]), (s, i)
    return timing, report


def test_batch_graph_replay_equals_standalone():
    """Graph replays: every member, after every slice, bit-exact with its
    oracle twin (pool, clock, census, live counts; estimates within the bar)
    and identical to its standalone GPU twin."""
    members = _members_small()
    counts = lambda s: streams.batch_packet_counts(4, len(members), s, lo=3.0, hi=5.0)
    timing, _ = _run_pair(members, 12, counts, graph=True)
    assert len(timing["replay"]) == 11


def test_batch_autotune_keeps_results():
    """The autotuner leaves the slice's results unchanged, and the replays
    after it match the oracle twins slice by slice."""
    members = _members_small()[:8]
    counts = lambda s: streams.batch_packet_counts(5, len(members), s, lo=3.0, hi=5.0)
    _, report = _run_pair(members, 5, counts, graph=True, tune_at=1)
    assert "best" in report and report["tune"]["estimate_block"] in (64, 128, 256)
    assert report["tune"]["estimate_lanes"] in (1, 4, 16) and report["tune"]["census_unroll"] in (1, 2, 4)
    # every (tile, second axis, grid) candidate of the three tuned phases was timed
    assert len(report["candidates"]) == 12 + 36 + 36


def test_batch_tune_cache(tmp_path):
    """A choice stored in the JSON cache under the batch geometry is set
    again, without timing, for a batch of the same geometry; another geometry
    is tuned afresh; the cached shapes still give the oracle's results."""
    members = _members_small()[:6]
    counts = lambda s: streams.batch_packet_counts(7, len(members), s, lo=3.0, hi=5.0)
    cache = str(tmp_path / "tune.json")
    dev = torch.device("cuda")

    def run(ms, n_slices):
        cfgs = [Config(m.log2_pool, m.width, m.k, m.g, 0, m.seed, m.seed + 1) for m in ms]
        hosts = [torch.randint(-2**31, 2**31, (m.n_hosts,), device=dev, dtype=torch.int64).to(torch.int32)
                 for m in ms]
        cs = [counts(s)[: len(ms)] for s in range(n_slices)]
        b = Batch([Sketch(c) for c in cfgs], [int(max(c[i] for c in cs)) for i in range(len(ms))], hosts)
        refs = [OracleSketch(c.log2_pool, c.width, c.k, c.g, c.seed_a, c.seed_b, c.partition) for c in cfgs]
        rep = None
        for s in range(n_slices):
            sl = [streams.member_slice_torch(m, hosts[i], s, int(cs[s][i]), dev) for i, m in enumerate(ms)]
            b.load(sl)
            b.slice()
            b.synchronize()
            if s == 0:
                rep = b.autotune(cache=cache)
                b.synchronize()
            for i, r in enumerate(refs):
                r.ingest(sl[i].cpu().numpy().view(np.uint32))
                r.close_slice()
        hn = [h.cpu().numpy().view(np.uint32) for h in hosts]
        for i, r in enumerate(refs):
            _check_oracle(b.sketches[i], b.est[i], b.live[i], r, hn[i], np.arange(hn[i].size), f"member {i}")
        return b, rep

    b1, r1 = run(members, 3)
    assert r1["cached"] is False and r1["key"] == b1.geometry_key()
    b2, r2 = run(members, 3)
    assert r2["cached"] is True and r2["tune"] == r1["tune"]
    _, r3 = run(members[:5], 2)
    assert r3["cached"] is False
    import json
    assert set(json.load(open(cache))) == {r1["key"], r3["key"]}


def test_batch_two_tunings_match_oracle():
    """The same members under two hand-set launch shapes (small tiles and grids,
    then large ones), replayed from graphs captured under each: every slice
    matches the oracle twins."""
    members = _members_small()[:10]
    counts = lambda s: streams.batch_packet_counts(6, len(members), s, lo=3.0, hi=5.0)
    small = {"ingest_tile": 512, "census_tile": 256, "estimate_block": 64, "grid_preserve": 7,
             "grid_ingest": 13, "grid_census": 11, "grid_estimate": 9, "estimate_lanes": 16,
             "census_unroll": 4}
    large = {"ingest_tile": 32768, "census_tile": 16384, "estimate_block": 256, "grid_preserve": 512,
             "grid_ingest": 4096, "grid_census": 2048, "grid_estimate": 8192, "estimate_lanes": 4,
             "census_unroll": 2}
    _run_pair(members, 8, counts, graph=True, tunes={0: small, 4: large})


def test_batch_full_size_16_sketches():
    """16 sketches, pools 2^20..2^26, 1e5..1e7 packets per sketch per slice,
    g = 1024: eager first slice, autotune, captured graph replays; each member
    bit-exact with its standalone twin at every slice, and with its oracle
    twin (pool, census; live counts and estimates of 512 sampled hosts) at the
    eager slice, after the autotuner and at the last replay."""
    members = streams.batch_members(seed=4)
    counts = lambda s: streams.batch_packet_counts(4, len(members), s)
    timing, report = _run_pair(members, 5, counts, graph=True, tune_at=1, oracle_hosts=512, oracle_every=2)
    print("batch timing (s)", timing, "tune", report["tune"] if report else None)

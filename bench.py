"""VATE hot-path benchmark on one MI355X.

One step = one 1 s time slice of the 40 Gb/s-shaped workload, the whole hot
path: advance + two-block preservation, ingest of 5M packets (SetAT), pool
census, and estimation of all 1M ANet hosts over the k = 60 slice window,
both by the closed form (Eq. 11) and by the learned estimator (one pass over
the VATs gives both).  Inputs (the packet stream and host list) are resident
in HBM before the timed region starts.  After the timed region the learned
and closed-form estimators are compared on held-out probe episodes with
known cardinalities, and 16 independent sketches of mixed geometry are run
through the batched launches (graph replay against one-by-one calls).
Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-eval] [--no-batch] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("packets/s AT update + hosts/s estimate on 1 GPU; "
          "learned vs closed-form rel. error")
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the code (comments and whitespace left out) of the sources that
    define the estimate-phase kernels."""
    import hashlib
    import re

    tok = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/|[^\s"\'/]+|\S', re.S)
    h = hashlib.sha256()
    for f in ("vate.hip", "vate_core.h", "vate_part.h", "vate_exact.h", "mlp_core.h"):
        text = open(os.path.join(ROOT, "paper_1812_00282_amd", "csrc", f)).read()
        code = [t for t in tok.findall(text) if not t.startswith(("//", "/*"))]
        h.update(" ".join(code).encode())
    return h.hexdigest()[:16]


def measured_traffic(path=None):
    """HBM bytes per slice of the estimate phase (FETCH_SIZE + WRITE_SIZE of
    its kernels, calibrated) from a committed rocprofv3 summary, or None if the
    kernel sources have changed since the counters were taken."""
    import glob

    cur = kernel_source_hash()
    paths = [path] if path else sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")),
                                       key=os.path.getmtime, reverse=True)
    for p in paths:
        for line in open(p):
            if line.startswith("TRAFFIC estimate_phase"):
                fields = dict(f.split("=", 1) for f in line.split()[2:])
                if fields.get("kernel_src_sha256_16") == cur:
                    return float(fields["bytes_per_launch"]), os.path.relpath(p, ROOT)
    return None, None


def cpu_info() -> dict:
    """Host cores this process may use and the CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": usable, "cpu_count": os.cpu_count(), "model": model}


def _oracle_estimate_worker(ref, k, hosts, conn) -> None:
    """One all-core worker: the Z_p scan alone, then the oracle's estimate of
    its shard (which scans again); the difference is the per-host work."""
    t0 = time.perf_counter()
    ref.pool_inactive(k)
    t1 = time.perf_counter()
    ref.estimate(hosts, want_live=False)
    t2 = time.perf_counter()
    conn.send((t1 - t0, t2 - t1))
    conn.close()


def cpu_baseline(wl, pop, slices, sample_hosts: int = 4096, measured: int = 4,
                 max_workers: int = 16) -> dict:
    """The CPU oracle on the same stream, in steady state: k untimed slices
    fill the window, then `measured` slices are timed phase by phase -
    PT (advance + preservation of the due blocks), ST (ingest of the slice's
    packets) and ET (the pool scan behind Z_p plus the per-host estimate,
    timed on `sample_hosts` hosts per slice and scaled to all hosts).  An
    all-core leg then forks worker processes from the same oracle state and
    shards a larger host sample over them (each worker runs the oracle's
    unchanged estimate, its own Z_p scan included).  Reported in packets/s
    per whole slice (ST + PT + ET for every host)."""
    import multiprocessing as mp

    from oracle.vate_ref import OracleSketch

    info = cpu_info()
    ref = OracleSketch(wl.log2_pool, wl.width, wl.k, wl.g, 0xA5A5, 0x5A5A)
    n = len(slices)
    t0 = time.perf_counter()
    for s in range(wl.k):
        ref.ingest(slices[s % n])
        ref.close_slice()
    t_fill = time.perf_counter() - t0
    log(f"[bench] cpu oracle: window filled ({wl.k} slices, {t_fill:.1f} s)")
    empty = np.zeros((0, 2), dtype=np.uint32)
    rng = np.random.default_rng(12345)
    st, pt, et_call = [], [], []
    for j in range(measured):
        s = wl.k + j
        t0 = time.perf_counter()
        ref.ingest(empty)                 # the closed slice advances: BACT0, t, Alg. 3
        t1 = time.perf_counter()
        ref.ingest(slices[s % n])         # SetAT for every packet
        t2 = time.perf_counter()
        ref.close_slice()
        hosts = pop.aips[rng.choice(pop.n_hosts, size=sample_hosts, replace=False)]
        t3 = time.perf_counter()
        ref.estimate(hosts, want_live=False)
        t4 = time.perf_counter()
        pt.append(t1 - t0)
        st.append(t2 - t1)
        et_call.append(t4 - t3)
        log(f"[bench] cpu oracle: slice {s} PT {pt[-1]:.3f} s, ST {st[-1]:.3f} s, "
            f"estimate of {sample_hosts} hosts {et_call[-1]:.2f} s")
    t0 = time.perf_counter()
    ref.pool_inactive(wl.k)
    t_scan = time.perf_counter() - t0
    per_host = max(float(np.mean(et_call)) - t_scan, 0.0) / sample_hosts
    st_s, pt_s = float(np.mean(st)), float(np.mean(pt))
    et_s = t_scan + per_host * pop.n_hosts
    slice_1 = st_s + pt_s + et_s

    # all-core leg: workers forked from this oracle state, each estimating a
    # shard of the host sample (fork: the 512 MiB pool is shared copy-on-write)
    workers = max(1, min(max_workers, info["nproc"]))
    shard = 4 * sample_hosts
    hosts = pop.aips[rng.choice(pop.n_hosts, size=workers * shard, replace=False)]
    ctx = mp.get_context("fork")
    procs, pipes = [], []
    t0 = time.perf_counter()
    for w in range(workers):
        a, b = ctx.Pipe(duplex=False)
        p = ctx.Process(target=_oracle_estimate_worker,
                        args=(ref, wl.k, hosts[w * shard:(w + 1) * shard], b))
        p.start()
        procs.append(p)
        pipes.append(a)
    worker_s = [c.recv() for c in pipes]
    for p in procs:
        p.join()
    wall = time.perf_counter() - t0
    # per-host work of each worker: its estimate minus its own Z_p scan
    busy = max(max(e - z for z, e in worker_s), 1e-9)
    per_host_all = busy / (workers * shard)
    et_all = t_scan + per_host_all * pop.n_hosts
    slice_all = st_s + pt_s + et_all
    log(f"[bench] cpu oracle: all-core estimate, {workers} workers x {shard} hosts, {wall:.2f} s")
    return {
        "value": wl.packets_per_slice / slice_all,
        "unit": "packets/s",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"the same stream in steady state: {wl.k} untimed slices fill the window, then "
                   f"{measured} slices timed per phase (PT advance+preserve, ST ingest of "
                   f"{wl.packets_per_slice} packets, ET = one Z_p pool scan + {sample_hosts} sampled "
                   f"hosts per slice scaled to all {pop.n_hosts}); value uses ET from the all-core leg "
                   f"({workers} forked workers x {shard} hosts; one Z_p scan + the hosts at the "
                   f"workers' combined rate), ST and PT single-threaded"),
        "cpu": info,
        "per_slice_s": {"ST": st_s, "PT": pt_s, "ET_one_core": et_s, "ET_all_cores": et_all,
                        "Z_p_scan": t_scan},
        "one_core": {"packets_per_s": wl.packets_per_slice / slice_1, "hosts_per_s": 1.0 / per_host,
                     "slice_s": slice_1},
        "all_cores": {"workers": workers, "packets_per_s": wl.packets_per_slice / slice_all,
                      "hosts_per_s": 1.0 / per_host_all, "slice_s": slice_all,
                      "worker_scan_and_estimate_s": [[round(z, 3), round(e, 3)] for z, e in worker_s]},
        "slices_timed": [wl.k, wl.k + measured - 1],
    }


def generate_slices(wl, pop, n: int) -> list:
    """The workload's first n slices (numpy, seeded per slice), drawn by a
    pool of threads (no fork: under a profiler the GPU is already open)."""
    from concurrent.futures import ThreadPoolExecutor

    workers = max(1, min(16, cpu_info()["nproc"], n))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda s: wl.slice(pop, s), range(n)))


def batched_leg(dev, n_slices: int = 8, tune_cache: str | None = None) -> dict:
    """16 independent sketches (pools 2^20..2^26, k in {8..128}, g = 1024,
    1e5..1e7 packets per sketch per slice) advanced a slice at a time by the
    batched launches: the first slice eager, then the autotuner, a captured
    graph and graph replays; the same sketches driven one after another
    through the single-sketch calls give the comparison, and the last slice's
    estimates of the two must be identical."""
    import torch

    from paper_1812_00282_amd import streams
    from paper_1812_00282_amd.batch import Batch
    from paper_1812_00282_amd.sketch import Config, Sketch

    members = streams.batch_members(seed=4)
    cfgs = [Config(m.log2_pool, m.width, m.k, m.g, 0, m.seed, m.seed + 1) for m in members]
    hosts = []
    for m in members:
        gen = torch.Generator(device=dev)
        gen.manual_seed(m.seed)
        hosts.append(torch.randint(-2**31, 2**31, (m.n_hosts,), generator=gen, device=dev,
                                   dtype=torch.int64).to(torch.int32))
    counts = [streams.batch_packet_counts(4, len(members), s) for s in range(n_slices)]
    caps = [int(max(c[i] for c in counts)) for i in range(len(members))]
    slices = [[streams.member_slice_torch(m, hosts[i], s, int(counts[s][i]), dev)
               for i, m in enumerate(members)] for s in range(n_slices)]
    batch = Batch([Sketch(c, device=dev) for c in cfgs], caps, hosts)
    times, tune = [], None
    for s in range(n_slices):
        batch.load(slices[s])
        batch.synchronize()
        t0 = time.perf_counter()
        if s == 0:
            batch.slice()
        else:
            batch.replay()
        batch.synchronize()
        times.append(time.perf_counter() - t0)
        if s == 0:
            t0 = time.perf_counter()
            rep = batch.autotune(cache=tune_cache)
            tune = dict(rep["tune"], cached=rep["cached"], key=batch.geometry_key(), cache=tune_cache,
                        seconds=time.perf_counter() - t0,
                        candidates=len(rep.get("candidates", [])))
            batch.capture()
    solo = [Sketch(c, device=dev) for c in cfgs]
    seq = []
    for s in range(n_slices):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = []
        for i, sk in enumerate(solo):
            sk.ingest(slices[s][i])
            sk.close_slice()
            outs.append(sk.estimate(hosts[i])[0])
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t0)
    identical = all(torch.equal(batch.est[i], outs[i]) for i in range(len(members)))
    replay_ms = float(np.median(times[2:])) * 1e3
    seq_ms = float(np.median(seq[2:])) * 1e3
    pkts = float(np.mean([c.sum() for c in counts[2:]]))
    hosts_n = sum(m.n_hosts for m in members)
    return {"sketches": len(members), "packets_per_slice": pkts, "hosts_per_slice": hosts_n,
            "eager_first_slice_ms": times[0] * 1e3, "graph_replay_ms": replay_ms,
            "one_by_one_ms": seq_ms, "packets_per_s": pkts / (replay_ms * 1e-3),
            "speedup_vs_one_by_one": seq_ms / replay_ms, "identical_to_one_by_one": identical,
            "tune": tune}


def blocked_leg(dev, slices, hosts, held_independent, block_log2: int = 6, steps: int = 10) -> dict:
    """The opt-in locality-blocked H (blocks of 2^b consecutive VATs; not the
    paper's H) on the same 40 Gb/s stream: estimate time for all 1M hosts
    (closed form, window k: the whole-block popcount gather; with the
    distance histogram: the per-VAT gather), and the closed form's accuracy on
    the held-out probe episodes against the independent H."""
    import torch

    from paper_1812_00282_amd import streams
    from paper_1812_00282_amd import train as T
    from paper_1812_00282_amd.sketch import Config, Sketch

    wl = streams.LINK40G
    cfg = Config(wl.log2_pool, wl.width, wl.k, wl.g, seed_a=0xA5A5, seed_b=0x5A5A, block_log2=block_log2)
    sk = Sketch(cfg, device=dev)
    est = torch.empty(hosts.numel(), dtype=torch.float32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    hist = torch.empty((hosts.numel(), wl.k + 1), dtype=torch.int32, device=dev)
    direct, with_hist = [], []
    for s in range(4 + steps):
        sk.ingest(slices[s % len(slices)])
        sk.close_slice()
        ev[0].record()
        sk.estimate(hosts, want_live=False, out=(est, None, None))
        ev[1].record()
        sk.estimate(hosts, want_live=False, out=(est, None, hist))
        ev[2].record()
        torch.cuda.synchronize()
        if s >= 4:
            direct.append(ev[0].elapsed_time(ev[1]))
            with_hist.append(ev[1].elapsed_time(ev[2]))
    del sk
    torch.cuda.empty_cache()
    bg = T.background(T.BG_SLICES, dev)
    held = T.generate(T.HELD_OUT_SEEDS[:2], bg, device=dev, block_log2=block_log2)
    return {"block_log2": block_log2, "hosts": hosts.numel(),
            "estimate_ms": float(np.median(direct)), "estimate_ms_with_histogram": float(np.median(with_hist)),
            "closed_form_rel_error": T.closed_form_error(held),
            "closed_form_rel_error_independent_h": T.closed_form_error(held_independent)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eval", action="store_true",
                    help="skip the learned vs closed-form comparison on held-out episodes")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-sketches leg (16 sketches, hipGraph replay)")
    ap.add_argument("--no-blocked", action="store_true",
                    help="skip the locality-blocked H leg (opt-in variant, not the paper's H)")
    ap.add_argument("--tune-cache", default=os.environ.get(
                        "VATE_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "vate", "batch_tune.json")),
                    help="JSON file of autotuned batch launch shapes, keyed by the batch geometry "
                         "('' to autotune every run without a cache)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    ap.add_argument("--profile-summary", default=None,
                    help="rocprofv3 summary holding the dominant kernel's HBM traffic "
                         "(default: the newest profiles/*.txt with a TRAFFIC line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the VATE "
              "path here is a single-GPU build.", file=sys.stderr)
        return 2

    import torch

    from paper_1812_00282_amd import learned as L
    from paper_1812_00282_amd import streams
    from paper_1812_00282_amd import train as T
    from paper_1812_00282_amd.sketch import Config, Sketch

    wl = streams.LINK40G
    n_gen = wl.n_slices
    log(f"[bench] generating {n_gen} slices of {wl.name}")
    pop = wl.population()
    host_slices = generate_slices(wl, pop, n_gen)
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the all-core leg forks worker processes
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(wl, pop, host_slices)
    dev = torch.device("cuda:0")
    slices = [torch.from_numpy(s.view(np.int32)).to(dev) for s in host_slices]
    hosts = torch.from_numpy(pop.aips.view(np.int32)).to(dev)
    cfg = Config(wl.log2_pool, wl.width, wl.k, wl.g, seed_a=0xA5A5, seed_b=0x5A5A)
    sk = Sketch(cfg, device=dev)
    est = torch.empty(pop.n_hosts, dtype=torch.float32, device=dev)
    est_cf = torch.empty(pop.n_hosts, dtype=torch.float32, device=dev)
    if os.path.exists(T.WEIGHTS):
        theta = T.load(device=dev)
        weights_src = os.path.relpath(T.WEIGHTS, ROOT)
    else:
        theta = T.init_theta(0, dev)
        weights_src = "untrained (zero output layer: equals the closed form)"
    weights = L.pack(theta, L.new_weights(dev))
    envelope = T.load_envelope() if os.path.exists(T.WEIGHTS) else None
    L.set_envelope(weights, envelope)      # hosts outside the training envelope get the closed form
    L.learned_workspace(sk, pop.n_hosts)
    torch.cuda.synchronize()

    def step(s, ev=None):
        if ev is not None:
            ev[0].record()
        sk.ingest(slices[s % n_gen])        # advance + preserve, then SetAT
        if ev is not None:
            ev[1].record()
        sk.close_slice()                    # census
        if ev is not None:
            ev[2].record()
        L.estimate_learned(sk, hosts, weights, out=(est, est_cf), partitioned=True)
        if ev is not None:
            ev[3].record()

    if args.copy_calibration:
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy of 1 GiB done")
        del src, dst
    # steady state: the window of k slices fills before anything is timed
    # (2k untimed slices, cycling the generated ones), whatever --warmup is
    preroll = 2 * wl.k
    log(f"[bench] pre-roll {preroll} slices, then warmup {args.warmup}")
    for s in range(preroll + args.warmup):
        step(s)
        if (s + 1) % 20 == 0:
            torch.cuda.synchronize()
            log(f"[bench] slice {s + 1} of {preroll + args.warmup} untimed")
    torch.cuda.synchronize()
    first = preroll + args.warmup
    L.fallbacks(weights, reset=True)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    log(f"[bench] timing {args.steps} steps (slices {first}..{first + args.steps - 1})")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(first + i, events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fell = L.fallbacks(weights, reset=True)
    ingest_ms = np.mean([e[0].elapsed_time(e[1]) for e in events])
    census_ms = np.mean([e[1].elapsed_time(e[2]) for e in events])
    est_ms = np.mean([e[2].elapsed_time(e[3]) for e in events])
    ms_per_step = elapsed * 1e3 / args.steps

    # update alone, and with the slice's host-to-device copy from pinned memory
    staged = torch.empty_like(slices[0])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    h2d, upd = [], []
    for r in range(5):
        pinned = torch.from_numpy(host_slices[(first + args.steps + r) % n_gen].view(np.int32)).pin_memory()
        ev[0].record()
        staged.copy_(pinned, non_blocking=True)
        ev[1].record()
        sk.ingest(staged)                   # the closed slice advances and preserves first
        ev[2].record()
        sk.close_slice()
        torch.cuda.synchronize()
        h2d.append(ev[0].elapsed_time(ev[1]))
        upd.append(ev[1].elapsed_time(ev[2]))
    update = {"packets_per_s": wl.packets_per_slice / (float(np.median(upd)) * 1e-3),
              "packets_per_s_with_h2d": wl.packets_per_slice / ((float(np.median(upd)) +
                                                                  float(np.median(h2d))) * 1e-3),
              "h2d_ms": float(np.median(h2d)),
              "note": "median of 5 ingest calls, each incl. the advance + preservation of the closed slice"}

    # the same slices with the host list planned once (the VAT addresses do
    # not depend on the pool): lookups, histograms and both estimates only
    sk.plan(hosts)
    torch.cuda.synchronize()
    pev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        sk.ingest(slices[(first + args.steps + 5 + i) % n_gen])
        sk.close_slice()
        pev[i][0].record()
        L.estimate_learned_run(sk, weights, out=(est, est_cf))
        pev[i][1].record()
    torch.cuda.synchronize()
    planned = {"ms_per_step": (time.perf_counter() - t0) * 1e3 / args.steps,
               "estimate_ms": float(np.mean([e[0].elapsed_time(e[1]) for e in pev])),
               "note": "host list planned once (vate_estimate_plan); not the headline value"}

    # dominant phase: the per-host estimate (VAT lookups + both estimates)
    bytes_per_host = 4 + wl.g * wl.width // 8 + 8
    achieved = bytes_per_host * pop.n_hosts / (est_ms * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic(args.profile_summary)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_source": traffic_src,
                "kernel": "estimate phase: k_run_scatter + k_run_lookup<8> + k_run_finalize<learned>",
                "algorithmic_bytes_per_launch": bytes_per_host * pop.n_hosts,
                "avg_launch_ms": est_ms,
                "traffic_gbs": traffic / (est_ms * 1e-3) / 1e9 if traffic else None,
                "traffic_frac": traffic / (est_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                "lookups_per_s": wl.g * pop.n_hosts / (est_ms * 1e-3),
                # VAT lookups per second against the rate a random-gather
                # design could reach if HBM served one 64-byte sector per
                # lookup at peak (context for the lookup design; the roofline
                # figure is frac, and traffic_frac for the bytes moved)
                "lookups_vs_random_gather_bound": wl.g * pop.n_hosts / (est_ms * 1e-3)
                / (HBM_PEAK_GBS * 1e9 / 64)}

    line = {
        "metric": METRIC,
        "value": wl.packets_per_slice * args.steps / elapsed,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl.name, "packets_per_slice": wl.packets_per_slice,
                   "hosts": pop.n_hosts, "log2_pool": wl.log2_pool, "width": wl.width,
                   "k": wl.k, "kprime": wl.k, "g": wl.g, "slices_generated": n_gen,
                   "slices_preroll": preroll, "slices_timed": [first, first + args.steps - 1]},
        "hosts_per_s": pop.n_hosts * args.steps / elapsed,
        "phases_ms": {"advance_preserve_ingest": ingest_ms, "census": census_ms,
                      "estimate": est_ms},
        "update": update,
        "planned_hosts": planned,
        "real_time_margin": 1000.0 / ms_per_step,    # 1 s slices (Sec. 5's real-time criterion)
        "learned_fallback": {"hosts_per_slice": fell / args.steps,
                             "fraction": fell / (args.steps * pop.n_hosts),
                             "envelope": None if envelope is None else
                             {"k": envelope["k"], "g": envelope["g"], "log2_pool": envelope["log2_pool"],
                              "width": envelope["width"]},
                             "note": "hosts of the timed slices given the closed form because a feature "
                                     "lies outside the network's training range"},
        "roofline": roofline,
    }
    held = None
    if not args.no_eval:
        log("[bench] learned vs closed form on held-out probe episodes")
        bg = T.background(T.BG_SLICES, dev)
        held = T.generate(T.HELD_OUT_SEEDS[:2], bg, device=dev)
        line["learned_vs_closed_form"] = {"weights": weights_src,
                                          **T.evaluate(theta, held, device=dev, env=envelope)}
        del bg
    if not args.no_blocked and held is not None:
        log("[bench] locality-blocked H (opt-in variant)")
        line["blocked_h"] = blocked_leg(dev, slices, hosts, held)
    if not args.no_batch:
        log("[bench] batched sketches")
        del sk
        torch.cuda.empty_cache()
        line["batched"] = batched_leg(dev, tune_cache=args.tune_cache or None)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

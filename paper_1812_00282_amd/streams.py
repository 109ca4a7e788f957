"""Seeded synthetic packet streams shaped like the paper's workloads.

This module only draws (aip, bip) pairs; it holds none of VATE's arithmetic
(no hashing, no AT values, no estimation), so both the HIP path and the CPU
oracle can consume its output.

The paper measures on one hour of CAIDA (10 Gb/s) and IPtas/CERNET (40 Gb/s)
traffic (Sec. 5) that is not available here; these generators stand in for it
with the shapes the paper reports: 1 s slices, heavy-tailed per-host
cardinalities with most hosts below 5000 (Sec. 5, Fig. 8), and ~5M packets per
slice for a 40 Gb/s link.

A population is a set of ANet hosts (distinct uniform 32-bit aips), each with
a universe of n_h opposite hosts (uniform 32-bit bips) and an activity weight.
A slice draws P packets: per-host packet counts from a multinomial over the
activity weights, shuffled, and each packet's bip uniform from its host's
universe.
Slice s of a stream is generated from its own child seed, so any slice can be
produced independently of the others.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _distinct_u32(rng: np.random.Generator, n: int) -> np.ndarray:
    out = np.unique(rng.integers(0, 2**32, size=int(n * 1.05) + 16, dtype=np.uint64))
    while out.size < n:
        more = rng.integers(0, 2**32, size=n, dtype=np.uint64)
        out = np.unique(np.concatenate([out, more]))
    rng.shuffle(out)
    return out[:n].astype(np.uint32)


@dataclass
class Population:
    aips: np.ndarray        # (H,) uint32 distinct host ids
    card: np.ndarray        # (H,) int64 universe size n_h
    weight: np.ndarray      # (H,) float64 activity probabilities, sum 1
    universe: np.ndarray    # (sum n_h,) uint32 opposite hosts, host-major
    offset: np.ndarray      # (H,) int64 start of each host's universe

    @property
    def n_hosts(self) -> int:
        return int(self.aips.size)


def make_population(seed: int, n_hosts: int, alpha: float, card_max: int,
                    activity: str = "card", zipf_s: float = 1.1) -> Population:
    """Hosts with n_h = clip(floor(Pareto(alpha, x_m=1)), 1, card_max).

    activity="card": host drawn with probability proportional to n_h;
    activity="zipf": Zipf(s) weights over a random rank permutation,
    independent of n_h.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xC0FFEE]))
    aips = _distinct_u32(rng, n_hosts)
    card = np.floor(rng.pareto(alpha, size=n_hosts) + 1.0)
    card = np.clip(card, 1, card_max).astype(np.int64)
    if activity == "card":
        w = card.astype(np.float64)
    elif activity == "zipf":
        ranks = rng.permutation(n_hosts).astype(np.float64) + 1.0
        w = ranks ** (-zipf_s)
    else:
        raise ValueError(activity)
    w = w / w.sum()
    offset = np.zeros(n_hosts, dtype=np.int64)
    np.cumsum(card[:-1], out=offset[1:])
    universe = rng.integers(0, 2**32, size=int(card.sum()), dtype=np.uint64).astype(np.uint32)
    return Population(aips, card, w, universe, offset)


def draw_slice(pop: Population, seed: int, s: int, n_packets: int) -> np.ndarray:
    """(n_packets, 2) uint32 array of (aip, bip) pairs for slice s."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x51CE, s]))
    # per-host packet counts ~ Multinomial(n_packets, weight), in random order
    h = np.repeat(np.arange(pop.n_hosts), rng.multinomial(n_packets, pop.weight))
    rng.shuffle(h)
    j = (rng.random(n_packets) * pop.card[h]).astype(np.int64)
    out = np.empty((n_packets, 2), dtype=np.uint32)
    out[:, 0] = pop.aips[h]
    out[:, 1] = pop.universe[pop.offset[h] + j]
    return out


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    n_hosts: int
    alpha: float
    card_max: int
    activity: str
    packets_per_slice: int
    n_slices: int
    log2_pool: int
    width: int
    k: int
    g: int

    def population(self) -> Population:
        return make_population(self.seed, self.n_hosts, self.alpha, self.card_max,
                               self.activity)

    def slice(self, pop: Population, s: int) -> np.ndarray:
        return draw_slice(pop, self.seed, s, self.packets_per_slice)


# Plain VATE, CPU-sized: 2^16 x 8-bit ATs, g=128, k=4, 8 slices of 25k
# packets, 1000 hosts with Pareto(1.2) cardinality clipped to [1, 2000].
SMALL = Workload("small-2^16x8b-g128-k4", seed=1, n_hosts=1000, alpha=1.2,
                 card_max=2000, activity="card", packets_per_slice=25_000,
                 n_slices=8, log2_pool=16, width=8, k=4, g=128)

# 40 Gb/s-shaped stream: 5M packets per 1 s slice, 64 slices, k=60, 1M hosts
# (Zipf 1.1 activity, Pareto(1.1) cardinality up to 1e5), 2^28 x 8-bit ATs,
# g=1024.
LINK40G = Workload("40G-2^28x8b-g1024-k60", seed=2, n_hosts=1_000_000, alpha=1.1,
                   card_max=100_000, activity="zipf", packets_per_slice=5_000_000,
                   n_slices=64, log2_pool=28, width=8, k=60, g=1024)


def sweep_workload(k: int, width: int, log2_pool: int) -> Workload:
    """Window/width sweep on the small stream, run for 3k+8 slices so that
    every block's ACT wraps and every preservation phase occurs."""
    return Workload(f"sweep-2^{log2_pool}x{width}b-g128-k{k}", seed=3 * 1000 + k,
                    n_hosts=1000, alpha=1.2, card_max=2000, activity="card",
                    packets_per_slice=25_000, n_slices=3 * k + 8,
                    log2_pool=log2_pool, width=width, k=k, g=128)


SWEEP = [(2, 4, 26), (16, 8, 27), (64, 8, 28), (256, 16, 29)]


# --------------------------------------------------------------------------
# Batched sketches: 16 independent sketches with windows k in {8..128},
# 8-bit ATs (16-bit for k = 128), pools 2^20..2^26, g = 1024, hosts per
# sketch proportional to 2^(c-8), packets per sketch per slice
# floor(10^U(5, 7)).
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class BatchMember:
    log2_pool: int
    width: int
    k: int
    g: int
    n_hosts: int
    seed: int


def batch_members(seed: int = 4, n: int = 16, pool_range=(20, 26), g: int = 1024,
                  host_shift: int = 8) -> list[BatchMember]:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xBA7C]))
    out = []
    for i in range(n):
        k = int(rng.choice([8, 16, 32, 64, 128]))
        c = int(rng.integers(pool_range[0], pool_range[1] + 1))
        out.append(BatchMember(c, 16 if k == 128 else 8, k, g, 2 ** (c - host_shift),
                               seed * 1000 + i))
    return out


def batch_packet_counts(seed: int, n_members: int, s: int, lo: float = 5.0, hi: float = 7.0) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xC0C0, s]))
    return np.floor(10.0 ** rng.uniform(lo, hi, size=n_members)).astype(np.int64)


def member_slice_torch(m: BatchMember, hosts, s: int, n_packets: int, device):
    """(n, 2) int32 pairs on the device: host uniform over the member's host
    list, bip from a per-host universe of 256 (repeated contacts)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(m.seed * 100003 + s)
    h = torch.randint(0, hosts.numel(), (n_packets,), generator=g, device=device)
    j = torch.randint(0, 256, (n_packets,), generator=g, device=device, dtype=torch.int64)
    aip = hosts[h].to(torch.int64)
    bip = (aip * 0x9E37 + j * 0x85EBCA6B + 0x1234567) % (2**32)
    bip = bip - (bip >= 2**31).to(torch.int64) * 2**32
    return torch.stack([hosts[h], bip.to(torch.int32)], 1).contiguous()

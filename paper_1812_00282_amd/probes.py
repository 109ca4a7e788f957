"""Seeded probe-host traffic with exactly known window cardinalities.

Used to produce (sketch state, true cardinality) pairs for the learned
estimator.  It only draws (aip, bip) pairs and counts distinct bips per
window; it holds none of VATE's arithmetic.  Everything runs on the GPU with
torch's counter-based generator, seeded per episode.

A probe host has a universe of M distinct opposite hosts (bip = base + j*odd
mod 2^32, j < M) and an activity profile over the episode: steady, bursty
(each slice on with probability d), starting at a random slice, or stopping at
a random slice.  While on, it sends Poisson(rho) packets per slice, each to a
uniform universe member.  M and rho are set from a target window cardinality
T drawn log-uniform in [1, 1e6] and a coverage factor f in [1.2, 4]
(M = T f, rho chosen so that the expected number of distinct members hit in
k active slices is T).  The exact cardinality of every probe over the window
W(t-k+1, k) is counted from the last slice each universe member was hit.
"""
from __future__ import annotations

import math

import torch

STEADY, BURSTY, START, STOP = 0, 1, 2, 3


class ProbeEpisode:
    def __init__(self, seed: int, n_probes: int, n_slices: int, k: int, device="cuda",
                 t_max: float = 1e6, max_universe: int = 4_000_000):
        self.device = torch.device(device)
        self.gen = torch.Generator(device=self.device)
        self.gen.manual_seed(int(seed))
        self.k, self.n_slices, self.P = k, n_slices, n_probes
        g, dev = self.gen, self.device
        u = lambda *s: torch.rand(*s, generator=g, device=dev, dtype=torch.float64)
        T = torch.exp(u(n_probes) * math.log(t_max))
        f = torch.exp(math.log(1.2) + u(n_probes) * (math.log(4.0) - math.log(1.2)))
        M = torch.clamp(torch.ceil(T * f), 1, max_universe).to(torch.int64)
        self.kind = torch.randint(0, 4, (n_probes,), generator=g, device=dev)
        self.duty = 0.2 + 0.7 * u(n_probes)
        self.t_on = torch.randint(0, n_slices, (n_probes,), generator=g, device=dev)
        duty = torch.where(self.kind == BURSTY, self.duty, torch.ones_like(self.duty))
        S = torch.clamp(duty * k, min=1.0)
        frac = torch.clamp(T / M, max=1.0 - 1e-9)
        self.rate = (-(M.to(torch.float64) / S) * torch.log1p(-frac)).to(torch.float32)
        self.M = M
        self.offset = torch.zeros(n_probes, dtype=torch.int64, device=dev)
        self.offset[1:] = torch.cumsum(M, 0)[:-1]
        self.total = int(M.sum().item())
        self.aip = torch.randint(0, 2**32, (n_probes,), generator=g, device=dev, dtype=torch.int64)
        self.base = torch.randint(0, 2**32, (n_probes,), generator=g, device=dev, dtype=torch.int64)
        self.mult = torch.randint(0, 2**31, (n_probes,), generator=g, device=dev, dtype=torch.int64) * 2 + 1
        never = -(1 << 30)
        self.last = torch.full((self.total,), never, dtype=torch.int32, device=dev)

    def aips_i32(self) -> torch.Tensor:
        """Probe aips as int32 tensors holding the uint32 bits."""
        return (self.aip - (self.aip >= 2**31).to(torch.int64) * 2**32).to(torch.int32)

    def on(self, t: int) -> torch.Tensor:
        coin = torch.rand(self.P, generator=self.gen, device=self.device, dtype=torch.float64)
        on = torch.ones(self.P, dtype=torch.bool, device=self.device)
        on = torch.where(self.kind == BURSTY, coin < self.duty, on)
        on = torch.where(self.kind == START, torch.full_like(on, True) & (t >= self.t_on), on)
        on = torch.where(self.kind == STOP, torch.full_like(on, True) & (t < self.t_on), on)
        return on

    def slice(self, t: int) -> torch.Tensor:
        """(n, 2) int32 (aip, bip) pairs of slice t; updates the last-hit table."""
        on = self.on(t)
        lam = torch.where(on, self.rate, torch.zeros_like(self.rate))
        cnt = torch.poisson(lam, generator=self.gen).to(torch.int64)
        h = torch.repeat_interleave(torch.arange(self.P, device=self.device), cnt)
        j = torch.floor(torch.rand(h.numel(), generator=self.gen, device=self.device,
                                   dtype=torch.float64) * self.M[h].to(torch.float64)).to(torch.int64)
        j = torch.minimum(j, self.M[h] - 1)
        self.last[self.offset[h] + j] = t
        bip = (self.base[h] + j * self.mult[h]) % (2**32)
        aip = self.aip[h]
        pairs = torch.stack([aip, bip], 1)
        pairs = pairs - (pairs >= 2**31).to(torch.int64) * 2**32
        return pairs.to(torch.int32).contiguous()

    def truth(self, t: int) -> torch.Tensor:
        """Exact distinct bips of every probe over W(t-k+1, k) (Def. 1)."""
        hit = (self.last >= t - self.k + 1).to(torch.int64)
        cs = torch.cumsum(hit, 0)
        end = cs[self.offset + self.M - 1]
        start = torch.where(self.offset > 0, cs[torch.clamp(self.offset - 1, min=0)],
                            torch.zeros_like(end))
        return end - start

"""Learned VATE estimator: state generation, training and evaluation on the GPU.

States come from the plain method itself: a 2^28 x 8-bit sketch (g = 1024,
k = 60) runs the 40 Gb/s-shaped background stream plus probe hosts with known
window cardinalities (probes.py); at the end of every slice the probes'
distance histograms are read with vate_estimate and turned into features
(vate_mlp_features).  Training runs the library's BF16 matrix-core kernels
(vate_mlp_train_step, vate_mlp_adam); evaluation compares exp(network) with
the closed form of Eq. 11 against the exact cardinalities.

    python -m paper_1812_00282_amd.train [--states 10000000] [--epochs 12]

writes the trained parameters to weights/learned_40G_k60_g1024.npz and the
held-out evaluation next to it (.json).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import learned as L
from . import streams
from .probes import ProbeEpisode
from .sketch import Config, Sketch

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "learned_40G_k60_g1024.npz")
HELD_OUT_SEEDS = list(range(50, 60))
# Distinct 40 Gb/s background slices the episodes cycle through: at least the
# window k = 60, so the pool's occupancy reaches that of the stream itself.
BG_SLICES = 64
BUCKETS = [(1, 100), (100, 5000), (5000, float("inf"))]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@dataclass
class StateSet:
    x: torch.Tensor       # (n, 64) int16 bf16 features
    r: torch.Tensor       # (n,) ln max(closed form, 1)
    y: torch.Tensor       # (n,) ln true cardinality
    cf: torch.Tensor      # (n,) closed-form estimate
    truth: torch.Tensor   # (n,) true cardinality

    def __len__(self):
        return self.x.shape[0]


def background(n_slices: int = BG_SLICES, device="cuda") -> list[torch.Tensor]:
    """Slices 1000.. of the 40 Gb/s stream on the device (drawn by threads)."""
    from concurrent.futures import ThreadPoolExecutor

    wl = streams.LINK40G
    pop = wl.population()
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        host = list(ex.map(lambda s: wl.slice(pop, 1000 + s), range(n_slices)))
    return [torch.from_numpy(h.view(np.int32)).to(device) for h in host]


def generate(seeds, bg, k=60, g=1024, log2_pool=28, n_slices=100, t0=8, device="cuda",
             probes_range=(64, 512), bg_range=(0.2, 1.0), block_log2=0) -> StateSet:
    cfg = Config(log2_pool, 8, k, g, seed_a=0x1EA7, seed_b=0x2EA7, block_log2=block_log2)
    xs, rs, ys, cfs, trs = [], [], [], [], []
    for seed in seeds:
        rng = np.random.default_rng(seed)
        P = int(round(math.exp(rng.uniform(math.log(probes_range[0]), math.log(probes_range[1])))))
        frac = rng.uniform(*bg_range)
        ep = ProbeEpisode(seed, P, n_slices, k, device=device)
        sk = Sketch(cfg, device=device)
        aips = ep.aips_i32()
        for t in range(n_slices):
            b = bg[t % len(bg)]
            sk.ingest(b[: int(frac * b.shape[0])])
            sk.ingest(ep.slice(t))
            sk.close_slice()
            if t < t0:
                continue
            est, _, hist = sk.estimate(aips, want_live=False, want_hist=True)
            cen = sk.census()
            occ = float(cfg_active_fraction(cen, k, log2_pool))
            x, r = L.features(hist, est, k, g, occ)
            tr = ep.truth(t)
            keep = tr >= 1
            xs.append(x[keep]); rs.append(r[keep]); cfs.append(est[keep])
            trs.append(tr[keep].to(torch.float32)); ys.append(torch.log(tr[keep].to(torch.float32)))
        del sk, ep
    return StateSet(torch.cat(xs), torch.cat(rs), torch.cat(ys), torch.cat(cfs), torch.cat(trs))


def cfg_active_fraction(census: np.ndarray, k: int, log2_pool: int) -> float:
    n = 2**log2_pool
    return (n - int(census[k])) / n


def init_theta(seed: int, device) -> torch.Tensor:
    """He-initialised hidden layers, zero output layer (starts at the closed form)."""
    g = torch.Generator().manual_seed(seed)
    th = torch.zeros(L.MLP_PARAMS, dtype=torch.float32)
    th[0:4096] = torch.randn(4096, generator=g) * math.sqrt(2.0 / 64)
    th[4160:8256] = torch.randn(4096, generator=g) * math.sqrt(2.0 / 64)
    return th.to(device)


def train(data: StateSet, epochs=6, batch=4096, lr=2e-3, seed=0, device="cuda", verbose=True):
    theta = init_theta(seed, device)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    w = L.pack(theta, L.new_weights(device))
    n = len(data)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    step = 0
    history = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=device)
        acc = 0.0
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb, rb, yb = data.x[idx].contiguous(), data.r[idx].contiguous(), data.y[idx].contiguous()
            L.fill(grad, 0.0)
            L.fill(loss, 0.0)
            L.train_step(w, xb, rb, yb, grad, loss)
            step += 1
            cur = lr * (0.02 + 0.98 * 0.5 * (1 + math.cos(math.pi * step / total)))
            L.adam(theta, grad, m, v, step, lr=cur)
            L.pack(theta, w)
            if b % 200 == 0:
                acc = loss.item()
        history.append(acc)
        if verbose:
            log(f"[train] epoch {ep} loss(last minibatch) {acc:.4f}")
    torch.cuda.synchronize()
    return theta, history


def closed_form_error(data: StateSet) -> dict:
    """Mean relative error of the closed form (clamped at 1), overall and by
    truth bucket."""
    tr = data.truth.double()
    cf = torch.clamp(data.cf.double(), min=1.0)
    err = torch.abs(cf - tr) / tr
    out = {"all": float(err.mean().item())}
    for lo, hi in BUCKETS:
        sel = (tr >= lo) & (tr < hi)
        out[f"[{lo},{hi})"] = float(err[sel].mean().item()) if sel.any() else None
    return out


def outside_envelope(data: StateSet, env: dict) -> torch.Tensor:
    """States with a feature outside the envelope's range (the rule the
    learned estimate kernels apply per host)."""
    xi = ((data.x.to(torch.int64) & 0xFFFF) << 16).to(torch.int32)
    xf = xi.view(torch.float32)
    lo = torch.from_numpy(np.asarray(env["lo"], dtype=np.float32)).to(xf.device)
    hi = torch.from_numpy(np.asarray(env["hi"], dtype=np.float32)).to(xf.device)
    return ((xf < lo) | (xf > hi)).any(dim=1)


def evaluate(theta: torch.Tensor, data: StateSet, device="cuda", env: dict | None = None) -> dict:
    """Mean relative errors of the network and of the closed form; with an
    envelope, states outside it take the closed form, as when served."""
    w = L.pack(theta, L.new_weights(device))
    o = L.forward(w, data.x, data.r)
    est = torch.exp(o.double())
    est = torch.where(torch.isfinite(est), est, data.cf.double())
    out = {"states": len(data)}
    if env is not None:
        off = outside_envelope(data, env)
        est = torch.where(off, data.cf.double(), est)
        out["outside_envelope"] = int(off.sum().item())
    tr = data.truth.double()
    cf = data.cf.double()

    def mre(e, sel):
        return float((torch.abs(e[sel] - tr[sel]) / tr[sel]).mean().item()) if sel.any() else None

    everything = torch.ones_like(tr, dtype=torch.bool)
    out["all"] = {"learned": mre(est, everything), "closed_form": mre(cf, everything),
                  "closed_form_clamped": mre(torch.clamp(cf, min=1.0), everything),
                  "n": int(everything.sum().item())}
    for lo, hi in BUCKETS:
        sel = (tr >= lo) & (tr < hi)
        out[f"[{lo},{hi})"] = {"learned": mre(est, sel), "closed_form": mre(cf, sel),
                               "closed_form_clamped": mre(torch.clamp(cf, min=1.0), sel),
                               "n": int(sel.sum().item())}
    return out


def envelope_of(data: StateSet, k=60, g=1024, log2_pool=28, width=8) -> dict:
    """The training envelope: the sketch geometry and every feature's range
    over the states (the BF16 values the network reads)."""
    xi = ((data.x.to(torch.int64) & 0xFFFF) << 16).to(torch.int32)
    xf = xi.view(torch.float32)
    return {"k": k, "g": g, "log2_pool": log2_pool, "width": width,
            "lo": xf.min(0).values.cpu().numpy().astype(np.float32),
            "hi": xf.max(0).values.cpu().numpy().astype(np.float32)}


def save(theta: torch.Tensor, path: str, meta: dict, env: dict | None = None) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    arrays = {"theta": theta.detach().cpu().numpy().astype(np.float32)}
    if env is not None:
        arrays.update(env_geo=np.array([env["k"], env["g"], env["log2_pool"], env["width"]], dtype=np.uint32),
                      env_lo=np.asarray(env["lo"], dtype=np.float32), env_hi=np.asarray(env["hi"], dtype=np.float32))
    np.savez(path, **arrays)
    with open(path.replace(".npz", ".json"), "w") as f:
        json.dump(meta, f, indent=1)


def load(path: str = WEIGHTS, device="cuda") -> torch.Tensor:
    with np.load(path, allow_pickle=False) as z:
        return torch.from_numpy(z["theta"].astype(np.float32)).to(device)


def load_envelope(path: str = WEIGHTS) -> dict | None:
    """The training envelope stored with the weights, or None."""
    with np.load(path, allow_pickle=False) as z:
        if "env_geo" not in z:
            return None
        k, g, c, w = (int(v) for v in z["env_geo"])
        return {"k": k, "g": g, "log2_pool": c, "width": w, "lo": z["env_lo"].copy(), "hi": z["env_hi"].copy()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--states", type=int, default=20_000_000)
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--envelope-only", type=int, default=0, metavar="EPISODES",
                    help="keep the trained weights in --out and store with them the envelope measured on "
                         "the first EPISODES training episodes (regenerated)")
    args = ap.parse_args()
    dev = torch.device("cuda")
    t0 = time.time()
    bg = background(BG_SLICES, dev)
    log(f"[train] background ready {time.time() - t0:.1f}s")
    if args.envelope_only:
        theta = load(args.out, dev)
        with open(args.out.replace(".npz", ".json")) as f:
            meta = json.load(f)
        parts = []
        for s0 in range(1000, 1000 + args.envelope_only, 8):
            parts.append(generate(range(s0, min(s0 + 8, 1000 + args.envelope_only)), bg, device=dev))
            log(f"[train] envelope: {s0 + 8 - 1000} episodes {time.time() - t0:.1f}s")
        data = StateSet(*(torch.cat([getattr(p, f) for p in parts]) for f in ("x", "r", "y", "cf", "truth")))
        meta["envelope"] = {"episodes": args.envelope_only, "states": len(data),
                            "note": "feature ranges of the first training episodes (seeds 1000+), regenerated"}
        save(theta, args.out, meta, envelope_of(data))
        print(json.dumps(meta["envelope"]), flush=True)
        return 0
    parts, have, seed = [], 0, 1000
    while have < args.states:
        chunk = generate(range(seed, seed + 8), bg, device=dev)
        parts.append(chunk)
        have += len(chunk)
        seed += 8
        log(f"[train] {have} states ({seed - 1000} episodes) {time.time() - t0:.1f}s")
    data = StateSet(*(torch.cat([getattr(p, f) for p in parts])[: args.states]
                      for f in ("x", "r", "y", "cf", "truth")))
    del parts
    held = generate(HELD_OUT_SEEDS, bg, device=dev)
    log(f"[train] held-out {len(held)} states {time.time() - t0:.1f}s")
    theta, hist = train(data, epochs=args.epochs, batch=args.batch, lr=args.lr)
    res = evaluate(theta, held)
    res_train = evaluate(theta, StateSet(*(getattr(data, f)[:1_000_000]
                                           for f in ("x", "r", "y", "cf", "truth"))))
    meta = {"train_states": len(data), "train_episodes": seed - 1000, "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "loss_history": hist,
            "held_out_seeds": HELD_OUT_SEEDS, "held_out": res, "train_subset": res_train,
            "seconds": time.time() - t0}
    save(theta, args.out, meta, envelope_of(data))
    print(json.dumps(meta["held_out"]), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Train the learned (normalised / offset) Min-Sum decoder on the GPU and
compare it with plain Min-Sum at equal frame error rate.

    python -m paper_2507_10424_amd.train_nms --steps 2000 --out weights.npz

Recipe: the (3,6)-regular n=1024 code (seed 2; `--code qc64800` takes the
irregular QC code n = 64800 of the same package instead), T = 10 unrolled iterations,
per-iteration per-check-degree scale and offset initialised to 1 and 0,
4096 fresh all-zero frames per step with Eb/N0 drawn per frame uniformly
from [1, 3] dB, checkpoints every 2 iterations, Adam (lr 1e-2).  Evaluation:
fresh frames at 2 dB decoded by plain Min-Sum (at most 50 iterations) and by
the learned decoder (at most T iterations), both with per-frame early exit,
until plain Min-Sum has made at least `--min-errors` frame errors; FER with
Wilson 95% intervals, mean iterations and decoded Gbit/s of each, at every
`--eval-ebn0` point.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def evaluate(g, alpha, beta, T, ebn0, L_plain=50, batch=65536, min_errors=100, max_frames=2_000_000, seed=5150,
             log=None):
    """FER / BER / iterations / throughput of plain (L_plain) and learned (T)
    decoding on the same fresh frames at one Eb/N0."""
    from . import ldpc
    from .nms import frame_errors
    dev = g.device
    rate = 1.0 - g.m / g.n
    stats = {k: dict(fe=0, be=0, it=0.0, ms=0.0) for k in ("plain", "learned")}
    frames = 0
    b = 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while frames < max_frames and (stats["plain"]["fe"] < min_errors or frames == 0):
        llr = ldpc.awgn_llr(batch, g.n, rate, ebn0, seed * 7919 + b, dev)
        b += 1
        for name, args in (("plain", (L_plain, None, None)), ("learned", (T, alpha, beta))):
            if b == 1:  # untimed first call: kernel loading and workspace allocation
                frame_errors(g, llr, *args)
            torch.cuda.synchronize()
            ev0.record()
            fe, be, it, _, _ = frame_errors(g, llr, *args)
            ev1.record()
            torch.cuda.synchronize()
            st = stats[name]
            st["fe"] += fe
            st["be"] += be
            st["it"] += it * batch
            st["ms"] += ev0.elapsed_time(ev1)
        frames += batch
        if log:
            log(f"[eval] {frames} frames: plain {stats['plain']['fe']} frame errors, "
                f"learned {stats['learned']['fe']}")
    out = {"ebn0_db": ebn0, "frames": frames}
    for name, st in stats.items():
        lo, hi = wilson(st["fe"], frames)
        out[name] = {"fer": st["fe"] / frames, "fer_ci95": [lo, hi], "ber": st["be"] / (frames * g.n),
                     "frame_errors": st["fe"], "mean_iters": st["it"] / frames,
                     "max_iters": L_plain if name == "plain" else T,
                     "coded_gbit_s": frames * g.n / (st["ms"] * 1e-3) / 1e9}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--T", type=int, default=10)
    ap.add_argument("--ckpt-every", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--ebn0-lo", type=float, default=1.0)
    ap.add_argument("--ebn0-hi", type=float, default=3.0)
    ap.add_argument("--code", default="regular1024", choices=["regular1024", "qc64800"])
    ap.add_argument("--eval-ebn0", type=float, nargs="+", default=[2.0])
    ap.add_argument("--max-eval-frames", type=int, default=2_000_000)
    ap.add_argument("--eval-batch", type=int, default=65536)
    ap.add_argument("--min-errors", type=int, default=100)
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--out", default=None, help="save alpha, beta and Adam state (.npz)")
    ap.add_argument("--save-weights", default=None,
                    help="save alpha, beta and the training record as JSON (the file bench.py reads)")
    ap.add_argument("--resume", default=None, help="continue from a saved .npz")
    ap.add_argument("--time-budget", type=float, default=None, help="stop training after this many seconds")
    args = ap.parse_args(argv)

    from . import ldpc
    from . import workloads as wl
    from .nms import NMSTrainer

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    if args.code == "qc64800":
        H, code_name = wl.large_qc_code(seed=5), "irregular QC n=64800 m=32400 Z=360"
    else:
        H, code_name = wl.regular_ldpc(1024, 512, 3, 6, seed=2), "(3,6)-regular n=1024 m=512"
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    tr = NMSTrainer(g, T=args.T, batch=args.batch, ckpt_every=args.ckpt_every,
                    ebn0_range=(args.ebn0_lo, args.ebn0_hi), lr=args.lr, seed=args.seed)
    if args.resume:
        d = np.load(args.resume)
        tr.load_state_dict({k: torch.from_numpy(d[k]) for k in ("alpha", "beta", "m1a", "m1b", "m2a", "m2b")}
                           | {"steps": int(d["steps"])})
    torch.cuda.synchronize()
    t0 = time.time()
    tr.train(args.steps, log_every=max(1, args.steps // 20), log=log, time_budget=args.time_budget)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    if args.out:
        sd = tr.state_dict()
        np.savez(args.out, **{k: (v.numpy() if torch.is_tensor(v) else np.asarray(v)) for k, v in sd.items()})
    res = [evaluate(g, tr.alpha, tr.beta, args.T, eb, batch=args.eval_batch, min_errors=args.min_errors,
                    max_frames=args.max_eval_frames, log=log) for eb in args.eval_ebn0]
    hist = torch.stack(tr.history).cpu().numpy() if tr.history else np.zeros(1)
    line = {"metric": "neural vs plain Min-Sum at equal FER", "code": code_name,
            "T": args.T, "train_steps": tr.steps, "train_batch": args.batch, "train_seconds": round(train_s, 2),
            "loss_first": float(hist[: min(10, hist.size)].mean()), "loss_last": float(hist[-10:].mean()),
            "alpha": tr.alpha.cpu().numpy().ravel().round(4).tolist(),
            "beta": tr.beta.cpu().numpy().ravel().round(4).tolist(), "eval": res}
    if args.save_weights:
        rec = {"code": args.code, "T": args.T, "alpha": tr.alpha.cpu().numpy().tolist(),
               "beta": tr.beta.cpu().numpy().tolist(), "check_degrees": list(g.check_degrees),
               "train": {k: line[k] for k in ("train_steps", "train_batch", "loss_first", "loss_last")}
               | {"ebn0_range": [args.ebn0_lo, args.ebn0_hi], "lr": args.lr, "ckpt_every": args.ckpt_every,
                  "seed": args.seed},
               "eval": res}
        with open(args.save_weights, "w") as f:
            json.dump(rec, f, indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

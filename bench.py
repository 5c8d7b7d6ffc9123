#!/usr/bin/env python
"""Throughput of batched Min-Sum LDPC decoding on one MI355X.

Workload (default): the (3,6)-regular code n = 1024, m = 512 (seeded
edge-socket construction), 65,536 random codewords per Eb/N0 point, BPSK over
AWGN at Eb/N0 = 1.0, 1.5, ..., 4.0 dB (7 points), at most 50 iterations with
per-frame syndrome exit.  One step decodes all 7 batches (458,752 frames);
inputs are generated on the GPU and resident in HBM before timing starts.

Prints one JSON line: coded Gbit/s (value), edge-messages/s, the roofline of
the dominant kernel (algorithmic bytes over its event-timed duration), and the
CPU oracle timed on a bounded sample of the same frames.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 32-bit VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


# HBM bytes per launch of the dominant kernel, measured with rocprofv3
# FETCH_SIZE and WRITE_SIZE (each in a run of its own, scaled by a plain copy:
# FETCH x 2.000, WRITE x 1.000), averaged over the launches of one step.  Each
# entry holds the hash of the kernel source it was taken with and, for the
# streaming kernels, the launch choices that fix how many frames one launch
# covers (path, non-temporal messages, chunk); once the source changes, or
# the run uses other choices, the figure no longer applies and `traffic` is
# reported as null.  Summaries: profiles/hbm_bytes_qc64800_regular1024.md.
MEASURED_TRAFFIC = {
    ("regular1024", "onchip"): {"bytes": 609770803, "source": "onchip_kernel.h", "sha256_16": "3d2318242d8c9707"},
    ("qc64800", "check"): {"bytes": 296898742, "source": "decode_stream.hip", "sha256_16": "c2cbb7afe5374b91",
                           "tuning": {"path": 2, "stream_nt": -1, "stream_chunk": -1}},
    ("qc64800", "bit"): {"bytes": 178185898, "source": "decode_stream.hip", "sha256_16": "c2cbb7afe5374b91",
                         "tuning": {"path": 2, "stream_nt": -1, "stream_chunk": -1}},
}


def measured_traffic(config: str, kernel: str, tuning=None):
    import hashlib
    rec = MEASURED_TRAFFIC.get((config, kernel))
    if rec is None:
        return None
    if "tuning" in rec and (tuning is None or any(tuning.get(k) != v for k, v in rec["tuning"].items())):
        return None
    path = os.path.join(ROOT, "paper_2507_10424_amd", "csrc", rec["source"])
    try:
        with open(path, "rb") as f:
            cur = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    return rec["bytes"] if cur == rec["sha256_16"] else None


# The paper's only throughput-like figure, for context (not a target, and not
# comparable: another code, another GPU, a dense formulation in Numba-CUDA,
# termination tested every 6 iterations): its profiled run decodes 4 SNR points
# x 50 frames of the CCSDS n = 8176 code in 48.31 s on an A100 node (Sec. IV,
# kernel-profile table), i.e. 200 x 8176 bits / 48.31 s.
PAPER_CONTEXT = {"value": round(200 * 8176 / 48.31 / 1e9, 9), "unit": "Gbit/s",
                 "hardware": "NVIDIA A100 (node of four), Numba-CUDA kernels on dense m x n matrices",
                 "workload": "CCSDS QC code n = 8176, 50 frames at each of 4 SNR points, up to 60 iterations, "
                             "codeword test every 6 iterations",
                 "derivation": "200 frames x 8176 bits / 48.31 s total run time (profiled run)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def min_pair_ops(d: int) -> int:
    """Instructions for the two smallest of d magnitudes with three-input
    min / median forms: the first group of three takes 2 (min3, med3), each
    further group of three 5 (min3, med3 of the group; min, max, min3 to join),
    each leftover value 2 (min, med3)."""
    if d <= 1:
        return 0
    if d == 2:
        return 2
    groups, rest = divmod(d, 3)
    return 2 + 5 * (groups - 1) + 2 * rest


def alu_ops_per_frame_iter(H) -> int:
    """Lane-operations one Min-Sum iteration of one frame needs on gfx950.

    Per check row of degree d >= 2: d subtractions x = s - eta; the min pair
    of |x| (|x| is a free source modifier); ceil((d - 1) / 2) three-input XORs
    for the sign parity and as many for the syndrome of the previous decision;
    two to fold min0, min1 and the parity sign into one word K; per edge a
    clamp of x to [-min1, min1] and one integer subtraction from K (2 d).  Per
    bit of degree dv: dv additions (dv - 1 messages and r).  Everything else a
    kernel issues (addresses, loop control, refills, reductions, LDS waits) is
    overhead against this count."""
    H = np.asarray(H)
    dr = H.sum(axis=1).astype(np.int64)
    dc = H.sum(axis=0).astype(np.int64)
    ops = 0
    for d, cnt in zip(*np.unique(dr[dr >= 2], return_counts=True)):
        d = int(d)
        ops += int(cnt) * (d + min_pair_ops(d) + 2 * ((d - 1 + 1) // 2) + 2 + 2 * d)
    ops += int(dc.sum())
    return ops


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="regular1024", choices=["regular1024", "qc64800", "regular96", "multi8"])
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--tuning", default=None,
                    help="set the tuning record instead of autotuning: path,variant,wg_per_cu,stream_waves,"
                         "waves_per_simd[,stream_nt[,stream_chunk]] (as printed by a tuned run)")
    ap.add_argument("--path", default="auto", choices=["auto", "stream", "onchip"])
    ap.add_argument("--streams", type=int, default=0,
                    help="HIP streams the Eb/N0 batches are issued on (0: 3 on the on-chip path, else 1)")
    ap.add_argument("--check-period", type=int, default=1,
                    help="codeword test after every k-th iteration (the paper's GPU runs use 6)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nms", action="store_true", help="skip the learned-decoder comparison")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense (Algorithm 2) ablation")
    ap.add_argument("--no-stream-alt", action="store_true",
                    help="skip the streaming-path measurement of the n = 1024 workload")
    ap.add_argument("--no-c4", action="store_true", help="skip the n = 64800 block of the default line")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-code block of the default line")
    ap.add_argument("--no-c0", action="store_true", help="skip the n = 96 block of the default line")
    ap.add_argument("--no-host-io", action="store_true",
                    help="skip the decode from and to pinned host memory (PCIe-inclusive rate)")
    ap.add_argument("--profile-only", action="store_true", help="warmup + timed steps, no extras (for rocprofv3)")
    ap.add_argument("--multi-tuning", default=None,
                    help="multi8: per code variant,waves_per_simd,wg_per_cu of the on-chip path, codes separated "
                         "by ';' (as printed by a tuned run), instead of autotuning each code")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB three times (calibrates the HBM byte counters of a profiler)")
    return ap.parse_args()


def workload(name):
    from paper_2507_10424_amd import workloads as wl
    if name == "regular1024":
        H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
        return dict(name="(3,6)-regular n=1024 m=512, 65536 random codewords x 7 Eb/N0 points 1.0..4.0 dB, "
                         "L=50, early exit", H=H, batch=65536, ebn0=[1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0],
                    L=50, rate=0.5, random_cw=True, seed_cw=200, seed_noise=300, nms_points=[1, 2, 3],
                    dense_frames=1024)
    if name == "qc64800":
        H = wl.large_qc_code(seed=5)
        return dict(name="irregular QC n=64800 m=32400 Z=360, 4096 all-zero frames x Eb/N0 1.0..1.6 dB, L=50, "
                         "early exit", H=H, batch=4096, ebn0=[1.0, 1.2, 1.4, 1.6], L=50, rate=0.5,
                    random_cw=False, seed_cw=0, seed_noise=500)
    if name == "multi8":
        fam = wl.qc_multi_code_family(seed=7)
        frames = sum(c["batch"] for c in fam)
        return dict(name="8 irregular QC codes n in {576,1152,1728,2304}, rates 1/2..5/6, Z in {24,48,72,96}, "
                         f"batches 512..16384 ({frames} frames), all-zero codewords at 2 dB, L=50, one call",
                    family=fam, ebn0=[2.0], L=50, seed_noise=700)
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    return dict(name="(3,6)-regular n=96 m=48, 1000 all-zero frames at 2 dB, L=20", H=H, batch=1000, ebn0=[2.0],
                L=20, rate=0.5, random_cw=False, seed_cw=0, seed_noise=100)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the decoder shards frames across GPUs "
              "by running one independent process per GPU, which this benchmark does not launch", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_launch": x.numel() * 4, "launches": 3}), flush=True)
        return
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = ldpc.load_library()
    import ctypes
    lib.ldpc_timing_enable.argtypes = [ctypes.c_int]
    lib.ldpc_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]

    W = workload(args.config)
    if args.config == "multi8":
        return bench_multi(args, W, dev, lib)
    H = W["H"]
    m, n = H.shape
    B, L = W["batch"], W["L"]
    flags = {"auto": 0, "stream": ldpc.LDPC_FORCE_STREAM, "onchip": ldpc.LDPC_FORCE_ONCHIP}[args.path]
    if args.check_period != 1:
        flags |= ldpc.check_period(args.check_period)
    log(f"[bench] workload: {W['name']}")
    t0 = time.time()
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    E = g.E
    enc = wl.gf2_encoder(H) if W["random_cw"] else None
    llrs, cws = [], []
    for p, eb in enumerate(W["ebn0"]):
        if enc is not None:
            cw = enc.random_codewords_torch(B, W["seed_cw"] + p, dev)
        else:
            cw = None
        llrs.append(wl.bpsk_awgn_llr_torch(cw, eb, W["rate"], W["seed_noise"] + p, dev, n=n, batch=B))
        cws.append(cw)
    torch.cuda.synchronize()
    log(f"[bench] inputs ready on the GPU in {time.time() - t0:.1f} s ({len(llrs)} x {B} x {n})")

    tuning = None
    if args.tuning:
        vals = [int(t) for t in args.tuning.split(",")]
        ldpc.set_tuning(g, *vals)
        tuning = ldpc.get_tuning(g)
        log(f"[bench] tuning set: {tuning}")
    elif not args.no_autotune and args.path == "auto":
        ta = time.time()
        tuning = ldpc.autotune(g, min(B, 65536), L, 2.0 if args.config != "qc64800" else 1.2)
        log(f"[bench] autotuned in {time.time() - ta:.1f} s: {tuning}")
    ws = torch.empty(max(1, ldpc.workspace_bytes(g, B, flags)), dtype=torch.uint8, device=dev)
    outs = [ldpc._outputs(B, n, dev, True) for _ in llrs]
    # The Eb/N0 batches are independent decodes.  On the on-chip path they are
    # issued round-robin on a few HIP streams (default priority), each with its
    # own workspace, so that one launch's last frames overlap the next launch's
    # first ones; the streaming path keeps one stream (its chunks are sized to
    # the Infinity Cache, which concurrent decodes would share).
    if args.path != "auto":
        onchip = args.path == "onchip"
    else:
        onchip = tuning["path"] == 1 if tuning else args.config != "qc64800"
    nstreams = args.streams if args.streams else (min(3, len(llrs)) if onchip else 1)
    side = [torch.cuda.Stream(device=dev) for _ in range(nstreams)] if nstreams > 1 else []
    side_ws = [ws] + [torch.empty_like(ws) for _ in range(nstreams - 1)]
    log(f"[bench] {nstreams} stream(s)")

    def step_on(k):
        if k <= 1:
            for x, o in zip(llrs, outs):
                ldpc.minsum_decode(g, x, L, flags=flags, workspace=ws, out=o)
            return
        cur = torch.cuda.current_stream()
        for st in side:
            st.wait_stream(cur)
        for i, (x, o) in enumerate(zip(llrs, outs)):
            with torch.cuda.stream(side[i % k]):
                ldpc.minsum_decode(g, x, L, flags=flags, workspace=side_ws[i % k], out=o)
        for st in side:
            cur.wait_stream(st)

    def step():
        step_on(nstreams)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    frames_step = B * len(llrs)
    gbits = frames_step * n / (ms_step * 1e-3) / 1e9
    log(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step, {gbits:.2f} coded Gbit/s")
    if args.profile_only:
        print(json.dumps({"ms_per_step": ms_step, "value": gbits}))
        return

    # decoding statistics of the last step
    iters_all = [o[2].to(torch.int64) for o in outs]
    tot_iters = int(sum(int(i.sum()) for i in iters_all))
    per_point = []
    for p, (eb, o) in enumerate(zip(W["ebn0"], outs)):
        bits, _, it, ok = o
        ref = cws[p] if cws[p] is not None else torch.zeros_like(bits)
        err = (bits != ref)
        fe = int(err.any(dim=1).sum())
        per_point.append(dict(ebn0_db=eb, mean_iters=round(float(it.float().mean()), 3), fer=fe / B,
                              ber=float(err.sum()) / (B * n), converged=float(ok.float().mean())))
    edge_msgs = 2.0 * E * tot_iters / (ms_step * 1e-3)
    k_info = (n - wl.gf2_encoder(H).rank) if W["random_cw"] else None

    # per-kernel durations from HIP events on the decode stream (one more
    # step, on one stream so that no two decodes share the GPU), after an
    # untimed step: the statistics above leave the GPU idle long enough
    # (about 0.15 s) for its clocks to drop, and the first launches after
    # that run up to 10% slower
    step_on(1)
    torch.cuda.synchronize()
    lib.ldpc_timing_enable(1)
    step_on(1)
    torch.cuda.synchronize()
    ktimes = {}
    for kid, kname in [(0, "check"), (1, "bit"), (2, "onchip")]:
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        lib.ldpc_timing_read(kid, ctypes.byref(ms), ctypes.byref(cnt))
        if cnt.value:
            ktimes[kname] = (ms.value, cnt.value)
    lib.ldpc_timing_enable(0)
    dom = max(ktimes, key=lambda k: ktimes[k][0])
    dom_ms, dom_launches = ktimes[dom]
    # Algorithmic work of that kernel over the step.  Streaming kernels are
    # HBM-bound: per frame-iteration the check kernel moves 8E + 4n bytes
    # (4E + 4n in iteration 1, which reads no messages) and the bit kernel
    # 4E + 8n.  The on-chip kernel keeps the state in LDS and moves only frame
    # I/O through HBM (4n in, 5n + 5 out); it is bound by VALU issue: the
    # lane-operations of alu_ops_per_frame_iter against 256 CUs x 64 lanes x
    # 2.4 GHz.
    its = torch.cat(iters_all).to(torch.float64)
    if dom == "onchip":
        ops_fi = alu_ops_per_frame_iter(H)
        ops = float(ops_fi * its.sum())
        achieved = ops / (dom_ms * 1e-3) / 1e12
        peak = VALU_PEAK_TOPS
        io = float(frames_step * (9 * n + 5))
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "Tops/s",
                    "frac": round(achieved / peak, 4), "traffic": measured_traffic(args.config, dom, tuning), "kernel": dom,
                    "lane_ops_per_frame_iter": ops_fi,
                    "kernel_ms_per_launch": round(dom_ms / dom_launches, 4), "launches_per_step": dom_launches,
                    "kernel_timing": "HIP events on the launch stream, one more step issued on one stream so that "
                                     "no two decodes overlap",
                    "frac_timed_step": round(ops / (ms_step * 1e-3) / 1e12 / peak, 4),
                    "frac_timed_step_note": f"the same lane-operations over the timed step ({ms_step:.3f} ms on "
                                            f"{nstreams} streams, whose launches overlap)",
                    "hbm_io_gb_s": round(io / (dom_ms * 1e-3) / 1e9, 1)}
    else:
        if dom == "check":
            algo = float(((its >= 1).double() * (4 * E + 4 * n) + (its - 1).clamp(min=0) * (8 * E + 4 * n)).sum())
        else:
            algo = float((its * (4 * E + 8 * n)).sum())
        achieved = algo / (dom_ms * 1e-3) / 1e9
        traffic = measured_traffic(args.config, dom, tuning)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_over_algorithmic": (round(traffic / (algo / dom_launches), 3) if traffic else None),
                    "kernel": dom,
                    "kernel_ms_per_launch": round(dom_ms / dom_launches, 4), "launches_per_step": dom_launches}

    # the same fraction per Eb/N0 point (one more decode of each batch, alone
    # on one stream): the per-frame cost of a refill weighs more where frames
    # stop after a few iterations
    for p, (x, o) in enumerate(zip(llrs, outs)):
        lib.ldpc_timing_enable(1)
        ldpc.minsum_decode(g, x, L, flags=flags, workspace=ws, out=o)
        torch.cuda.synchronize()
        kt = {}
        for kid, kname in [(0, "check"), (1, "bit"), (2, "onchip")]:
            ms_k, cnt = ctypes.c_double(), ctypes.c_int64()
            lib.ldpc_timing_read(kid, ctypes.byref(ms_k), ctypes.byref(cnt))
            kt[kname] = ms_k.value
        lib.ldpc_timing_enable(0)
        pits = o[2].to(torch.float64)
        if dom == "onchip":
            fr = alu_ops_per_frame_iter(H) * float(pits.sum()) / (kt["onchip"] * 1e-3) / 1e12 / VALU_PEAK_TOPS
            per_point[p]["kernel_ms"] = round(kt["onchip"], 4)
        else:
            pb = float((pits * (12 * E + 12 * n)).sum() - (pits >= 1).double().sum() * 4 * E)
            fr = pb / ((kt["check"] + kt["bit"]) * 1e-3) / 1e9 / HBM_PEAK_GBS
            per_point[p]["kernel_ms"] = round(kt["check"] + kt["bit"], 4)
        per_point[p]["roofline_frac"] = round(fr, 4)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the same frames: the first `per` frames of every Eb/N0
        # batch, all threads of this process's CPU share, then one thread
        samples = [x for x in llrs]
        cpu = cpu_oracle_baseline(H, samples, L, args.cpu_seconds, args.check_period, E)
        gpu_sample = [tuple(t[: cpu["frames_per_batch"]] for t in o) for o in outs]
        cpu["gpu_mismatches_on_sample"] = parity_counts(gpu_sample, cpu.pop("_ref"))

    # A streaming decode in chunks keeps each chunk's state in the Infinity
    # Cache; the same step decoding the whole batch at once (every launch
    # streams all frames' state through HBM) is timed beside it.
    whole = None
    if tuning is not None and tuning.get("path") == 2 and tuning.get("stream_chunk") != 0:
        ref_out = [(o[0].clone(), o[2].clone()) for o in outs]
        ldpc.set_tuning(g, 2, stream_waves=tuning["stream_waves"], stream_nt=-1, stream_chunk=0)
        step()
        torch.cuda.synchronize()
        ev0.record()
        step()
        ev1.record()
        torch.cuda.synchronize()
        wms = ev0.elapsed_time(ev1)
        lib.ldpc_timing_enable(1)
        step()
        torch.cuda.synchronize()
        wk = {}
        for kid, kname in [(0, "check"), (1, "bit")]:
            ms_k, cnt = ctypes.c_double(), ctypes.c_int64()
            lib.ldpc_timing_read(kid, ctypes.byref(ms_k), ctypes.byref(cnt))
            wk[kname] = (ms_k.value, cnt.value)
        lib.ldpc_timing_enable(0)
        wits = torch.cat([o[2].to(torch.int64) for o in outs]).to(torch.float64)
        walgo = float(((wits >= 1).double() * (4 * E + 4 * n) + (wits - 1).clamp(min=0) * (8 * E + 4 * n)).sum())
        whole = {"stream_chunk": 0, "coded_gbit_s": round(frames_step * n / (wms * 1e-3) / 1e9, 3),
                 "ms_per_step": round(wms, 3),
                 "check_kernel_ms_per_launch": round(wk["check"][0] / max(wk["check"][1], 1), 4),
                 "check_hbm_frac": round(walgo / (wk["check"][0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "outputs_equal_chunked": all(torch.equal(a[0], o[0]) and torch.equal(a[1], o[2])
                                              for a, o in zip(ref_out, outs))}
        del ref_out
        ldpc.set_tuning(g, 2, variant=tuning["variant"], wg_per_cu=tuning["wg_per_cu"],
                        stream_waves=tuning["stream_waves"], waves_per_simd=tuning["waves_per_simd"],
                        stream_nt=tuning["stream_nt"], stream_chunk=tuning["stream_chunk"])
        log(f"[bench] whole batch per launch (no chunks): {whole['coded_gbit_s']} Gbit/s, "
            f"check HBM frac {whole['check_hbm_frac']}")

    # The same workload on the HBM-resident streaming path (one timed step),
    # for its share of HBM bandwidth on this code.
    stream_alt = None
    if args.config == "regular1024" and args.path == "auto" and not args.no_stream_alt:
        sflags = flags | ldpc.LDPC_FORCE_STREAM
        sws = torch.empty(max(1, ldpc.workspace_bytes(g, B, sflags)), dtype=torch.uint8, device=dev)
        souts = [ldpc._outputs(B, n, dev, True) for _ in llrs]

        def sstep():
            for x, o in zip(llrs, souts):
                ldpc.minsum_decode(g, x, L, flags=sflags, workspace=sws, out=o)

        sstep()
        torch.cuda.synchronize()
        ev0.record()
        sstep()
        ev1.record()
        torch.cuda.synchronize()
        sms = ev0.elapsed_time(ev1)
        # kernel durations from one more step with per-dispatch timing
        lib.ldpc_timing_enable(1)
        sstep()
        torch.cuda.synchronize()
        st_k = {}
        for kid, kname in [(0, "check"), (1, "bit")]:
            ms_k, cnt = ctypes.c_double(), ctypes.c_int64()
            lib.ldpc_timing_read(kid, ctypes.byref(ms_k), ctypes.byref(cnt))
            st_k[kname] = (ms_k.value, cnt.value)
        lib.ldpc_timing_enable(0)
        sits = torch.cat([o[2].to(torch.int64) for o in souts]).to(torch.float64)
        sbytes = float((sits * (12 * E + 12 * n)).sum() - (sits >= 1).double().sum() * 4 * E)
        same = all(torch.equal(a[0], b[0]) and torch.equal(a[2], b[2]) for a, b in zip(souts, outs))
        del sws
        stream_alt = {"path": "stream", "coded_gbit_s": round(frames_step * n / (sms * 1e-3) / 1e9, 3),
                      "ms_per_step": round(sms, 3),
                      "hbm": {"achieved": round(sbytes / ((st_k["check"][0] + st_k["bit"][0]) * 1e-3) / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(sbytes / ((st_k["check"][0] + st_k["bit"][0]) * 1e-3) / 1e9
                                            / HBM_PEAK_GBS, 4),
                              "note": "algorithmic bytes 12E + 12n per frame-iteration (4E less in iteration 1) "
                                      "over the summed check and bit kernel time"},
                      "outputs_equal_on_chip_path": bool(same)}
        log(f"[bench] streaming path on the same workload: {stream_alt['coded_gbit_s']} Gbit/s, "
            f"HBM frac {stream_alt['hbm']['frac']}")

    host_io = None
    if args.config == "regular1024" and not args.no_host_io:
        host_io = host_inclusive(args, g, llrs, outs, L, flags, side, side_ws, ws, n)

    nms = dense = None
    try:
        if not args.no_nms:
            nms = nms_vs_plain(args, W, g, llrs, cws, flags, ws)
        if W.get("dense_frames") and not args.no_dense:
            dense = dense_ablation(args, W, g, llrs, flags)
    except ldpc.LdpcError as e:  # report, keep the main result
        log(f"[bench] side measurement failed: {e}")
        nms = nms if nms is not None else {"error": str(e)}

    # The other workloads, untimed by the step above: n = 64800 (HBM-resident
    # streaming path), the eight-code family (one call), n = 96 in full.
    c4 = multi = c0 = None
    if args.config == "regular1024" and args.path == "auto":
        try:
            if not args.no_c4:
                c4 = block_qc64800(args, dev, lib)
            if not args.no_multi:
                multi = multi_measure(args, workload("multi8"), dev, lib, autotune=not args.no_autotune, steps=5,
                                      warmup=1)
            if not args.no_c0:
                c0 = block_regular96(args, dev)
        except ldpc.LdpcError as e:  # report, keep the main result
            log(f"[bench] side workload failed: {e}")

    line = {
        "metric": "coded Gbit/s & edge-msg/s (% HBM BW); neural vs plain Min-Sum at equal FER",
        "value": round(gbits, 3), "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["name"], "n": n, "m": m, "edges": E, "batch": B, "batches_per_step": len(llrs),
                   "ebn0_db": W["ebn0"], "max_iter": L, "path": args.path, "check_period": args.check_period,
                   "tuning": tuning, "streams": nstreams},
        "edge_msg_per_s": edge_msgs, "info_gbit_s": round(gbits * k_info / n, 3) if k_info else None,
        "mean_iters": round(tot_iters / frames_step, 3), "per_point": per_point,
        "roofline": roofline, "cpu_baseline": cpu, "hbm_resident_path": stream_alt, "whole_batch_stream": whole,
        "host_io": host_io, "nms_vs_plain": nms,
        "dense_ablation": dense, "qc64800": c4, "multi_code": multi, "regular96": c0,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


def host_inclusive(args, g, llrs, outs, L, flags, side, side_ws, ws, n):
    """The timed step's decodes with the frames in pinned host memory: per
    batch, the LLRs copied in, the decode, bits, posteriors, iterations and
    flags copied out, batches spread over the step's streams so that copies
    and decodes overlap.  `value` never includes this: the decoder's inputs
    and outputs are device buffers; this is the rate a caller holding the
    frames on the host would see over PCIe."""
    import torch
    from paper_2507_10424_amd import ldpc
    dev = llrs[0].device
    B = llrs[0].shape[0]
    h_llr = [torch.empty(x.shape, dtype=x.dtype, pin_memory=True) for x in llrs]
    for h, x in zip(h_llr, llrs):
        h.copy_(x)
    h_out = [tuple(torch.empty(t.shape, dtype=t.dtype, pin_memory=True) for t in o) for o in outs]
    streams = side if side else [torch.cuda.current_stream()]
    wss = side_ws if side else [ws]
    k = len(streams)
    d_llr = [torch.empty_like(llrs[0]) for _ in range(k)]
    d_out = [ldpc._outputs(B, n, dev, True) for _ in range(k)]

    def run():
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for i in range(len(llrs)):
            j = i % k
            with torch.cuda.stream(streams[j]):
                d_llr[j].copy_(h_llr[i], non_blocking=True)
                ldpc.minsum_decode(g, d_llr[j], L, flags=flags, workspace=wss[j], out=d_out[j])
                for h, d in zip(h_out[i], d_out[j]):
                    h.copy_(d, non_blocking=True)
        for st in streams:
            cur.wait_stream(st)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    same = all(torch.equal(h[0], o[0].cpu()) and torch.equal(h[2], o[2].cpu()) for h, o in zip(h_out, outs))
    moved = sum(x.numel() * 4 for x in llrs) + sum(t.numel() * t.element_size() for o in outs for t in o)
    res = {"coded_gbit_s": round(len(llrs) * B * n / sec / 1e9, 3), "ms_per_step": round(sec * 1e3, 3),
           "pcie_bytes": moved, "pcie_gb_s": round(moved / sec / 1e9, 1), "streams": k,
           "outputs_equal_device_step": bool(same),
           "note": "LLRs from and bits, posteriors, iterations, flags to pinned host memory, host clock; "
                   "copies and decodes of different batches overlap on the streams"}
    log(f"[bench] from and to host memory: {res['coded_gbit_s']} Gbit/s ({res['pcie_gb_s']} GB/s over PCIe)")
    del h_llr, h_out, d_llr, d_out
    return res


def host_cpu_info():
    """CPU model, logical CPUs and the threads this process may use (its
    affinity, capped by the thread share OMP_NUM_THREADS gives one GPU's job
    on a shared host)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    logical = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = logical
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(affinity, share) if share > 0 else affinity
    return {"cpu_model": model, "logical_cpus": logical, "affinity_cpus": affinity,
            "thread_share": share or None, "threads": max(1, threads)}


def parity_counts(gpu, ref):
    """Frames whose GPU outputs differ from the oracle's, per output: bits,
    iteration counts and convergence flags exactly, posteriors beyond
    1e-5 (1 + |oracle|).  gpu: per batch (bits, post, iters, ok) tensors;
    ref: per batch the oracle's numpy tuple on the same frames."""
    c = {"frames": 0, "bits": 0, "iters": 0, "ok": 0, "post": 0}
    for o, (ob, op, oi, oo) in zip(gpu, ref):
        gb, gp, gi, go = (None if t is None else t.cpu().numpy() for t in o)
        c["frames"] += int(ob.shape[0])
        c["bits"] += int(np.any(gb != ob, axis=1).sum())
        c["iters"] += int((gi != oi).sum())
        c["ok"] += int((go != oo).sum())
        if gp is not None:
            bad = np.abs(gp.astype(np.float64) - op) > 1e-5 * (1.0 + np.abs(op))
            c["post"] += int(np.any(bad, axis=1).sum())
    c["total"] = c["bits"] + c["iters"] + c["ok"] + c["post"]
    return c


def cpu_oracle_baseline(H, batches, L, seconds, check_period=1, E=None, alpha=None, beta=None, min_frames=4):
    """The CPU oracle (as it stands) on a bounded sample of the same frames:
    the first `per` frames of every batch, sized to about `seconds` of work on
    all threads of this process's share, timed there and on one thread (a
    smaller sample).  Returns the report and, under "_ref", the oracle's
    outputs on the all-thread sample for the parity check."""
    import oracle
    info = host_cpu_info()
    nthreads = info["threads"]
    m, n = H.shape
    E = int(H.sum()) if E is None else E
    probe = [x[:4].cpu().numpy() for x in batches]

    def run(xs, threads):
        if alpha is None:
            return [oracle.minsum_decode(H, x, L, nthreads=threads, check_period=check_period) for x in xs]
        return [oracle.nms_decode(H, x, L, alpha, beta, nthreads=threads) for x in xs]

    tp = time.time()
    run(probe, 1)
    t_probe = (time.time() - tp) / (4 * len(probe))  # s per frame on one thread
    B = batches[0].shape[0]
    per = max(min_frames, min(B, int(seconds * nthreads / max(t_probe, 1e-6) / len(batches))))
    per = min(per, B)
    sample = [x[:per].cpu().numpy() for x in batches]
    tc = time.time()
    ref = run(sample, nthreads)
    t_all = time.time() - tc
    per1 = max(1, min(per, int(0.3 * seconds / max(t_probe, 1e-6) / len(batches))))
    t1 = time.time()
    ref1 = run([x[:per1] for x in sample], 1)
    t_one = time.time() - t1
    frames_all, frames_one = per * len(sample), per1 * len(sample)
    msgs_all = 2.0 * E * sum(int(r[2].sum()) for r in ref)
    msgs_one = 2.0 * E * sum(int(r[2].sum()) for r in ref1)
    return {"value": round(frames_all * n / t_all / 1e9, 6), "unit": "Gbit/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first {per} frames of each of the {len(sample)} batches ({frames_all} frames, {t_all:.1f} s "
                      f"on {nthreads} threads); single thread: first {per1} of each ({frames_one} frames, "
                      f"{t_one:.1f} s)",
            "all_threads": {"threads": nthreads, "frames": frames_all, "seconds": round(t_all, 3),
                            "frames_per_s": round(frames_all / t_all, 2),
                            "coded_gbit_s": round(frames_all * n / t_all / 1e9, 6),
                            "edge_msg_per_s": round(msgs_all / t_all, 1)},
            "single_thread": {"threads": 1, "frames": frames_one, "seconds": round(t_one, 3),
                              "frames_per_s": round(frames_one / t_one, 2),
                              "coded_gbit_s": round(frames_one * n / t_one / 1e9, 6),
                              "edge_msg_per_s": round(msgs_one / t_one, 1)},
            "host": info, "frames_per_batch": per, "_ref": ref}


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return [0.0, 1.0]
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * (p * (1 - p) / n + z * z / (4 * n * n)) ** 0.5 / d
    return [round(max(0.0, c - h), 6), round(min(1.0, c + h), 6)]


def nms_vs_plain(args, W, g, llrs, cws, flags, ws, path=None):
    """The learned decoder (T iterations, weights trained by train_nms.py and
    stored in the package) against plain Min-Sum (L iterations) on the same
    frames: FER with Wilson 95% intervals and coded Gbit/s of each."""
    import torch
    from paper_2507_10424_amd import ldpc
    path = path or os.path.join(ROOT, "paper_2507_10424_amd", "weights", f"nms_{args.config}.json")
    if not os.path.exists(path):
        log(f"[bench] no learned weights at {path}; skipping the learned decoder")
        return None
    with open(path) as f:
        rec = json.load(f)
    dev = llrs[0].device
    alpha = torch.tensor(rec["alpha"], dtype=torch.float32, device=dev)
    beta = torch.tensor(rec["beta"], dtype=torch.float32, device=dev)
    T, L = int(rec["T"]), W["L"]
    points = W.get("nms_points", list(range(len(llrs))))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = []
    for p in points:
        x, cw = llrs[p], cws[p]
        B, n = x.shape
        row = {"ebn0_db": W["ebn0"][p], "frames": B}
        for name, fn in (("plain", lambda: ldpc.minsum_decode(g, x, L, flags=flags, want_post=False, workspace=ws)),
                         ("learned", lambda: ldpc.nms_decode(g, x, T, alpha, beta, flags=flags, want_post=False,
                                                             workspace=ws))):
            fn()  # warm-up
            torch.cuda.synchronize()
            ev0.record()
            out = fn()
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            ref = cw if cw is not None else torch.zeros_like(out[0])
            fe = int((out[0] != ref).any(dim=1).sum())
            row[name] = {"max_iter": L if name == "plain" else T, "fer": fe / B, "fer_ci95": wilson(fe, B),
                         "mean_iters": round(float(out[2].float().mean()), 3),
                         "coded_gbit_s": round(B * n / (ms * 1e-3) / 1e9, 3)}
        lo_p, hi_p = row["plain"]["fer_ci95"]
        lo_l, hi_l = row["learned"]["fer_ci95"]
        row["fer_intervals_overlap"] = bool(lo_l <= hi_p and lo_p <= hi_l)
        row["speedup"] = round(row["learned"]["coded_gbit_s"] / row["plain"]["coded_gbit_s"], 3)
        res.append(row)
    return {"weights": os.path.relpath(path, ROOT), "T": T, "train": rec.get("train"), "points": res}


def stream_kernel_ms(lib, run):
    """Summed event-timed milliseconds and launches of the streaming check and
    bit kernels over one call of run()."""
    import ctypes
    import torch
    lib.ldpc_timing_enable(1)
    run()
    torch.cuda.synchronize()
    res = {}
    for kid, kname in [(0, "check"), (1, "bit")]:
        ms_k, cnt = ctypes.c_double(), ctypes.c_int64()
        lib.ldpc_timing_read(kid, ctypes.byref(ms_k), ctypes.byref(cnt))
        res[kname] = (ms_k.value, cnt.value)
    lib.ldpc_timing_enable(0)
    return res


def stream_algo_bytes(its, E, n):
    """Algorithmic HBM bytes of the streaming kernels for per-frame iteration
    counts `its`: check 8E + 4n per frame-iteration (4E + 4n in iteration 1,
    which reads no messages), bit 4E + 8n."""
    check = float(((its >= 1).double() * (4 * E + 4 * n) + (its - 1).clamp(min=0) * (8 * E + 4 * n)).sum())
    bit = float((its * (4 * E + 8 * n)).sum())
    return check, bit


def block_qc64800(args, dev, lib):
    """The irregular QC n = 64800 workload at one Eb/N0 point (4,096 all-zero
    frames at 1.4 dB, L = 50) on the streaming path: chunks kept in the
    Infinity Cache (the size rule) and the whole batch in every launch
    (every byte streamed from HBM), with the full-iteration HBM fraction of
    each; the oracle on the first frames (all outputs compared) and timed on
    the host; the learned decoder against plain Min-Sum on the same frames."""
    import torch
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd import workloads as wl
    W = workload("qc64800")
    H = W["H"]
    m, n = H.shape
    B, L, eb = W["batch"], W["L"], 1.4
    p = W["ebn0"].index(eb)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    E = g.E
    llr = wl.bpsk_awgn_llr_torch(None, eb, W["rate"], W["seed_noise"] + p, dev, n=n, batch=B)
    ws = torch.empty(max(1, ldpc.workspace_bytes(g, B, ldpc.LDPC_FORCE_STREAM)), dtype=torch.uint8, device=dev)
    res = {"workload": f"irregular QC n=64800 m=32400 Z=360, {B} all-zero frames at {eb} dB, L={L}, early exit",
           "n": n, "m": m, "edges": E, "batch": B, "ebn0_db": eb, "max_iter": L}
    outs = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, chunk in (("chunked", -1), ("whole_batch", 0)):
        ldpc.set_tuning(g, 2, stream_waves=4, stream_nt=-1, stream_chunk=chunk)
        o = ldpc._outputs(B, n, dev, True)

        def run():
            ldpc.minsum_decode(g, llr, L, workspace=ws, out=o)

        run()
        torch.cuda.synchronize()
        reps = 2
        ev0.record()
        for _ in range(reps):
            run()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        kt = stream_kernel_ms(lib, run)
        its = o[2].to(torch.float64)
        a_chk, a_bit = stream_algo_bytes(its, E, n)
        t_chk, t_bit = kt["check"][0], kt["bit"][0]
        res[name] = {"stream_chunk": chunk, "tiles_per_chunk": "by size (200 MiB)" if chunk < 0 else "all",
                     "ms_per_decode": round(ms, 3), "coded_gbit_s": round(B * n / (ms * 1e-3) / 1e9, 3),
                     "edge_msg_per_s": round(2.0 * E * float(its.sum()) / (ms * 1e-3), 1),
                     "check_ms_per_launch": round(t_chk / max(kt["check"][1], 1), 4),
                     "bit_ms_per_launch": round(t_bit / max(kt["bit"][1], 1), 4),
                     "launches": kt["check"][1] + kt["bit"][1],
                     "hbm_frac_check": round(a_chk / (t_chk * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "hbm_frac_bit": round(a_bit / (t_bit * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "hbm_frac_full_iteration": round((a_chk + a_bit) / ((t_chk + t_bit) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                      4)}
        outs[name] = o
        log(f"[bench] n=64800 {name}: {res[name]['coded_gbit_s']} Gbit/s, HBM frac (check + bit) "
            f"{res[name]['hbm_frac_full_iteration']}")
    res["note"] = ("HBM fractions: algorithmic bytes (12E + 12n per frame-iteration, 4E less in iteration 1) over "
                   "the event-timed kernel time; with chunks most launches after a chunk's first are served by the "
                   "Infinity Cache, so only the whole-batch figures are HBM-bound")
    a, b = outs["chunked"], outs["whole_batch"]
    res["outputs_equal_chunked_whole"] = bool(all(torch.equal(x, y) for x, y in zip(a, b)))
    its = a[2].to(torch.float64)
    err = a[0] != 0
    fe = int(err.any(dim=1).sum())
    res["plain"] = {"fer": fe / B, "fer_ci95": wilson(fe, B), "ber": float(err.sum()) / (B * n),
                    "mean_iters": round(float(its.mean()), 3)}
    ldpc.set_tuning(g, None)
    if not args.no_cpu_baseline:
        cpu = cpu_oracle_baseline(H, [llr], L, args.cpu_seconds / 2, 1, E, min_frames=256)
        gs = [tuple(t[: cpu["frames_per_batch"]] for t in a)]
        cpu["gpu_mismatches_on_sample"] = parity_counts(gs, cpu.pop("_ref"))
        res["cpu_baseline"] = cpu
    if not args.no_nms:
        learned = []
        for wname in ("nms_qc64800_T10.json", "nms_qc64800.json"):
            path = os.path.join(ROOT, "paper_2507_10424_amd", "weights", wname)
            if os.path.exists(path):
                r = nms_vs_plain(args, {"L": L, "ebn0": [eb]}, g, [llr], [None], 0, ws, path=path)
                learned.append(r)
        res["nms_vs_plain"] = learned
    del ws
    return res


def block_regular96(args, dev):
    """The (3,6)-regular n = 96 workload in full: 1000 all-zero frames at
    2 dB, L = 20, decoded on the GPU and by the oracle (every output of every
    frame compared), and the oracle timed on the host."""
    import torch
    from paper_2507_10424_amd import ldpc
    W = workload("regular96")
    H = W["H"]
    m, n = H.shape
    B, L = W["batch"], W["L"]
    from paper_2507_10424_amd import workloads as wl
    llr_np = wl.bpsk_awgn_llr(None, W["ebn0"][0], W["rate"], seed=W["seed_noise"], n=n, batch=B)
    llr = torch.from_numpy(llr_np).to(dev)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    out = ldpc.minsum_decode(g, llr, L)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    out = ldpc.minsum_decode(g, llr, L)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    res = {"workload": W["name"], "frames": B, "gpu_ms": round(ms, 4),
           "gpu_coded_gbit_s": round(B * n / (ms * 1e-3) / 1e9, 4),
           "fer": float((out[0] != 0).any(dim=1).float().mean()),
           "mean_iters": round(float(out[2].float().mean()), 3)}
    if not args.no_cpu_baseline:
        cpu = cpu_oracle_baseline(H, [llr], L, 2.0, 1, g.E, min_frames=B)
        res["gpu_mismatches"] = parity_counts([out], cpu.pop("_ref"))
        res["cpu_baseline"] = cpu
    return res


def dense_ablation(args, W, g, llrs, flags):
    """The paper's dense map-reduce form (Algorithm 2 on m x n matrices) against
    the sparse decoder on the same frames: the first `dense_frames` frames of
    the 2 dB batch.  Both outputs must agree."""
    import torch
    from paper_2507_10424_amd import ldpc
    p = W["ebn0"].index(2.0)
    x = llrs[p][: W["dense_frames"]].contiguous()
    B, n = x.shape
    L = W["L"]
    dflags = flags & ~(ldpc.LDPC_FORCE_STREAM | ldpc.LDPC_FORCE_ONCHIP)
    dws = torch.empty(max(1, ldpc.dense_workspace_bytes(g, B)), dtype=torch.uint8, device=x.device)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"frames": B, "ebn0_db": 2.0}
    outs = {}
    for name, fn in (("dense", lambda: ldpc.minsum_decode_dense(g, x, L, flags=dflags, workspace=dws)),
                     ("sparse", lambda: ldpc.minsum_decode(g, x, L, flags=flags))):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        outs[name] = fn()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        res[name] = {"ms": round(ms, 4), "coded_gbit_s": round(B * n / (ms * 1e-3) / 1e9, 4)}
    its = outs["dense"][2].to(torch.float64)
    # dense message traffic: 12 m n bytes per frame-iteration (4 m n in iteration 1, which reads no eta)
    mn = float(g.m) * float(g.n)
    dbytes = float(((its >= 1).double() * 8 * mn + (its - 1).clamp(min=0) * 12 * mn).sum())
    res["dense"]["message_gb_s"] = round(dbytes / (res["dense"]["ms"] * 1e-3) / 1e9, 1)
    res["outputs_agree"] = bool(all(torch.equal(a, b) for a, b in zip(outs["dense"], outs["sparse"])))
    res["sparse_over_dense"] = round(res["dense"]["ms"] / res["sparse"]["ms"], 1)
    return res


def multi_measure(args, W, dev, lib, autotune=True, steps=None, warmup=None):
    """Eight codes at their configured batches: one ldpc_minsum_decode_multi
    call per step against one ldpc_minsum_decode per code, the same at 1/32
    of the batches, the launches the call makes, the ALU roofline of the call,
    and the oracle on the first frames of every code (all outputs compared)."""
    import torch
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd import workloads as wl
    import ctypes
    fam, L = W["family"], W["L"]
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    graphs, llrs, tunings = [], [], []
    ta = time.time()
    fixed = None
    if getattr(args, "multi_tuning", None):
        fixed = [[int(x) for x in part.split(",")] for part in args.multi_tuning.split(";")]
        if len(fixed) != len(fam) or any(len(f) != 3 for f in fixed):
            raise SystemExit(f"--multi-tuning needs {len(fam)} entries of variant,waves_per_simd,wg_per_cu")
    for k, c in enumerate(fam):
        graphs.append(ldpc.build_graph(torch.from_numpy(c["H"]).to(dev)))
        llrs.append(wl.bpsk_awgn_llr_torch(None, W["ebn0"][0], c["rate"], W["seed_noise"] + k, dev, n=c["n"],
                                           batch=c["batch"]))
        if fixed:
            v, wps, wpc = fixed[k]
            ldpc.set_tuning(graphs[-1], 1, variant=v, waves_per_simd=wps, wg_per_cu=wpc)
            tunings.append(ldpc.get_tuning(graphs[-1]))
        elif autotune:  # each code's own launch choice, as for one code
            tunings.append(ldpc.autotune(graphs[-1], min(c["batch"], 65536), L, W["ebn0"][0]))
    if tunings:
        how = "tunings from --multi-tuning" if fixed else f"autotuned in {time.time() - ta:.1f} s"
        log(f"[bench] multi-code: {how}, variants {[t['variant'] for t in tunings]}")
    jobs = list(zip(graphs, llrs))
    outs = [ldpc._outputs(c["batch"], c["n"], dev, True) for c in fam]
    ws = torch.empty(int(lib.ldpc_multi_workspace_bytes(len(jobs))), dtype=torch.uint8, device=dev)
    frames = sum(c["batch"] for c in fam)
    bits = sum(c["batch"] * c["n"] for c in fam)

    def step_multi():
        ldpc.minsum_decode_multi(jobs, L, workspace=ws, outs=outs)

    def step_each():
        for (g, x), o in zip(jobs, outs):
            ldpc.minsum_decode(g, x, L, workspace=ws, out=o)

    def timed(fn):
        for _ in range(warmup):
            fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    if args.profile_only:  # the one call's warmup and timed steps only
        ms_multi = timed(step_multi)
        log(f"[bench] multi-code: one call {ms_multi:.3f} ms/step")
        return {"profile_only": True, "ms_per_step_one_call": round(ms_multi, 4), "tuning": tunings or None}
    ms_each = timed(step_each)
    ms_multi = timed(step_multi)
    # launches of the one call (every on-chip launch is event-timed)
    lib.ldpc_timing_enable(1)
    step_multi()
    torch.cuda.synchronize()
    kms, kcnt = ctypes.c_double(), ctypes.c_int64()
    lib.ldpc_timing_read(2, ctypes.byref(kms), ctypes.byref(kcnt))
    lib.ldpc_timing_enable(0)
    step_multi()  # outputs of an untimed call for the statistics below
    torch.cuda.synchronize()

    # the same codes with 1/32 of the batches: here one shared persistent
    # launch has to carry the small batches that underfill the GPU one by one
    small_llrs = [x[: max(1, x.shape[0] // 32)].contiguous() for x in llrs]
    small_jobs = list(zip(graphs, small_llrs))
    small_bits = sum(x.shape[0] * x.shape[1] for x in small_llrs)
    ms_small_multi = timed(lambda: ldpc.minsum_decode_multi(small_jobs, L, workspace=ws))
    ms_small_each = timed(lambda: [ldpc.minsum_decode(g, x, L, workspace=ws) for g, x in small_jobs])
    gbits = bits / (ms_multi * 1e-3) / 1e9
    log(f"[bench] multi-code: one call {ms_multi:.3f} ms/step ({gbits:.2f} Gbit/s, {kcnt.value} launches), "
        f"one launch per code {ms_each:.3f} ms/step")
    iters = sum(int(o[2].to(torch.int64).sum()) for o in outs)
    edges_iters = sum(int(o[2].to(torch.int64).sum()) * g.E for o, g in zip(outs, graphs))
    per_code = []
    for c, o in zip(fam, outs):
        fe = int((o[0] != 0).any(dim=1).sum())
        per_code.append(dict(n=c["n"], rate=round(c["rate"], 4), Z=c["Z"], batch=c["batch"], fer=fe / c["batch"],
                             mean_iters=round(float(o[2].float().mean()), 3)))
    ops = float(sum(alu_ops_per_frame_iter(c["H"]) * int(o[2].to(torch.int64).sum()) for c, o in zip(fam, outs)))
    achieved = ops / (ms_multi * 1e-3) / 1e12
    res = {
        "workload": W["name"], "frames": frames, "max_iter": L, "ebn0_db": W["ebn0"],
        "tuning": tunings or None,
        "coded_gbit_s": round(gbits, 3), "ms_per_step_one_call": round(ms_multi, 4),
        "launches_per_call": int(kcnt.value),
        "ms_per_step_one_launch_per_code": round(ms_each, 4),
        "gbit_s_one_launch_per_code": round(bits / (ms_each * 1e-3) / 1e9, 3),
        "edge_msg_per_s": 2.0 * edges_iters / (ms_multi * 1e-3), "mean_iters": round(iters / frames, 3),
        "per_code": per_code,
        "small_batches": {"frames": sum(x.shape[0] for x in small_llrs), "ms_one_call": round(ms_small_multi, 4),
                          "ms_one_launch_per_code": round(ms_small_each, 4),
                          "gbit_s_one_call": round(small_bits / (ms_small_multi * 1e-3) / 1e9, 3),
                          "gbit_s_one_launch_per_code": round(small_bits / (ms_small_each * 1e-3) / 1e9, 3)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                     "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None, "kernel": "onchip (one call)",
                     "note": "algorithmic lane-operations of every frame-iteration over the call's time"},
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = 64
        ref, got = [], []
        tc = time.time()
        for c, x, o in zip(fam, llrs, outs):
            ref.append(oracle.minsum_decode(c["H"], x[:sample].cpu().numpy(), L,
                                            nthreads=host_cpu_info()["threads"]))
            got.append(tuple(t[:sample] for t in o))
        res["oracle_check"] = {"frames_per_code": sample, "seconds": round(time.time() - tc, 2),
                               "gpu_mismatches": parity_counts(got, ref)}
    return res


def bench_multi(args, W, dev, lib):
    """The multi-code workload as the benchmark line of its own."""
    res = multi_measure(args, W, dev, lib, autotune=not args.no_autotune)
    if res.get("profile_only"):
        print(json.dumps(res), flush=True)
        return
    line = {
        "metric": "coded Gbit/s & edge-msg/s (% HBM BW); neural vs plain Min-Sum at equal FER",
        "value": res["coded_gbit_s"], "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step_one_call"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["name"], "frames": res["frames"], "max_iter": W["L"], "ebn0_db": W["ebn0"],
                   "tuning": res["tuning"]},
        "roofline": res["roofline"], "cpu_baseline": None, "multi_code": res,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

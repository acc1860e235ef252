"""Benchmark: extracted output Gbps of the block-wise inner-product extractor
on one MI355X, paper-scale block workload (n = 8192-bit blocks, m = 2048
output bits per block pair, 65536 pairs of i.i.d. Gaussian 8-bit ADC samples
per source, seeds 11 and 12).

One step = one pass of the whole hot path (one ext_extract over all 65536
block pairs, inputs resident in HBM, outputs written to HBM).  Prints one
JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_BITS = 8192
M_BITS = 2048
N_PAIRS = 65536
# 256 CUs x 64 lanes x 2.4 GHz x 32 bit-MACs per v_bitop3_b32 lane-op
PEAK_BITMAC_T = 256 * 64 * 2.4e9 * 32 / 1e12
KERNEL_SOURCE = os.path.join(ROOT, "paper_2402_14607_amd", "csrc", "ext_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ext_ip_kernel_paper_block_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "ext_ip_kernel_paper_block_valu.txt")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def profile_value(path: str, key: str):
    """A key=value figure of a committed rocprofv3 counter summary, if the
    summary was taken on the current kernel source."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(rec[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)."""
    return profile_value(TRAFFIC_FILE, "hbm_bytes_per_launch")


def cpu_baseline(w, target_s: float = 12.0):
    """The oracle, as it stands, on a bounded sample of the same workload,
    one block pair per call spread over the host's cores."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    cores = min(16, len(os.sched_getaffinity(0)))
    t0 = time.time()
    oracle.ext_sampled(w.x, w.y, np.arange(4, dtype=np.uint64), w.n_bits, w.m_bits)
    per_pair = (time.time() - t0) / 4
    count = int(max(cores, min(w.n_pairs, target_s * cores / max(per_pair, 1e-6))))
    stride = max(1, w.n_pairs // count)
    idx = (np.arange(count, dtype=np.uint64) * stride) % w.n_pairs
    chunks = np.array_split(idx, cores)
    log("cpu baseline: oracle on %d pairs over %d threads (~%.1f ms/pair/core)"
        % (count, cores, per_pair * 1e3))
    t0 = time.time()
    with cf.ThreadPoolExecutor(cores) as pool:
        list(pool.map(lambda c: oracle.ext_sampled(w.x, w.y, c, w.n_bits, w.m_bits), chunks))
    dt = time.time() - t0
    return {
        "value": round(count * w.m_bits / dt / 1e9, 6),
        "unit": "Gbps",
        "cores": cores,
        "kind": "oracle",
        "sample": "%d of the %d block pairs (every %d-th), bit-by-bit C oracle, %.1f s"
                  % (count, w.n_pairs, stride, dt),
    }


def batched_leg(dev, stream, steps: int, warmup: int):
    """The batched workload (64 stream pairs, n drawn from 2048..32768, m = n/4,
    4096 pairs each): plain form (one launch per stream) against the batched
    form (one persistent launch, replayed from a captured graph)."""
    import torch

    from paper_2402_14607_amd import binding, inputs

    log("batched leg: generating 64 stream pairs")
    w = inputs.batched()
    items = []
    for s in w.streams:
        out = torch.empty(s.n_pairs * s.m_bits // 8, dtype=torch.uint8, device=dev)
        items.append((s.n_bits, s.m_bits, torch.from_numpy(s.x).to(dev),
                      torch.from_numpy(s.y).to(dev), out, s.n_pairs))
    out_bits = sum(s.n_pairs * s.m_bits for s in w.streams)
    in_bits = sum(2 * s.n_pairs * s.n_bits for s in w.streams)
    bitmacs = sum(s.n_pairs * s.n_bits * s.m_bits for s in w.streams)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    exs = [binding.Extractor(n, m, device_memory=True, stream=stream.cuda_stream)
           for (n, m, _, _, _, _) in items]

    def plain_step():
        for ex, (n, m, x, y, out, pairs) in zip(exs, items):
            ex.extract(x, y, out, pairs)

    ms_plain = timed(plain_step)
    batch = binding.Batch(items, stream=stream.cuda_stream, autotune=True)
    desc = json.loads(batch.describe())
    ms_batch = timed(batch.run)
    log("batched leg: plain %.3f ms/pass, batched %.3f ms/pass" % (ms_plain, ms_batch))
    res = {
        "workload": "64 stream pairs, n uniform on {2048,...,32768} per stream, m=n/4, "
                    "4096 pairs each, iid 8-bit Gaussian ADC samples",
        "plain_ms_per_pass": round(ms_plain, 4),
        "plain_output_gbps": round(out_bits / (ms_plain * 1e-3) / 1e9, 3),
        "batched_ms_per_pass": round(ms_batch, 4),
        "batched_output_gbps": round(out_bits / (ms_batch * 1e-3) / 1e9, 3),
        "batched_input_gbps": round(in_bits / (ms_batch * 1e-3) / 1e9, 3),
        "batched_roofline_frac": round(bitmacs / (ms_batch * 1e-3) / 1e12 / PEAK_BITMAC_T, 4),
        "speedup": round(ms_plain / ms_batch, 3),
        "launches": desc["launches"],
        "graph": desc["graph"],
    }
    batch.close()
    for ex in exs:
        ex.close()
    return res


def paper_point_leg(dev, stream, steps: int, warmup: int):
    """The paper's own parameter point (Sec. 4.2): n_e = 71 elements of F_2^80
    per block, 16-bit Gaussian samples, 262144 block pairs in one launch per
    step; sampled pairs checked against the oracle.  The paper's simulated
    FPGA rate for this shape is 64 Gbps of output (context only)."""
    import numpy as np
    import torch

    import oracle
    from paper_2402_14607_amd import binding, inputs

    log("paper-point leg: generating 262144 pairs of 16-bit samples")
    w = inputs.paper_point()
    n, m, pairs = w.n_bits, w.m_bits, w.n_pairs
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    out = torch.empty(pairs * m // 8, dtype=torch.uint8, device=dev)
    ex = binding.Extractor(n, m, device_memory=True, sample_bits=16, stream=stream.cuda_stream,
                           autotune=True)
    plan = json.loads(ex.describe())
    log("paper-point leg: autotuned plan %s" % json.dumps(plan))
    for _ in range(warmup):
        ex.extract(x, y, out, pairs)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        ex.extract(x, y, out, pairs)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    got = out.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.unique(np.concatenate([[0, pairs - 1], rng.integers(0, pairs, 14)])).astype(np.uint64)
    want = oracle.ext_sampled(w.x, w.y, idx, n, m)
    qb = m // 8
    g = np.concatenate([got[int(i) * qb:(int(i) + 1) * qb] for i in idx])
    parity = "bit-exact on %d sampled pairs" % idx.size if np.array_equal(g, want) else "MISMATCH"
    out_gbps = pairs * m / (ms * 1e-3) / 1e9
    log("paper-point leg: %.4f ms per launch, %.2f Gbps output, %s" % (ms, out_gbps, parity))
    ex.close()
    # the other kernel on the same launch, for comparison
    other = binding.KERNEL_WORD if plan.get("kernel") == "bitslice" else binding.KERNEL_BITSLICE
    ex2 = binding.Extractor(n, m, device_memory=True, sample_bits=16, stream=stream.cuda_stream,
                            autotune=True, kernel=other)
    out2 = torch.empty_like(out)
    ex2.extract(x, y, out2, pairs)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        ex2.extract(x, y, out2, pairs)
    b.record(stream)
    torch.cuda.synchronize()
    ms2 = a.elapsed_time(b) / steps
    same = bool(torch.equal(out, out2))
    other_plan = json.loads(ex2.describe())
    ex2.close()
    log("paper-point leg: %s kernel %.4f ms per launch, same bytes: %s"
        % (other_plan["kernel"], ms2, same))
    return {
        "workload": "paper parameter point: n_e=71 elements of F_2^80 per block (n=5680 bits, "
                    "355 16-bit samples), 262144 block pairs, iid round(N(32768, 682^2)) "
                    "16-bit samples, seeds 31/32",
        "ms_per_launch": round(ms, 5),
        "output_gbps": round(out_gbps, 3),
        "input_gbps": round(2 * pairs * n / (ms * 1e-3) / 1e9, 3),
        "roofline_frac": round(pairs * n * m / (ms * 1e-3) / 1e12 / PEAK_BITMAC_T, 4),
        "parity": parity,
        "kernel_plan": plan,
        "other_kernel": {"kernel": other_plan["kernel"], "ms_per_launch": round(ms2, 5),
                         "output_gbps": round(pairs * m / (ms2 * 1e-3) / 1e9, 3),
                         "same_bytes": same},
        "context_fpga_output_gbps": 64.0,
    }


def growing_leg(dev, stream, steps: int, warmup: int):
    """Algorithm 2 at the paper's rate point: n_e = 71 elements per block,
    q_l = 80 + 16 l (Delta = 1, b = 16), the first 64 blocks (q up to 1088) of
    16-bit Gaussian streams per call; every block checked against the oracle."""
    import numpy as np
    import torch

    import oracle
    from oracle import params as orc_params
    from paper_2402_14607_amd import binding, inputs

    n_e, q1, dsteps, b, k = 71, 80, 1, 16, 64
    sched = orc_params.schedule(q1, dsteps, b, n_e, k)
    n_bytes = (sched[-1][0] + sched[-1][1]) * b // 8
    xh = inputs.gaussian_adc16(n_bytes // 2, 33)
    yh = inputs.gaussian_adc16(n_bytes // 2, 34)
    x = torch.from_numpy(xh).to(dev)
    y = torch.from_numpy(yh).to(dev)
    with binding.Growing(n_e, q1, dsteps, sample_bits=b, stream=stream.cuda_stream) as g:
        kk, nin, nout = g.blocks(n_bytes)
        out = torch.empty(nout, dtype=torch.uint8, device=dev)
        for _ in range(warmup):
            g.extract(x, y, n_bytes, out, nout)
        torch.cuda.synchronize()
        import time

        t0 = time.perf_counter()
        for _ in range(steps):
            g.extract(x, y, n_bytes, out, nout)  # returns after the outputs are written
        ms = (time.perf_counter() - t0) * 1e3 / steps
    got = out.cpu().numpy()
    want = np.concatenate([oracle.ext_blocks(xh[s * 2:(s + z) * 2], yh[s * 2:(s + z) * 2],
                                             q * n_e, q) for s, z, q in sched])
    parity = "bit-exact on all %d blocks" % kk if np.array_equal(got, want) else "MISMATCH"
    bitmacs = sum(n_e * q * q for _, _, q in sched)
    log("growing leg: %.3f ms per call, %s" % (ms, parity))
    return {
        "workload": "Algorithm 2: n_e=71, q_l = 80 + 16 l for the first 64 blocks (q up to 1088), "
                    "16-bit Gaussian samples, seeds 33/34",
        "ms_per_call": round(ms, 4),
        "output_gbps": round(nout * 8 / (ms * 1e-3) / 1e9, 4),
        "input_gbps": round(2 * nin * 8 / (ms * 1e-3) / 1e9, 4),
        "roofline_frac": round(bitmacs / (ms * 1e-3) / 1e12 / PEAK_BITMAC_T, 5),
        "timing": "host wall clock per call (planning, copies of the launch tables, launches, "
                  "wait for the outputs)",
        "parity": parity,
    }


def served_leg(w, duration_s: float, warmup_s: float, modes=("served", "plain",
                                                             "plain_at_1/16_load"),
               wg_per_cu: int = 0, max_inflight: int = 0, split_pairs: int = -1,
               producers: int = 4, timing: int = 0):
    """The served workload: 256 channel pairs with Poisson chunk arrivals of
    1..64 blocks, 64 Gbps aggregate raw input; three quarters i.i.d. Gaussian
    with n from 2048..32768, one quarter AR(1) with n = 65536.  Served form
    (continuous batching) against the plain form (one ext_stream and one
    launch per chunk per channel) on the same arrival trace."""
    import numpy as np

    from paper_2402_14607_amd import binding, inputs

    shapes = inputs.served_channels()
    log("served leg: AR(1) pools")
    ar = inputs.plain_workload(65536, 16384, 8192, 21, 22, kind="ar1")  # 64 MiB per side
    chans = []
    for c, (n, m, kind) in enumerate(shapes):
        nb = n // 8
        if kind == "ar1":
            px, py = ar.x, ar.y
        else:
            px, py = w.x, w.y
        # each channel starts at its own place in the pool (block aligned)
        off = (c * 7919 * nb) % (px.size // 2) // nb * nb
        length = (px.size - off) // nb * nb
        chans.append((n, m, px[off:off + length], py[off:off + length]))
    rate = 64e9 / 8  # bytes per second, X + Y
    out = {"workload": "256 channel pairs, Poisson chunks of 1-64 blocks, 64 Gbps aggregate raw "
                       "input; 192 iid Gaussian (n in 2048..32768, m=n/4), 64 AR(1) "
                       "(n=65536, m=16384)",
           "window_s": duration_s}
    runs = (("served", binding.EXT_SIM_SERVED, rate, 0.0),
            ("plain", binding.EXT_SIM_PLAIN, rate, 0.5),
            ("plain_at_1/16_load", binding.EXT_SIM_PLAIN, rate / 16, 0.5))
    for name, mode, r, lag in runs:
        if name not in modes:
            continue
        log("served leg: %s, %.1f Gbps raw, %.0f s window" % (name, r * 8 / 1e9, duration_s))
        res, _ = binding.simulate(chans, mode=mode, raw_bytes_per_s=r, warmup_s=warmup_s,
                                  duration_s=duration_s, grace_s=2.0, max_lag_s=lag, seed=4,
                                  producer_threads=producers,
                                  config=binding.server_config(
                                      wg_per_cu=wg_per_cu, timing=timing,
                                      **({"max_inflight": max_inflight} if max_inflight else {}),
                                      **({"split_pairs": split_pairs} if split_pairs >= 0 else {})))
        log("served leg: %s: %s" % (name, json.dumps(res)))
        out[name] = {
            "output_gbps": round(res["out_gbps"], 3),
            "input_gbps": round(res["in_gbps"], 3),
            "offered_input_gbps": round(res["offered_in_gbps"], 3),
            "p50_latency_ms": round(res["lat_p50_us"] / 1e3, 4),
            "p99_latency_ms": round(res["lat_p99_us"] / 1e3, 4),
            "max_latency_ms": round(res["lat_max_us"] / 1e3, 4),
            "blocks": int(res["blocks_measured"]),
            "blocks_missing": int(res["blocks_missing"]),
            "eagain": int(res["eagain"]),
            "max_submit_lag_ms": round(res["max_submit_lag_us"] / 1e3, 3),
            "p99_submit_lag_ms": round(res["submit_lag_p99_us"] / 1e3, 4),
            "p50_service_ms": round(res["service_p50_us"] / 1e3, 4),
            "p99_service_ms": round(res["service_p99_us"] / 1e3, 4),
            "chunks_submitted": int(res["chunks"]),
            "cycles": int(res["cycles"]),
            "mean_cycle_ms": round(res["mean_cycle_us"] / 1e3, 4),
            "eagain_ring": int(res["eagain_ring"]),
            "eagain_stage": int(res["eagain_stage"]),
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-point", action="store_true")
    ap.add_argument("--no-growing", action="store_true", help="skip the Algorithm 2 leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form leg")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-modes", default="served,plain,plain_at_1/16_load",
                    help="comma-separated subset of the served-leg runs")
    ap.add_argument("--serve-inflight", type=int, default=0,
                    help="server cycles queued on the GPU at once (0 = library default)")
    ap.add_argument("--serve-split", type=int, default=-1,
                    help="server split_pairs (1: slice large pairs over work-groups, 0: whole "
                         "pairs; -1 = library default)")
    ap.add_argument("--serve-producers", type=int, default=4,
                    help="load generator threads submitting chunks")
    ap.add_argument("--serve-timing", type=int, default=0,
                    help="1: time every server cycle's phases with GPU events (diagnostic)")
    ap.add_argument("--serve-wg-per-cu", type=int, default=0,
                    help="persistent work-groups per CU in a served cycle (0 = as many as fit)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, also run a plain 64 MiB device copy 4 times (the "
                         "reference kernel that scales HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every block pair is independent, so N GPUs "
              "would each run this same kernel on their own range of block pairs and write "
              "their outputs in place, with no exchange; --gpus %d is not supported."
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_2402_14607_amd import inputs

    log("generating the paper-block workload (n=%d, m=%d, %d pairs)" % (N_BITS, M_BITS, N_PAIRS))
    w = inputs.paper_block(N_PAIRS)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)
        log("cpu baseline: %.4f Gbps" % cpu["value"])

    import torch

    from paper_2402_14607_amd import binding

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)  # the library launches on this stream; events go on it too
    torch.cuda.set_stream(stream)
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    out = torch.empty(N_PAIRS * M_BITS // 8, dtype=torch.uint8, device=dev)
    ex = binding.Extractor(N_BITS, M_BITS, device_memory=True, stream=stream.cuda_stream)
    plan = json.loads(ex.describe())
    log("plan: %s" % json.dumps(plan))

    for _ in range(args.warmup):
        ex.extract(x, y, out, N_PAIRS)
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        ex.extract(x, y, out, N_PAIRS)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(stop) / args.steps
    log("timed %d steps: %.4f ms/step (events), %.4f ms/step (wall)"
        % (args.steps, ms, wall * 1e3 / args.steps))

    if args.copy_probe:
        probe = torch.empty_like(x)
        for _ in range(4):
            probe.copy_(x)
        torch.cuda.synchronize()
        log("copy probe: 4 x %d bytes device-to-device" % x.numel())

    # parity check of the last step's output on sampled pairs (not timed)
    import oracle

    got = out.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(2024))
    idx = np.unique(np.concatenate([[0, N_PAIRS - 1], rng.integers(0, N_PAIRS, 14)])).astype(np.uint64)
    want = oracle.ext_sampled(w.x, w.y, idx, N_BITS, M_BITS)
    qb = M_BITS // 8
    g = np.concatenate([got[int(i) * qb:(int(i) + 1) * qb] for i in idx])
    parity = "bit-exact on %d sampled pairs" % idx.size if np.array_equal(g, want) else "MISMATCH"
    log("parity: %s" % parity)

    batched = None
    if not args.no_batched:
        batched = batched_leg(dev, stream, steps=max(3, min(20, args.steps // 10)), warmup=2)

    paper_point = None
    if not args.no_paper_point:
        paper_point = paper_point_leg(dev, stream, steps=max(5, min(50, args.steps // 4)),
                                      warmup=3)

    growing = None
    if not args.no_growing:
        growing = growing_leg(dev, stream, steps=10, warmup=2)

    served = None
    if not args.no_served:
        served = served_leg(w, duration_s=args.serve_seconds, warmup_s=1.0,
                            modes=args.serve_modes.split(","), wg_per_cu=args.serve_wg_per_cu,
                            max_inflight=args.serve_inflight, split_pairs=args.serve_split,
                            producers=args.serve_producers, timing=args.serve_timing)

    sec = ms * 1e-3
    out_gbps = N_PAIRS * M_BITS / sec / 1e9
    in_gbps = 2 * N_PAIRS * N_BITS / sec / 1e9
    bitmacs = N_PAIRS * N_BITS * M_BITS  # n*m bit-MACs per pair, schoolbook count
    achieved = bitmacs / sec / 1e12
    traffic = measured_traffic()
    # VALU rate against the probe: the launch's VALU lane-ops (rocprofv3
    # summary of this kernel source) per second over the rate the chip
    # delivers now on dependent v_bitop3_b32 / v_alignbit chains
    valu_rate = binding.probe_valu_rate()
    valu_insts = profile_value(VALU_FILE, "valu_insts_per_launch")
    valu_frac = (round(valu_insts * 64 / (valu_rate * sec), 4)
                 if valu_insts and valu_rate > 0 else None)
    log("VALU probe: %.4e lane-ops/s; launch VALU rate / probe rate %s" % (valu_rate, valu_frac))
    res = {
        "metric": "extracted output Gbps at n=8192 (bit-exact); p99 per-block latency when "
                  "streaming",
        "value": round(out_gbps, 3),
        "unit": "Gbps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "paper-scale block: n=8192-bit blocks, m=2048, 65536 block pairs per "
                        "source, iid round(N(128, 20^2)) 8-bit samples, seeds 11/12",
            "n_bits": N_BITS, "m_bits": M_BITS, "block_pairs": N_PAIRS, "form": "plain",
        },
        "input_gbps": round(in_gbps, 3),
        "parity": parity,
        "kernel_plan": plan,
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(PEAK_BITMAC_T, 1),
            "unit": "Tbit-MAC/s",
            "frac": round(achieved / PEAK_BITMAC_T, 4),
            "traffic": traffic,
            "valu_rate_vs_probe": valu_frac,
            "valu_probe_lane_ops_per_s": round(valu_rate, -9),
            # 256 CUs x 4 SIMDs x 16 lanes issue one v_bitop3_b32 lane-op per clock
            "probe_clock_ghz": round(valu_rate / (256 * 64) / 1e9, 3) if valu_rate > 0 else None,
            "note": "achieved counts the schoolbook n*m bit-MACs per pair; peak is one "
                    "32-bit AND-XOR (v_bitop3_b32) per lane per clock on every lane; the "
                    "kernel uses Karatsuba, so frac above 1 is possible; valu_rate_vs_probe "
                    "is the launch's VALU lane-ops (rocprofv3 SQ_INSTS_VALU x 64) per second "
                    "over the rate of the library's probe (dependent v_bitop3_b32 and "
                    "v_alignbit chains on every CU) measured in this run: near 1 the launch "
                    "issues VALU work as fast as the probe; it can exceed 1, since part of "
                    "the counted instructions issue faster than the probe's, so it is a rate "
                    "comparison, not a utilisation",
        },
        "cpu_baseline": cpu,
        "batched": batched,
        "paper_point": paper_point,
        "growing": growing,
        "served": served,
        "context": "paper's simulated FPGA rate: 64 Gbps output (Xilinx Kintex-7 XC7K480T, "
                   "200 MHz, n=71 elements of F_2^80); a different shape, not a target",
    }
    print(json.dumps(res), flush=True)
    ex.close()


if __name__ == "__main__":
    main()

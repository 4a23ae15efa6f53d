"""Benchmark of the FNT Reed-Solomon hot path on one MI355X.

One step = encode a batch of codeword blocks, build the locator of a fresh
erasure pattern, and decode the batch from the received rows (every row of
the method: encoder FNT, locator steps 1-3, decoder steps 4-6).

Workload (default): k = 4096 source symbols, n = 8192, 2048 16-bit lanes per
symbol (4 KiB), 64 codeword blocks sharing one uniformly random erasure
pattern of n - k positions; inputs are uniform 16-bit source symbols stored as
uint32 residues, resident in device memory before timing starts.

Prints one JSON line (see the fields below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOADS = {
    # name: (k, n, lanes, blocks)
    "k4096_n8192_l2048_b64": (4096, 8192, 2048, 64),
    "k256_n512_l512_b1": (256, 512, 512, 1),
    "k32768_n65536_l512_b1": (32768, 65536, 512, 1),
}
DEFAULT = "k4096_n8192_l2048_b64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def decode_butterflies(n, k, lanes, blocks):
    """Radix-2 butterflies of the decoder per launch: inverse FNT_n + FNT_2k + inverse FNT_2k."""
    ln = n.bit_length() - 1
    l2k = (2 * k).bit_length() - 1
    return lanes * blocks * ((n // 2) * ln + 2 * k * l2k)


def cpu_baseline(k, n, seed):
    """The CPU oracle timed on a bounded sample of the workload (one block, a few lanes)."""
    from oracle import codec
    from paper_0907_1788_amd import synth
    lanes_enc, lanes_dec = 32, 32
    src = synth.source(seed, 1, k, lanes_enc)[0].astype(np.int64)
    t0 = time.perf_counter()
    e = codec.encode(src, n)
    t_enc = time.perf_counter() - t0
    z = synth.received_positions(seed + 1, n, k)
    t0 = time.perf_counter()
    d = codec.decode_lagrange(n, z, e[z][:, :lanes_dec])
    t_dec = time.perf_counter() - t0
    assert np.array_equal(d, src[:, :lanes_dec])
    # payload: 2 bytes per source symbol lane, for encode and for decode
    enc_rate = 2 * k * lanes_enc / t_enc
    dec_rate = 2 * k * lanes_dec / t_dec
    value = 2.0 / (1.0 / enc_rate + 1.0 / dec_rate) / 1e9
    return {"value": value, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"one block, encode of {lanes_enc} lanes (Horner) and decode of {lanes_dec} lanes "
                      f"(Lagrange), k={k} n={n}; {t_enc:.1f}s + {t_dec:.1f}s of CPU, single-threaded numpy",
            "enc_GBps": enc_rate / 1e9, "dec_GBps": dec_rate / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   "the coding path needs no inter-GPU exchange (see DESIGN.md)"}))
        sys.exit(2)

    import torch
    from paper_0907_1788_amd import fntrs, synth

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": args.steps}), flush=True)
        return

    k, n, lanes, blocks = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    log("workload", args.workload, "generating inputs")
    src = torch.empty((blocks, k, lanes), dtype=torch.int32, device=dev)
    for b in range(blocks):
        src[b] = torch.from_numpy(synth.source(args.seed * 1000 + b, 1, k, lanes)[0].astype(np.int32)).to(dev)
    enc = torch.empty((blocks, n, lanes), dtype=torch.int32, device=dev)
    out = torch.empty((blocks, k, lanes), dtype=torch.int32, device=dev)
    nsteps = args.steps + args.warmup
    patterns = [synth.received_positions(args.seed + 17 * i, n, k) for i in range(nsteps)]
    ctx = fntrs.Context(0)
    stream = torch.cuda.current_stream()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(nsteps)]
    step_ms = []

    def step(i):
        e = ev[i]
        e[0].record(stream)
        ctx.encode(src, enc, n, stream=stream)
        e[1].record(stream)
        loc = ctx.locator(n, k, patterns[i], stream=stream)
        e[2].record(stream)
        ctx.decode(loc, enc, out, fntrs.FNTRS_RECV_FULL, stream=stream)
        e[3].record(stream)
        loc.release()

    log("warmup", args.warmup)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    log("timed", args.steps)
    t0 = time.perf_counter()
    for i in range(args.warmup, nsteps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for i in range(args.warmup, nsteps):
        step_ms.append(ev[i][0].elapsed_time(ev[i][3]))
    enc_ms = [ev[i][0].elapsed_time(ev[i][1]) for i in range(args.warmup, nsteps)]
    loc_ms = [ev[i][1].elapsed_time(ev[i][2]) for i in range(args.warmup, nsteps)]
    dec_ms = [ev[i][2].elapsed_time(ev[i][3]) for i in range(args.warmup, nsteps)]

    # bit-exactness: every lane of every block decodes back to its source
    exact = bool(torch.equal(out, src))
    log("exact", exact)

    ms = wall * 1e3 / args.steps
    payload = 2 * k * lanes * blocks              # bytes of 16-bit source per direction
    value = 2 * payload / (ms * 1e-3) / 1e9
    dec_avg = float(np.mean(dec_ms))
    enc_avg = float(np.mean(enc_ms))
    dec_bytes = 8 * k * lanes * blocks
    enc_bytes = 4 * (k + n) * lanes * blocks
    res = {
        "metric": "encode/decode payload GB/s (bit-exact) + p50/p99 latency, batched vs plain",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "k": k, "n": n, "lanes": lanes, "blocks": blocks,
                   "pattern": "uniform random n-k erasures, fresh pattern (locator rebuilt) every step",
                   "parallelism": "single GPU"},
        "bit_exact": exact,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "phases_ms": {"encode": enc_avg, "locator": float(np.mean(loc_ms)), "decode": dec_avg},
        "roofline": {"bound": "hbm", "achieved": round(dec_bytes / (dec_avg * 1e-3) / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dec_bytes / (dec_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_decode"},
        "encode_hbm": {"achieved": round(enc_bytes / (enc_avg * 1e-3) / 1e9, 2), "unit": "GB/s"},
        "decode_butterflies_per_s": decode_butterflies(n, k, lanes, blocks) / (dec_avg * 1e-3),
    }

    if not args.no_plain:
        # plain path: one synchronous request per block, no batching
        lat = []
        t0 = time.perf_counter()
        for b in range(blocks):
            t1 = time.perf_counter()
            ctx.encode(src[b], enc[b], n, stream=stream)
            loc = ctx.locator(n, k, patterns[0], stream=stream)
            ctx.decode(loc, enc[b], out[b], fntrs.FNTRS_RECV_FULL, stream=stream)
            loc.release()
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1) * 1e3)
        tp = time.perf_counter() - t0
        res["plain"] = {"value": round(2 * payload / tp / 1e9, 3), "unit": "GB/s",
                        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                        "exact": bool(torch.equal(out, src))}
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(k, n, args.seed)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

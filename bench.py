"""Benchmark of the FNT Reed-Solomon hot path on one MI355X.

Default workload (the headline): an uneven batch of 512 codewords, k = 2^6 ..
2^14, rate 1/2 or 1/4 (n = 128 .. 65536), 128 .. 8192 16-bit lanes per symbol,
each codeword with its own uniformly random erasure pattern.  One step =
batched encode of every codeword, the locators of a fresh pattern per
codeword built together, batched decode (every row of the method: encoder
FNT, locator steps 1-3, decoder steps 4-6).  The same batch is also run as
replayed HIP graphs and through the plain per-codeword calls.  The
single-size workloads (k=4096 n=8192 2048 lanes x 64 blocks; k=256 n=512 512
lanes; k=32768 n=65536 512 lanes) follow as secondary figures.

Inputs are uniform 16-bit source symbols stored as uint32 residues, resident
in device memory before timing starts.  Prints one JSON line.
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

# ALU roofline of the coding kernels: 256 CUs x 64 int32 lanes x 2.4 GHz =
# 39.3 T lane-ops/s; a modular radix-2 butterfly over GF(65537) costs at
# least 6 int32 operations in the kernels' representation (two 24-bit
# multiplies, two folding adds, one add, one subtract), so the chip tops out
# at 39.3e12 / 6 butterflies per second.  The 6 is the instruction floor of
# the representation, an assumption of the peak, not a measured count.
VALU_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_BUTTERFLY = 6
ALU_PEAK_BFLY = VALU_LANE_OPS / OPS_PER_BUTTERFLY
PEAK_BASIS = ("256 CUs x 64 int32 lanes x 2.4 GHz / 6 VALU ops per radix-2 butterfly "
              "(2 mul24 + 2 fold + add + sub: the floor of the representation, assumed)")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    # name: (k, n, lanes, blocks)
    "k4096_n8192_l2048_b64": (4096, 8192, 2048, 64),
    "k256_n512_l512_b1": (256, 512, 512, 1),
    "k32768_n65536_l512_b1": (32768, 65536, 512, 1),
}
# uneven batch: 512 codewords, k = 2^(6..14), rate 1/2 or 1/4, 128..8192 lanes,
# one erasure pattern per codeword (sizes from synth.uneven_batch, seed 4)
UNEVEN = "uneven512_seed4"
# served stream: Poisson arrivals of encode (60%) and decode (40%) requests with
# sizes from the uneven-batch distribution, offered load swept around the
# measured batched peak, 32 GB device working-set cap
SERVED = "served_poisson"
# evaluation of 4 x 2048 polynomials of degree < 4096 at 4096 points of a
# geometric sequence (the chirp of Sec. II-B): one product of length 8192
CHIRP = "chirp_L4096_M4096_l2048_b4"
CHIRP_SHAPE = (4096, 4096, 2048, 4)   # L, M, lanes, blocks
DEFAULT = UNEVEN
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# The paper's best reported encoding speed (non-systematic FNT code, rate 1/2)
# and the machine it was measured on (Abstract; Sec. IV): context beside the
# figures here, not a baseline of the same workload (vs_baseline stays null).
PAPER_CONTEXT = {"encode_Mbps": 150, "encode_GBps": 0.01875,
                 "hardware": "Intel Core 2 Extreme at 3.06 GHz, one CPU (thread count not stated)",
                 "workload": "codes of up to several 10^4 symbols; packet size not stated"}


def decode_butterflies(n, k, lanes, blocks):
    """Radix-2 butterflies of one decode launch: inverse FNT_n (step 5) and the
    two length-M transforms of the low product (step 6), M = 2^max(ceil(log2 k) + 1,
    log2 n - 1): at least 2k and n/2, as the library chooses it."""
    ln = n.bit_length() - 1
    lm = max((k - 1).bit_length() + 1, ln - 1)
    return lanes * blocks * ((n // 2) * ln + 2 * ((1 << lm) // 2) * lm)


def encode_butterflies(n, k, lanes, blocks):
    """Radix-2 butterflies of one encode launch: n/K transforms of size K = 2^ceil(log2 k)."""
    lk = max(1, (k - 1).bit_length())
    return lanes * blocks * (n // (1 << lk)) * ((1 << lk) // 2) * lk


def source_hash():
    """Hash of the HIP sources, to tell whether stored counter figures still apply."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0907_1788_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it matches these sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("workload") != workload or e.get("src_hash") != source_hash():
        return None
    return e["hbm_bytes_per_launch"]


def oracle_workers():
    """Worker processes for the CPU oracle: the host's cores, at most 16 (the
    CPU share of one GPU on the benchmark machines)."""
    return max(1, min(16, os.cpu_count() or 1))


def _oracle_leg(job):
    """One timed leg of the CPU oracle, run in a worker process: Horner
    encode and Lagrange decode (or the systematic code) of `lanes` lanes of one
    codeword; returns (k, n, lanes, encode s, decode s)."""
    k, n, lanes, seed, systematic = job
    from oracle import codec
    from paper_0907_1788_amd import synth
    src = synth.source(seed, 1, k, lanes)[0].astype(np.int64)
    z = synth.received_positions(seed + 1, n, k)
    encode = codec.systematic_encode if systematic else codec.encode
    decode = codec.systematic_decode if systematic else codec.decode_lagrange
    t0 = time.perf_counter()
    e = encode(src, n)
    te = time.perf_counter() - t0
    t0 = time.perf_counter()
    d = decode(n, z, e[z])
    td = time.perf_counter() - t0
    if not np.array_equal(d, src):
        raise AssertionError(f"oracle round trip failed at k={k} n={n}")
    return k, n, lanes, te, td


def _oracle_lanes(k, n, budget_s):
    """Lanes of one leg that take about budget_s seconds (the oracle's cost
    is about n*k multiply-adds per lane to encode and a few k^2 to decode)."""
    per_lane = 8e-9 * n * k + 3e-8 * k * k
    return int(max(1, min(4096, budget_s / per_lane)))


def _run_legs(jobs, workers):
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_oracle_leg, jobs, chunksize=1)


def cpu_baseline(k, n, seed, budget_s=8.0, systematic=False):
    """The CPU oracle on a bounded sample of a single-size workload: every
    worker process times encode + decode of its own share of one block's
    lanes; the aggregate rate over the workers is the oracle's throughput."""
    workers = oracle_workers()
    lanes = _oracle_lanes(k, n, budget_s)
    legs = _run_legs([(k, n, lanes, seed + 101 * w, systematic) for w in range(workers)], workers)
    enc_rate = sum(2 * k * l / te for _, _, l, te, _ in legs)
    dec_rate = sum(2 * k * l / td for _, _, l, _, td in legs)
    value = 2.0 / (1.0 / enc_rate + 1.0 / dec_rate) / 1e9
    wall = max(te + td for *_, te, td in legs)
    return {"value": value, "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": f"k={k} n={n}: {workers} processes, each the {'systematic ' if systematic else ''}encode "
                      f"(Horner) and decode (Lagrange) of {lanes} lanes of one block, {wall:.1f} s wall; "
                      f"rate = sum over the processes, extrapolated linearly in lanes to the full payload "
                      f"(host reports {os.cpu_count()} cores)",
            "enc_GBps": enc_rate / 1e9, "dec_GBps": dec_rate / 1e9}


def cpu_baseline_uneven(sizes, seed, budget_s=6.0):
    """The CPU oracle on a bounded sample of the uneven batch: one leg per
    distinct (k, n) of the batch, a few lanes each, in parallel worker
    processes; every codeword's time is its class's time per lane times its
    lanes, and the batch's time is their sum divided over the workers."""
    workers = oracle_workers()
    classes = sorted({(k, n) for k, n, _ in sizes}, key=lambda c: -c[0] * c[1])
    jobs = [(k, n, _oracle_lanes(k, n, budget_s), seed + 7 * i, False) for i, (k, n) in enumerate(classes)]
    legs = _run_legs(jobs, workers)
    per_lane = {(k, n): ((te + td) / l, te / l, td / l) for k, n, l, te, td in legs}
    t1 = sum(per_lane[(k, n)][0] * l for k, n, l in sizes)
    payload = sum(2 * k * l for k, n, l in sizes)
    wall = max(te + td for *_, te, td in legs)
    return {"value": 2 * payload / (t1 / workers) / 1e9, "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": f"one leg per (k, n) class of the batch ({len(classes)} classes, "
                      f"{sum(j[2] for j in jobs)} lanes in all) timed in {workers} worker processes "
                      f"({wall:.1f} s wall for the longest): Horner encode + Lagrange decode; extrapolated "
                      f"linearly in lanes to every codeword of the batch and divided over {workers} cores "
                      f"(host reports {os.cpu_count()} cores)"}


def run_uneven(args, torch, fntrs, synth):
    """Uneven batch: one step = batched encode of all codewords, the locators
    of a fresh erasure pattern per codeword built together, batched decode.
    Returns the result dict (printed by main)."""
    sizes = synth.uneven_batch(4, 512)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    log("workload", UNEVEN, "allocating", len(sizes), "codewords")
    cws = []
    for k, n, lanes in sizes:
        src = torch.randint(0, 65536, (1, k, lanes), dtype=torch.int32, device=dev, generator=gen)
        enc = torch.empty((1, n, lanes), dtype=torch.int32, device=dev)
        dec = torch.empty((1, k, lanes), dtype=torch.int32, device=dev)
        cws.append((k, n, lanes, src, enc, dec))
    torch.cuda.synchronize()
    ndef = 0 if args.no_tune else min(3, args.steps)   # steps timed with the default configurations
    nsteps = args.steps + args.warmup + ndef + (0 if args.no_tune else 1)
    rng = np.random.default_rng(args.seed)
    log("drawing", nsteps, "x", len(sizes), "erasure patterns")
    patterns = [[(n, k, np.sort(rng.choice(n, k, replace=False)).astype(np.uint32)) for k, n, _ in sizes]
                for _ in range(nsteps)]
    ctx = fntrs.Context(0, workspace_cap_bytes=16 << 30)
    stream = torch.cuda.current_stream()
    enc_jobs = [ctx.encode_job(src, enc, n) for k, n, lanes, src, enc, dec in cws]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nsteps)]
    held = []

    def step(i):
        e = ev[i]
        e[0].record(stream)
        ctx.submit(enc_jobs, stream=stream)
        e[1].record(stream)
        locs = ctx.locators(patterns[i], stream=stream)
        e[2].record(stream)
        ctx.submit([ctx.decode_job(loc, enc, dec, fntrs.FNTRS_RECV_FULL)
                    for loc, (k, n, lanes, src, enc, dec) in zip(locs, cws)], stream=stream)
        e[3].record(stream)
        held.append(locs)

    log("warmup", args.warmup)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    tuning = None
    default_ms = None
    first = args.warmup
    if not args.no_tune:
        # the default configurations, then the autotuner on this batch's own jobs
        t0 = time.perf_counter()
        for i in range(first, first + ndef):
            step(i)
        torch.cuda.synchronize()
        default_ms = (time.perf_counter() - t0) * 1e3 / ndef
        log("default configurations", round(default_ms, 3), "ms/step; tuning")
        tl = ctx.locators(patterns[0], stream=stream)
        tuning = ctx.autotune_batch(enc_jobs, reps=3, stream=stream)
        tuning += ctx.autotune_batch([ctx.decode_job(loc, enc, dec, fntrs.FNTRS_RECV_FULL)
                                      for loc, (k, n, lanes, src, enc, dec) in zip(tl, cws)], reps=3, stream=stream)
        for loc in tl:
            loc.release()
        step(first + ndef)   # warm-up with the tuned configurations
        torch.cuda.synchronize()
        first += ndef + 1
    log("timed", args.steps)
    t0 = time.perf_counter()
    for i in range(first, nsteps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    exact = all(torch.equal(dec, src) for k, n, lanes, src, enc, dec in cws)
    log("exact", exact)
    ph = {name: float(np.mean([ev[i][a].elapsed_time(ev[i][b]) for i in range(first, nsteps)]))
          for name, a, b in (("encode", 0, 1), ("locator", 1, 2), ("decode", 2, 3))}
    step_ms = [ev[i][0].elapsed_time(ev[i][3]) for i in range(first, nsteps)]
    for locs in held:
        for loc in locs:
            loc.release()
    held.clear()
    ks = np.array([c[0] for c in cws], dtype=np.float64)
    ns = np.array([c[1] for c in cws], dtype=np.float64)
    ls = np.array([c[2] for c in cws], dtype=np.float64)
    payload = float((2 * ks * ls).sum())
    ms = wall * 1e3 / args.steps
    bfly = float(sum(encode_butterflies(int(n), int(k), int(l), 1) + decode_butterflies(int(n), int(k), int(l), 1)
                     for k, n, l in zip(ks, ns, ls)))
    alg = float((4 * (ks + ns) * ls + 8 * ks * ls).sum())
    res = {
        "metric": "encode/decode payload GB/s (bit-exact) + p50/p99 latency, batched vs plain",
        "value": round(2 * payload / (ms * 1e-3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "paper_context": PAPER_CONTEXT, "dtype": "u32", "data": "synthetic",
        "config": {"workload": UNEVEN, "codewords": len(cws), "payload_bytes": int(payload),
                   "k": "2^6..2^14", "rate": "1/2 or 1/4", "lanes": "128..8192",
                   "pattern": "fresh uniform random n-k erasures per codeword every step (locators rebuilt)",
                   "parallelism": "single GPU"},
        "bit_exact": bool(exact),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "phases_ms": ph,
        "tuning": None if tuning is None else {
            "default_ms_per_step": round(default_ms, 4),
            "classes": [{key: t[key] for key in ("op", "log2_size", "method", "tile_lanes", "threads",
                                                 "lanes_per_thread", "radix_log2", "ms", "default_ms")}
                        for t in tuning]},
        "step": {"butterflies": bfly, "algorithmic_hbm_bytes": alg,
                 "alu_frac": round(bfly / (ms * 1e-3) / ALU_PEAK_BFLY, 4),
                 "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    # the same batch captured in graphs (fixed patterns), replayed
    locs = ctx.locators(patterns[-1], stream=stream)
    g_enc = ctx.graph(enc_jobs)
    g_dec = ctx.graph([ctx.decode_job(loc, enc, dec, fntrs.FNTRS_RECV_FULL)
                       for loc, (k, n, lanes, src, enc, dec) in zip(locs, cws)])
    g_enc.launch(stream)
    g_dec.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g_enc.launch(stream)
        g_dec.launch(stream)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / args.steps
    res["graph"] = {"value": round(2 * payload / (gms * 1e-3) / 1e9, 3), "unit": "GB/s", "ms_per_step": round(gms, 4),
                    "note": "encode and decode graphs replayed, locators prebuilt",
                    "exact": bool(all(torch.equal(dec, src) for k, n, lanes, src, enc, dec in cws))}
    g_enc.destroy()
    g_dec.destroy()
    # The dominant kernel class of this workload: the four-step decoder
    # (k4_dec1..4, transforms of 2^14 points or more), about half of the
    # summed kernel time.  One call on the largest such code of the batch,
    # timed with events on the stream it runs on.
    j4 = max((i for i, c in enumerate(cws) if c[1] >= 16384), key=lambda i: (cws[i][1], cws[i][2]))
    k4, n4, l4, src4, enc4, dec4 = cws[j4]
    ctx.decode(locs[j4], enc4, dec4, fntrs.FNTRS_RECV_FULL, stream=stream)
    e4 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    e4[0].record(stream)
    for _ in range(reps):
        ctx.decode(locs[j4], enc4, dec4, fntrs.FNTRS_RECV_FULL, stream=stream)
    e4[1].record(stream)
    torch.cuda.synchronize()
    ms4 = e4[0].elapsed_time(e4[1]) / reps
    b4 = decode_butterflies(n4, k4, l4, 1)
    a4 = 8 * k4 * l4
    res["roofline"] = {"bound": "alu", "kernel": f"four-step decoder k4_dec1..4 (one call: n={n4} k={k4} "
                                                 f"lanes={l4}, four launches back to back)",
                       "achieved": round(b4 / (ms4 * 1e-3) / 1e12, 4), "peak": round(ALU_PEAK_BFLY / 1e12, 4),
                       "unit": "Tbutterfly/s", "frac": round(b4 / (ms4 * 1e-3) / ALU_PEAK_BFLY, 4),
                       "traffic": stored_traffic("k4_dec", UNEVEN), "ms_per_call": round(ms4, 4),
                       "butterflies_per_call": b4, "algorithmic_hbm_bytes": a4,
                       "hbm_frac": round(a4 / (ms4 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "peak_basis": PEAK_BASIS}
    if not args.no_plain:
        # plain path: one synchronous request per codeword, no batching
        lat = []
        t0 = time.perf_counter()
        for (k, n, lanes, src, enc, dec), loc in zip(cws, locs):
            t1 = time.perf_counter()
            ctx.encode(src, enc, n, stream=stream)
            ctx.decode(loc, enc, dec, fntrs.FNTRS_RECV_FULL, stream=stream)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1) * 1e3)
        tp = time.perf_counter() - t0
        res["plain"] = {"value": round(2 * payload / tp / 1e9, 3), "unit": "GB/s",
                        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                        "exact": bool(all(torch.equal(dec, src) for k, n, lanes, src, enc, dec in cws)),
                        "note": "per-codeword encode + decode, synchronous; locators prebuilt"}
    for loc in locs:
        loc.release()
    ctx.close()
    del cws, enc_jobs
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline_uneven(sizes, args.seed)
    return res


def served_pool(torch, ctx, synth, seed, count=64):
    """The resident codewords of the served stream: sizes of the uneven-batch
    distribution, uniform 16-bit source, encoded once: (k, n, lanes, src, enc)."""
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    pool = []
    for k, n, lanes in synth.uneven_batch(seed + 1, count):
        src = torch.randint(0, 65536, (1, k, lanes), dtype=torch.int32, device=dev, generator=gen)
        enc = torch.empty((1, n, lanes), dtype=torch.int32, device=dev)
        ctx.encode(src, enc, n)
        pool.append((k, n, lanes, src, enc))
    return pool


def served_requests(serve, pool, rng, count, arrivals, pattern_pool=0):
    """`count` requests over `pool`: 60% encode, 40% decode from the full
    codeword with a uniformly random erasure pattern, or (pattern_pool > 0)
    one of `pattern_pool` patterns per code, so that locators repeat."""
    out = []
    for i in range(count):
        k, n, lanes, src, enc = pool[int(rng.integers(len(pool)))]
        if rng.random() < 0.6:
            r = serve.Request(serve.ENCODE, n, k, lanes, src)
        else:
            if pattern_pool:
                prng = np.random.default_rng(n * 131 + k * 7 + int(rng.integers(pattern_pool)))
            else:
                prng = rng
            z = np.sort(prng.choice(n, k, replace=False)).astype(np.uint32)
            r = serve.Request(serve.DECODE, n, k, lanes, enc, positions=z)
            r.src_ref = src
        r.arrival = float(arrivals[i])
        r.rid = i
        out.append(r)
    return out


def run_served(args, torch, fntrs, synth):
    """Served stream over a pool of 64 resident codewords of the uneven-batch
    size distribution: the closed-loop peak (all requests at once), then
    Poisson arrivals at a sweep of offered loads (fresh erasure pattern per
    decode request).  The point with 16 patterns per code (locator cache hits)
    is not run: its only run ended in a GPU memory fault whose cause is not
    shown."""
    from paper_0907_1788_amd import serve
    ctx = fntrs.Context(0, workspace_cap_bytes=args.workspace_gib << 30)
    pool = served_pool(torch, ctx, synth, args.seed)
    torch.cuda.synchronize()
    log("pool of", len(pool), "codewords,", sum(2 * k * l for k, n, l, _, _ in pool) / 1e9, "GB payload")
    rng = np.random.default_rng(args.seed)

    def requests(count, arrivals, pattern_pool=0):
        return served_requests(serve, pool, rng, count, arrivals, pattern_pool)

    # mismatching elements of every decode result against its source, summed
    # on the device (no host synchronisation inside the serving loop)
    bad = torch.zeros((), dtype=torch.int64, device="cuda")

    def check(r):
        if r.op == serve.DECODE:
            bad.add_((r.out != r.src_ref).sum())
            # the comparison runs on this stream: keep the block from being
            # reused by a later batch on the request's stream until it has
            r.out.record_stream(torch.cuda.current_stream())
        r.out = None

    cap = 32 << 30
    # the kernel configurations of the served size classes, tuned once on one
    # request of each pool entry and kind (kept in the context for every batch)
    tuned = []
    if not args.no_tune:
        sample = []
        for k, n, lanes, src, enc in pool:
            sample.append(serve.Request(serve.ENCODE, n, k, lanes, src))
            z = np.sort(rng.choice(n, k, replace=False)).astype(np.uint32)
            sample.append(serve.Request(serve.DECODE, n, k, lanes, enc, positions=z))
        tuned = serve.Server(ctx, mem_cap_bytes=cap).autotune(sample)
        torch.cuda.synchronize()
        log("tuned", len(tuned), "classes")
    # closed loop: every request present at t = 0
    reqs = requests(args.requests, np.zeros(args.requests))
    serve.Server(ctx, mem_cap_bytes=cap).run(reqs[: min(200, len(reqs))], on_done=check)   # warm-up
    st = serve.Server(ctx, mem_cap_bytes=cap).run(reqs, on_done=check)
    peak = st.gbps
    mean_payload = st.payload_bytes / st.completed
    closed = {"GBps": round(peak, 3), "seconds": round(st.seconds, 3), "batches": st.batches,
              "mean_batch": round(st.mean_batch, 2), "peak_working_set_GB": round(st.peak_bytes / 1e9, 2),
              "host_ms": st.host_ms}
    log("closed-loop peak", closed)
    sweep = []
    for load in args.loads:
        rate = load * peak * 1e9 / mean_payload
        reqs = requests(args.requests, serve.poisson_arrivals(rate, args.requests, args.seed + int(load * 100)))
        st = serve.Server(ctx, mem_cap_bytes=cap).run(reqs, on_done=check)
        sweep.append({"offered_load": load, "offered_GBps": round(load * peak, 3), "achieved_GBps": round(st.gbps, 3),
                      "p50_ms": round(st.latency_ms["p50"], 3), "p99_ms": round(st.latency_ms["p99"], 3),
                      "batches": st.batches, "mean_batch": round(st.mean_batch, 2),
                      "peak_inflight": st.peak_inflight, "peak_working_set_GB": round(st.peak_bytes / 1e9, 2),
                      "seconds": round(st.seconds, 3), "host_ms": st.host_ms})
        log("load", load, sweep[-1])
    ctx.close()
    at100 = min(sweep, key=lambda p: abs(p["offered_load"] - 1.0))
    res = {
        "metric": "encode/decode payload GB/s (bit-exact) + p50/p99 latency, batched vs plain",
        "value": round(max(p["achieved_GBps"] for p in sweep), 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.requests, "warmup": 200, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": SERVED, "pool_codewords": len(pool), "requests_per_point": args.requests,
                   "mix": "60% encode / 40% decode", "working_set_cap_GB": cap / 2**30,
                   "context_workspace_GiB": args.workspace_gib,
                   "parallelism": "single GPU"},
        "bit_exact": int(bad.item()) == 0,
        "closed_loop_peak_GBps": round(peak, 3),
        "closed_loop": closed,
        "latency_ms": {"p50": at100["p50_ms"], "p99": at100["p99_ms"], "at_offered_load": at100["offered_load"]},
        "sweep": sweep,
        "locator_cache_point": "not run: its only GPU run ended in a memory fault whose cause is not shown",
        "tuning": tuned,
    }
    print(json.dumps(res), flush=True)


def cpu_baseline_chirp(synth, L, M, seed, budget_s=10.0):
    """The oracle's chirp evaluation (one schoolbook product per lane) on
    whole lanes of the workload, one process, until the budget is spent."""
    from oracle import chirp
    c = synth.residues(seed, (L, 64))
    t0 = time.perf_counter()
    done = 0
    while done < 64 and time.perf_counter() - t0 < budget_s:
        chirp.chirp_eval(c[:, done], 3, M, 5)
        done += 1
    dt = time.perf_counter() - t0
    return {"value": round(4 * (L + M) * done / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} lanes of L = {L}, M = {M} (oracle/chirp.py, schoolbook middle product), {dt:.1f} s"}


def run_chirp(args, torch, fntrs, synth, cpu=True):
    """Evaluation on a geometric sequence by one middle product (fntrs_chirp_eval):
    one step = one call over every block.  Exactness: Horner's rule at sampled
    points on the host, every lane of the first and last block."""
    L, M, lanes, blocks = CHIRP_SHAPE
    dev = torch.device("cuda:0")
    a, q = 5, 3
    coef = torch.from_numpy(synth.residues(args.seed, (blocks, L, lanes)).astype(np.int32)).to(dev)
    out = torch.empty((blocks, M, lanes), dtype=torch.int32, device=dev)
    ctx = fntrs.Context(0)
    stream = torch.cuda.current_stream()
    nsteps = args.steps + args.warmup
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(nsteps)]
    for i in range(nsteps):
        ev[i][0].record(stream)
        ctx.chirp_eval(coef, out, a, q, stream=stream)
        ev[i][1].record(stream)
        if i == args.warmup - 1:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    ms_list = [ev[i][0].elapsed_time(ev[i][1]) for i in range(args.warmup, nsteps)]
    ms = float(np.mean(ms_list))
    pick = np.array([0, 1, 2, 977, 2048, M - 1])
    x = np.array([a * pow(q, int(i), 65537) % 65537 for i in pick], dtype=np.int64)[:, None]
    exact = True
    for b in (0, blocks - 1):
        cb = coef[b].cpu().numpy().astype(np.int64)
        ref = np.zeros((pick.size, lanes), dtype=np.int64)
        for j in range(L - 1, -1, -1):
            ref = (ref * x + cb[j][None, :]) % 65537
        exact &= bool(np.array_equal(out[b].cpu().numpy().astype(np.int64)[pick], ref))
    log("chirp exact", exact, "ms", ms)
    nbytes = 4 * (L + M) * lanes * blocks
    P = 1 << (L + M - 2).bit_length()            # the product length, 2^ceil(log2(L+M-1))
    bfly = 2 * (P // 2) * (P.bit_length() - 1) * lanes * blocks   # two P-point transforms per lane
    res = {
        "metric": "chirp evaluation GB/s (coefficients in + values out, bit-exact)",
        "value": round(nbytes / (ms * 1e-3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": CHIRP, "L": L, "M": M, "lanes": lanes, "blocks": blocks, "a": a, "q": q,
                   "product_length": 8192, "parallelism": "single GPU"},
        "bit_exact": exact,
        "latency_ms": {"p50": float(np.percentile(ms_list, 50)), "p99": float(np.percentile(ms_list, 99))},
        # the fused kernel (k_chirp: DIF FNT_P, product, inverse DIT FNT_P per
        # lane, in LDS) holds most of the call; the call is timed as a whole
        "roofline": {"bound": "alu", "kernel": "fntrs_chirp_eval (fused k_chirp<13> + table kernels, whole call)",
                     "achieved": round(bfly / (ms * 1e-3) / 1e12, 4), "peak": round(ALU_PEAK_BFLY / 1e12, 4),
                     "unit": "Tbutterfly/s", "peak_basis": PEAK_BASIS,
                     "frac": round(bfly / (ms * 1e-3) / ALU_PEAK_BFLY, 4), "traffic": None,
                     "butterflies_per_call": bfly, "algorithmic_hbm_bytes": nbytes,
                     "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    ctx.close()
    if cpu:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline_chirp(synth, L, M, args.seed)
    return res


def run_single(args, torch, fntrs, synth, workload, cpu=True):
    """A single-size workload: one step = encode every block, build the locator
    of a fresh pattern shared by the blocks, decode every block.  Returns the
    result dict."""
    k, n, lanes, blocks = WORKLOADS[workload]
    dev = torch.device("cuda:0")
    log("workload", workload, "generating inputs")
    src = torch.empty((blocks, k, lanes), dtype=torch.int32, device=dev)
    for b in range(blocks):
        src[b] = torch.from_numpy(synth.source(args.seed * 1000 + b, 1, k, lanes)[0].astype(np.int32)).to(dev)
    enc = torch.empty((blocks, n, lanes), dtype=torch.int32, device=dev)
    out = torch.empty((blocks, k, lanes), dtype=torch.int32, device=dev)
    nsteps = args.steps + args.warmup
    patterns = [synth.received_positions(args.seed + 17 * i, n, k) for i in range(nsteps)]
    ctx = fntrs.Context(0)
    stream = torch.cuda.current_stream()
    # a workload that fits in the caches (L2 4 MiB per XCD, 256 MiB Infinity
    # Cache) would otherwise start every step from the previous step's data
    footprint = 4 * lanes * blocks * (2 * k + n)
    flush = None
    if args.flush_mib > 0 and footprint < (1 << 30):
        flush = torch.empty(args.flush_mib << 18, dtype=torch.int32, device=dev)

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(nsteps)]
    step_ms = []

    sysf = fntrs.FNTRS_SYSTEMATIC if args.systematic else 0
    if getattr(args, "direct", False):
        sysf |= fntrs.FNTRS_DIRECT   # the quadratic methods of Sec. III (small codes)

    def step(i):
        e = ev[i]
        if flush is not None:
            flush.fill_(i)   # outside the step's events
        e[0].record(stream)
        ctx.encode(src, enc, n, flags=sysf, stream=stream)
        e[1].record(stream)
        loc = ctx.locator(n, k, patterns[i], stream=stream)
        e[2].record(stream)
        ctx.decode(loc, enc, out, fntrs.FNTRS_RECV_FULL | sysf, stream=stream)
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

    # with flushes between steps the step time comes from its events, which
    # exclude the flush; otherwise from the wall clock over all steps
    ms = float(np.mean(step_ms)) if flush is not None else wall * 1e3 / args.steps
    payload = 2 * k * lanes * blocks              # bytes of 16-bit source per direction
    value = 2 * payload / (ms * 1e-3) / 1e9
    dec_avg = float(np.mean(dec_ms))
    enc_avg = float(np.mean(enc_ms))
    dec_bytes = 8 * k * lanes * blocks
    enc_bytes = 4 * (k + n) * lanes * blocks
    dec_bfly = decode_butterflies(n, k, lanes, blocks)
    enc_bfly = encode_butterflies(n, k, lanes, blocks)
    if args.systematic:
        # each side runs the decoder's transforms and the encoder's
        dec_bfly = enc_bfly = dec_bfly + enc_bfly
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
        "paper_context": PAPER_CONTEXT,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": workload, "k": k, "n": n, "lanes": lanes, "blocks": blocks,
                   "code": "systematic" if args.systematic else "non-systematic",
                   "method": "direct (quadratic)" if getattr(args, "direct", False) else "FNT",
                   "pattern": "uniform random n-k erasures, fresh pattern (locator rebuilt) every step",
                   "caches": (f"{args.flush_mib} MiB written between steps, outside the timed events"
                              if flush is not None else "buffers larger than the caches" if footprint >= (1 << 30)
                              else "no flush between steps: buffers may be cache-resident"),
                   "parallelism": "single GPU"},
        "bit_exact": exact,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "phases_ms": {"encode": enc_avg, "locator": float(np.mean(loc_ms)), "decode": dec_avg},
        # dominant kernel: the decoder, bound by the integer vector ALUs
        "roofline": {"bound": "alu", "kernel": "k_dec + k_enc_cos (systematic decode)" if args.systematic else "k_dec",
                     "achieved": round(dec_bfly / (dec_avg * 1e-3) / 1e12, 4),
                     "peak": round(ALU_PEAK_BFLY / 1e12, 4), "unit": "Tbutterfly/s", "peak_basis": PEAK_BASIS,
                     "frac": round(dec_bfly / (dec_avg * 1e-3) / ALU_PEAK_BFLY, 4),
                     "traffic": None if args.systematic else stored_traffic("k_dec", workload),
                     "algorithmic_hbm_bytes": dec_bytes,
                     "hbm_frac": round(dec_bytes / (dec_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "encode_roofline": {"bound": "alu", "kernel": "k_dec + k_enc_cos (systematic encode)"
                            if args.systematic else "k_enc_cos",
                            "achieved": round(enc_bfly / (enc_avg * 1e-3) / 1e12, 4),
                            "peak": round(ALU_PEAK_BFLY / 1e12, 4), "unit": "Tbutterfly/s",
                            "frac": round(enc_bfly / (enc_avg * 1e-3) / ALU_PEAK_BFLY, 4),
                            "traffic": None if args.systematic else stored_traffic("k_enc_cos", workload),
                            "algorithmic_hbm_bytes": enc_bytes,
                            "hbm_frac": round(enc_bytes / (enc_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }

    if not args.no_plain:
        # plain path: one synchronous request per block, no batching
        lat = []
        if flush is not None:
            flush.fill_(-1)
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(blocks):
            t1 = time.perf_counter()
            ctx.encode(src[b], enc[b], n, flags=sysf, stream=stream)
            loc = ctx.locator(n, k, patterns[0], stream=stream)
            ctx.decode(loc, enc[b], out[b], fntrs.FNTRS_RECV_FULL | sysf, stream=stream)
            loc.release()
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1) * 1e3)
        tp = time.perf_counter() - t0
        res["plain"] = {"value": round(2 * payload / tp / 1e9, 3), "unit": "GB/s",
                        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                        "exact": bool(torch.equal(out, src))}
    ctx.close()
    del src, enc, out, flush
    torch.cuda.empty_cache()
    if cpu:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(k, n, args.seed, systematic=args.systematic)
    return res




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + [UNEVEN, SERVED, CHIRP])
    ap.add_argument("--requests", type=int, default=2000, help="requests per load point (served workload)")
    ap.add_argument("--workspace-gib", type=int, default=40,
                    help="served workload: the context's workspace cap (locator cache, stream-ordered pool kept)")
    ap.add_argument("--loads", type=lambda t: [float(x) for x in t.split(",")],
                    default=[0.10, 0.25, 0.50, 0.75, 0.90, 1.00, 1.10, 1.20],
                    help="offered loads of the served sweep, as fractions of the closed-loop peak")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="uneven batch only, without the single-size workloads")
    ap.add_argument("--no-tune", action="store_true", help="uneven batch: keep the default kernel configurations")
    ap.add_argument("--systematic", action="store_true",
                    help="the systematic code (Sec. II-C): interpolation + transform on both sides")
    ap.add_argument("--direct", action="store_true",
                    help="the direct (quadratic) encoder and decoder of Sec. III instead of the transforms")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--flush-mib", type=int, default=512,
                    help="MiB written between steps when the workload's buffers total under 1 GiB, so that "
                         "no step starts from data the previous one left in the caches (0: never)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: lanes, codewords and "
                                   "requests shard over GPUs with no exchange, so one GPU's "
                                   "throughput is the figure"}))
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

    if args.workload == SERVED:
        run_served(args, torch, fntrs, synth)
        return
    if args.workload == CHIRP:
        print(json.dumps(run_chirp(args, torch, fntrs, synth, cpu=not args.no_cpu_baseline)), flush=True)
        return
    if args.workload != UNEVEN:
        print(json.dumps(run_single(args, torch, fntrs, synth, args.workload, cpu=not args.no_cpu_baseline)),
              flush=True)
        return
    res = run_uneven(args, torch, fntrs, synth)
    if not args.no_secondary:
        # the single-size workloads, briefly, as secondary figures
        sec = argparse.Namespace(**vars(args))
        sec.steps, sec.warmup, sec.systematic, sec.direct = max(3, min(args.steps, 10)), 2, False, False
        other = {}
        for w in ("k4096_n8192_l2048_b64", "k256_n512_l512_b1", "k32768_n65536_l512_b1"):
            r = run_single(sec, torch, fntrs, synth, w, cpu=False)
            other[w] = {key: r[key] for key in ("value", "ms_per_step", "bit_exact", "latency_ms", "phases_ms")}
            other[w]["steps"] = sec.steps
            other[w]["plain_GBps"] = r.get("plain", {}).get("value")
            other[w]["decoder_alu_frac"] = r["roofline"]["frac"]
            other[w]["encoder_alu_frac"] = r["encode_roofline"]["frac"]
            log(w, other[w]["value"], "GB/s")
        res["other_workloads"] = other
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

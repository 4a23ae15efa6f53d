"""Replays the served request stream through libfntrs on the stream-order
checker (fake_hip.cpp) instead of a GPU.

Run as a script in a fresh process: it loads the checker under the HIP
runtime's soname before libfntrs, so every HIP call of the library lands in
the checker, and it stands a minimal `torch` in for the real one (device
buffers, streams and events over the checker), so that the unmodified
serve.Server and the benchmark's own pool and request generators drive the
library.  Kernels do not run: the checker executes each enqueued operation
in a seeded random order and verifies the ranges it touches.  Prints one
JSON line: the checker's error messages and counts.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import types

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))


def load(fake_path):
    """The checker (global symbols, HIP runtime soname) and then libfntrs."""
    fake = ctypes.CDLL(fake_path, mode=ctypes.RTLD_GLOBAL)
    fake.fakehip_error_text.restype = ctypes.c_char_p
    fake.fakehip_set_lag.argtypes = [ctypes.c_double]
    fake.fakehip_seed.argtypes = [ctypes.c_uint64]
    fake.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    fake.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
    fake.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    fake.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    fake.hipEventQuery.argtypes = [ctypes.c_void_p]
    fake.hipStreamWaitEvent.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint]
    fake.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    return fake


def fake_torch(fake):
    """A stand-in for the parts of torch that serve.py, fntrs.py and the
    benchmark's pool builder use, backed by the checker."""
    t = types.ModuleType("torch")
    t.int32 = "int32"

    class device:  # noqa: N801
        def __init__(self, *a, **k):
            pass

    class Generator:
        def __init__(self, *a, **k):
            pass

        def manual_seed(self, s):
            return self

    class Tensor:
        def __init__(self, shape):
            self.shape = tuple(shape)
            n = 1
            for d in self.shape:
                n *= d
            p = ctypes.c_void_p()
            assert fake.hipMalloc(ctypes.byref(p), max(4, 4 * n)) == 0
            self.ptr = p.value
            st, acc = [], 1
            for d in reversed(self.shape):
                st.append(acc)
                acc *= d
            self._stride = tuple(reversed(st))

        def data_ptr(self):
            return self.ptr

        def dim(self):
            return len(self.shape)

        def stride(self, i=None):
            return self._stride if i is None else self._stride[i]

        def unsqueeze(self, i):
            assert i == 0
            u = Tensor.__new__(Tensor)
            u.shape, u.ptr, u._stride = (1,) + self.shape, self.ptr, (self.shape[0] * self._stride[0],) + self._stride
            return u

    class Stream:
        def __init__(self, handle=None):
            if handle is None:
                h = ctypes.c_void_p()
                assert fake.hipStreamCreateWithFlags(ctypes.byref(h), 1) == 0
                handle = h.value or 0
            self.cuda_stream = handle

        def wait_event(self, ev):
            assert fake.hipStreamWaitEvent(self.cuda_stream, ev.h, 0) == 0

    class Event:
        def __init__(self, *a, **k):
            h = ctypes.c_void_p()
            assert fake.hipEventCreate(ctypes.byref(h)) == 0
            self.h = h.value

        def record(self, stream=None):
            s = stream if stream is not None else cuda.current_stream()
            assert fake.hipEventRecord(self.h, s.cuda_stream) == 0

        def query(self):
            return fake.hipEventQuery(self.h) == 0

    null = Stream(0)

    class _StreamCtx:
        def __init__(self, s):
            self.s = s

        def __enter__(self):
            return self.s

        def __exit__(self, *e):
            return False

    cuda = types.SimpleNamespace(
        Stream=Stream, Event=Event, current_stream=lambda: null, stream=_StreamCtx,
        synchronize=lambda: fake.fakehip_drain(), is_available=lambda: True)
    t.cuda = cuda
    t.device = device
    t.Generator = Generator
    t.Tensor = Tensor
    t.empty = lambda shape, dtype=None, device=None: Tensor(shape)
    t.randint = lambda lo, hi, shape, dtype=None, device=None, generator=None: Tensor(shape)
    return t


def scenario(name, fake, torch, fntrs):
    """A small sequence with a known verdict, to show the checker sees what it
    should: *_ok ones are correctly ordered, the others are not."""
    import numpy as np
    ctx = fntrs.Context(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    n, k, lanes = 512, 256, 64
    a = torch.empty((1, k, lanes))
    b = torch.empty((1, n, lanes))
    c = torch.empty((1, 2 * n, lanes))
    if name in ("encode_chain_ok", "encode_chain_race"):
        # b = encode(a) on s1; c = encode(b's first k rows) on s2
        ctx.encode(a, b, n, stream=s1)
        if name == "encode_chain_ok":
            ev = torch.cuda.Event()
            ev.record(s1)
            s2.wait_event(ev)
        bk = torch.Tensor.__new__(torch.Tensor)
        bk.shape, bk.ptr, bk._stride = (1, n, lanes), b.ptr, b._stride
        ctx.encode(bk, c, 2 * n, stream=s2)
    elif name == "decode_other_stream_ok":
        # a locator built on s1 and used on s2: the library orders them
        z = np.arange(0, n, 2, dtype=np.uint32)
        loc = ctx.locator(n, k, z, stream=s1)
        out = torch.empty((1, k, lanes))
        ctx.decode(loc, b, out, fntrs.FNTRS_RECV_FULL, stream=s2)
        fake.fakehip_drain()
        loc.release()
    elif name == "large_locator_ok":
        # one large pattern (the logarithmic route: a table built on first
        # use, transforms through scratch) on s1, decoded on s2, twice
        # (its coefficients are taken on first use: by the export, or by
        # the direct decoder on s2)
        N = 16384
        for rep, K in enumerate((4096, 1024)):
            z = np.arange(rep, N, 3, dtype=np.uint32)[:K]
            loc = ctx.locator(N, K, z, stream=s1)
            recv = torch.empty((1, N, 32))
            out = torch.empty((1, K, 32))
            ctx.decode(loc, recv, out, fntrs.FNTRS_RECV_FULL, stream=s2)
            if rep == 0:
                loc.export()
            else:
                ctx.decode(loc, recv, out, fntrs.FNTRS_RECV_FULL | fntrs.FNTRS_DIRECT, stream=s2)
            fake.fakehip_drain()
            loc.release()
    elif name == "direct_ok":
        # the direct methods' matrices are built on one stream and used on another
        z = np.arange(1, n, 2, dtype=np.uint32)[:k]
        loc = ctx.locator(n, k, z, stream=s1)
        outs = [torch.empty((1, k, lanes)) for _ in range(4)]
        ctx.decode(loc, b, outs[0], fntrs.FNTRS_RECV_FULL | fntrs.FNTRS_DIRECT, stream=s1)
        ctx.decode(loc, b, outs[1], fntrs.FNTRS_RECV_FULL | fntrs.FNTRS_DIRECT, stream=s2)
        ctx.decode(loc, b, outs[2], fntrs.FNTRS_RECV_FULL | fntrs.FNTRS_DIRECT | fntrs.FNTRS_SYSTEMATIC, stream=s1)
        ctx.decode(loc, b, outs[3], fntrs.FNTRS_RECV_FULL | fntrs.FNTRS_DIRECT | fntrs.FNTRS_SYSTEMATIC, stream=s2)
        encs = [torch.empty((1, n, lanes)) for _ in range(3)]
        ctx.encode(a, encs[0], n, flags=fntrs.FNTRS_DIRECT, stream=s1)
        ctx.encode(a, encs[1], n, flags=fntrs.FNTRS_DIRECT | fntrs.FNTRS_SYSTEMATIC, stream=s2)
        ctx.encode(a, encs[2], n, flags=fntrs.FNTRS_DIRECT | fntrs.FNTRS_SYSTEMATIC, stream=s1)
        fake.fakehip_drain()
        loc.release()
    elif name == "out_of_bounds":
        fake.hipMemsetAsync.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
        fake.hipMemsetAsync(a.ptr, 0, 4 * k * lanes + 4, s1.cuda_stream)
    elif name == "use_after_free":
        fake.hipMallocAsync.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_void_p]
        fake.hipFreeAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        fake.hipMemsetAsync.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
        p = ctypes.c_void_p()
        fake.hipMallocAsync(ctypes.byref(p), 4096, s1.cuda_stream)
        fake.hipFreeAsync(p, s1.cuda_stream)
        ev = torch.cuda.Event()
        ev.record(s1)
        s2.wait_event(ev)
        fake.hipMemsetAsync(p, 0, 4096, s2.cuda_stream)
    elif name == "pinned_reuse":
        fake.hipHostMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
        fake.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
        h = ctypes.c_void_p()
        fake.hipHostMalloc(ctypes.byref(h), 4096, 0)
        ctypes.memset(h, 1, 4096)
        fake.fakehip_set_lag(1.0)                 # the device stays behind
        fake.hipMemcpyAsync(a.ptr, h, 4096, 1, s1.cuda_stream)
        ctypes.memset(h, 2, 4096)                 # reused before the copy ran
    else:
        raise SystemExit(f"unknown scenario {name}")
    fake.fakehip_drain()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scenario", default=None, help="run one checker self-test sequence instead of the replay")
    ap.add_argument("--fake", required=True, help="path of the built checker (libamdhip64.so.7)")
    ap.add_argument("--seed", type=int, default=1, help="checker scheduling seed")
    ap.add_argument("--lag", type=float, default=0.7, help="probability that a host call leaves the device idle")
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--pattern-pool", type=int, default=16, help="patterns per code (0: a fresh one per decode)")
    ap.add_argument("--span-s", type=float, default=0.0, help="arrivals spread over this many seconds (0: closed loop)")
    ap.add_argument("--ctx-cap-mib", type=int, default=8192, help="context workspace cap (locator cache)")
    ap.add_argument("--pool", type=int, default=64, help="resident codewords")
    ap.add_argument("--max-inflight", type=int, default=4)
    ap.add_argument("--bench-seed", type=int, default=2024)
    args = ap.parse_args()

    fake = load(args.fake)
    fake.fakehip_seed(args.seed)
    fake.fakehip_set_lag(args.lag)
    torch = fake_torch(fake)
    sys.modules["torch"] = torch
    sys.path.insert(0, ROOT)
    import numpy as np

    from paper_0907_1788_amd import fntrs, serve, synth
    L = ctypes.CDLL(fntrs.LIB_PATH)
    for name, (res, argt) in fntrs.SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = argt
    fntrs._lib = L
    if args.scenario:
        scenario(args.scenario, fake, torch, fntrs)
        errs = [fake.fakehip_error_text(i).decode() for i in range(fake.fakehip_errors())]
        print(json.dumps({"errors": errs}), flush=True)
        return
    import bench

    ctx = fntrs.Context(0, workspace_cap_bytes=args.ctx_cap_mib << 20)
    pool = bench.served_pool(torch, ctx, synth, args.bench_seed, count=args.pool)
    fake.fakehip_drain()
    rng = np.random.default_rng(args.bench_seed)
    if args.span_s > 0:
        arrivals = serve.poisson_arrivals(args.requests / args.span_s, args.requests, args.bench_seed + 999)
    else:
        arrivals = np.zeros(args.requests)
    reqs = bench.served_requests(serve, pool, rng, args.requests, arrivals, args.pattern_pool)
    srv = serve.Server(ctx, mem_cap_bytes=32 << 30, max_inflight=args.max_inflight)
    st = srv.run(reqs, keep=lambda r: False)
    fake.fakehip_drain()
    ctx.close()
    ops, kernels, checks = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    fake.fakehip_stats(ctypes.byref(ops), ctypes.byref(kernels), ctypes.byref(checks))
    nm, nma, nw = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    fake.fakehip_alloc_stats(ctypes.byref(nm), ctypes.byref(nma), ctypes.byref(nw))
    errs = [fake.fakehip_error_text(i).decode() for i in range(fake.fakehip_errors())]
    print(json.dumps({"errors": errs, "requests": st.completed, "batches": st.batches,
                      "peak_inflight": st.peak_inflight, "ops": ops.value, "kernels": kernels.value,
                      "checks": checks.value, "hipMalloc": nm.value, "hipMallocAsync": nma.value,
                      "hipStreamWaitEvent": nw.value}), flush=True)


if __name__ == "__main__":
    main()

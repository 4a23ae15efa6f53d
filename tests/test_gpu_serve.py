"""The continuous-batching server on the GPU.

Each request's result must be the same whether it is served alone or in the
mix (bit-exact: integer arithmetic modulo 65537 with a unique result,
Sec. II-B), decode requests must return their source, encode requests must
match the oracle on sampled rows, admission must respect the memory cap, and
batches must overlap on the device.
"""
import numpy as np
import pytest

from oracle import codec
from paper_0907_1788_amd import fntrs, serve, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = fntrs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int32)).cuda()


def make_pool(ctx, count, seed):
    """Codewords of the uneven-batch size distribution (lanes scaled down): source and encoded rows."""
    pool = []
    for i, (k, n, lanes) in enumerate(synth.uneven_batch(seed, 4 * count)):
        if k > 4096:
            continue
        lanes = max(1, lanes // 64)
        src = synth.source(seed * 1000 + i, 1, k, lanes)
        s = dev(src)
        e = torch.empty((1, n, lanes), dtype=torch.int32, device="cuda")
        ctx.encode(s, e, n)
        pool.append((k, n, lanes, src, s, e))
        if len(pool) == count:
            break
    # one maximum-length code (four-step decode)
    k, n, lanes = 16384, 65536, 6
    src = synth.source(seed * 1000 + 999, 1, k, lanes)
    s = dev(src)
    e = torch.empty((1, n, lanes), dtype=torch.int32, device="cuda")
    ctx.encode(s, e, n)
    pool.append((k, n, lanes, src, s, e))
    torch.cuda.synchronize()
    return pool


def make_requests(pool, count, seed, rate):
    rng = np.random.default_rng(seed)
    arrivals = serve.poisson_arrivals(rate, count, seed)
    reqs = []
    for i in range(count):
        k, n, lanes, src, s, e = pool[int(rng.integers(len(pool)))]
        if rng.random() < 0.6:
            r = serve.Request(serve.ENCODE, n, k, lanes, s)
        else:
            # own pattern, or one of 3 shared patterns of this code (locator cache)
            pseed = int(rng.integers(1 << 30)) if rng.random() < 0.5 else 77 + int(rng.integers(3)) + n
            z = synth.received_positions(pseed, n, k)
            compact = bool(rng.random() < 0.3)
            inp = e.index_select(1, torch.from_numpy(z.astype(np.int64)).cuda()).contiguous() if compact else e
            r = serve.Request(serve.DECODE, n, k, lanes, inp, positions=z, compact=compact)
            r.src_ref = src
        r.arrival = float(arrivals[i])
        r.rid = i
        r.pool_src = s
        reqs.append(r)
    torch.cuda.synchronize()
    return reqs


def solo(ctx, r):
    """The request computed alone, through the single calls."""
    if r.op == serve.ENCODE:
        out = torch.empty((1, r.n, r.lanes), dtype=torch.int32, device="cuda")
        ctx.encode(r.inp, out, r.n)
    else:
        loc = ctx.locator(r.n, r.k, r.positions)
        out = torch.empty((1, r.k, r.lanes), dtype=torch.int32, device="cuda")
        ctx.decode(loc, r.inp, out, fntrs.FNTRS_RECV_COMPACT if r.compact else fntrs.FNTRS_RECV_FULL)
        torch.cuda.synchronize()
        loc.release()
    torch.cuda.synchronize()
    return out


def test_served_results_equal_solo_results(ctx):
    pool = make_pool(ctx, 20, seed=11)
    reqs = make_requests(pool, 150, seed=12, rate=3000.0)
    say("serve", len(reqs), "requests")
    cap = max(r.device_bytes() for r in reqs) * 6
    srv = serve.Server(ctx, mem_cap_bytes=cap, max_inflight=3, max_batch=12)
    st = srv.run(reqs)
    assert st.completed == len(reqs)
    assert st.peak_bytes <= cap
    assert st.peak_inflight >= 2, "batches never overlapped"
    assert all(np.isfinite(r.t_done) and r.t_done >= r.arrival for r in reqs)
    for r in reqs:
        assert torch.equal(r.out, solo(ctx, r)), ("mix vs alone", r.rid, r.op, r.n, r.k, r.lanes)
        if r.op == serve.DECODE:
            assert np.array_equal(r.out.cpu().numpy().astype(np.int64), r.src_ref.astype(np.int64)), r.rid
    # a few encode requests against the oracle on sampled rows
    checked = 0
    for r in reqs:
        if r.op == serve.ENCODE and checked < 5:
            rows = np.unique((synth.stream(r.rid, 5) % np.uint64(r.n)).astype(np.int64))
            src = r.pool_src.cpu().numpy().astype(np.int64)[0]
            got = r.out.cpu().numpy().astype(np.int64)[0][rows][:, :1]
            assert np.array_equal(got, codec.encode(src[:, :1], r.n, rows=rows))
            checked += 1


def test_tuned_server_results_equal_default_results(ctx):
    """Server.autotune keeps the fastest configuration of each size class in
    its context; the outputs stay those of the default configurations."""
    tctx = fntrs.Context(0)
    try:
        pool = make_pool(tctx, 12, seed=31)
        reqs = make_requests(pool, 60, seed=32, rate=5000.0)
        say("tuned serve", len(reqs), "requests")
        srv = serve.Server(tctx, mem_cap_bytes=max(r.device_bytes() for r in reqs) * 6, max_inflight=3)
        classes = srv.autotune(reqs[:30])
        assert classes and all(c["ms"] > 0 for c in classes)
        st = srv.run(reqs)
        assert st.completed == len(reqs)
        for r in reqs:
            assert torch.equal(r.out, solo(ctx, r)), ("tuned vs default", r.rid, r.op, r.n, r.k, r.lanes)
    finally:
        torch.cuda.synchronize()
        tctx.close()


def test_admission_rejects_oversized_request(ctx):
    s = torch.zeros((1, 64, 4), dtype=torch.int32, device="cuda")
    r = serve.Request(serve.ENCODE, 128, 64, 4, s)
    srv = serve.Server(ctx, mem_cap_bytes=r.device_bytes() - 1, max_inflight=1)
    with pytest.raises(ValueError):
        srv.run([r])


def test_burst_under_tight_cap_serialises_but_completes(ctx):
    pool = make_pool(ctx, 6, seed=21)
    reqs = make_requests(pool, 40, seed=22, rate=1e9)       # everything arrives at once
    cap = max(r.device_bytes() for r in reqs)               # one request at a time at worst
    st = serve.Server(ctx, mem_cap_bytes=cap, max_inflight=4, max_batch=64).run(reqs)
    assert st.completed == len(reqs) and st.peak_bytes <= cap
    for r in reqs:
        assert torch.equal(r.out, solo(ctx, r)), r.rid

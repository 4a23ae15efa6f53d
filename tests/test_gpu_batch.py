"""The batched path (fntrs_submit, captured graphs, autotuner) on the GPU.

A batch must compute exactly what its jobs compute one call at a time: every
output is compared with the single-call path element by element, decoding
must return the source on every lane (unique interpolant, Sec. II-B), and
sampled rows / lanes are checked against the CPU oracle.  Sizes follow the
uneven-batch workload (k = 2^6..2^14, rate 1/2 or 1/4, uneven lane counts,
one erasure pattern per codeword), scaled down in lanes so the oracle checks
stay fast.
"""
import numpy as np
import pytest

from oracle import codec
from paper_0907_1788_amd import fntrs, synth

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


def host(t):
    return t.cpu().numpy().astype(np.int64)


class Codeword:
    """One codeword block set of the batch: source, encoded, received, decoded buffers."""

    def __init__(self, ctx, i, k, n, lanes, blocks=1, seed=0, full=False):
        self.k, self.n, self.lanes, self.blocks, self.full = k, n, lanes, blocks, full
        self.src_np = synth.source(seed * 100003 + i, blocks, k, lanes)
        self.src = dev(self.src_np)
        self.enc = torch.full((blocks, n, lanes), -7, dtype=torch.int32, device="cuda")
        self.z = synth.received_positions(seed * 7919 + i, n, k)
        self.loc = ctx.locator(n, k, self.z)
        self.dec = torch.full((blocks, k, lanes), -7, dtype=torch.int32, device="cuda")
        self.recv = None

    def make_recv(self):
        """Received rows (compact) from the encoded buffer, or the full buffer itself."""
        if self.full:
            self.recv = self.enc
        else:
            idx = torch.from_numpy(self.z.astype(np.int64)).cuda()
            self.recv = self.enc.index_select(1, idx).contiguous()

    def dec_flags(self):
        return fntrs.FNTRS_RECV_FULL if self.full else fntrs.FNTRS_RECV_COMPACT


def build_batch(ctx, sizes, seed, blocks=1):
    return [Codeword(ctx, i, k, n, lanes, blocks, seed, full=(i % 3 == 0)) for i, (k, n, lanes) in enumerate(sizes)]


def check_against_singles(ctx, cws):
    """Batch outputs equal the single calls' outputs, bit for bit."""
    for cw in cws:
        e = torch.empty_like(cw.enc)
        ctx.encode(cw.src, e, cw.n)
        d = torch.empty_like(cw.dec)
        ctx.decode(cw.loc, cw.recv, d, cw.dec_flags())
        torch.cuda.synchronize()
        assert torch.equal(e, cw.enc), ("encode", cw.k, cw.n, cw.lanes)
        assert torch.equal(d, cw.dec), ("decode", cw.k, cw.n, cw.lanes)


def check_against_oracle(cws, lanes_checked=2):
    for cw in cws:
        # every lane decodes back to its source (P14)
        assert np.array_equal(host(cw.dec), cw.src_np.astype(np.int64)), ("roundtrip", cw.k, cw.n, cw.lanes)
        # sampled encoded rows against the oracle's Horner evaluation
        rows = np.unique(np.concatenate([[0, 1 % cw.n, cw.n - 1], synth.stream(cw.n + cw.k, 6) % np.uint64(cw.n)])
                         .astype(np.int64))
        lanes = [0, cw.lanes - 1][:lanes_checked]
        got = host(cw.enc)[0][rows][:, lanes]
        ref = codec.encode(cw.src_np[0][:, lanes], cw.n, rows=rows)
        assert np.array_equal(got, ref), ("encode rows", cw.k, cw.n)


def small_uneven(seed, count, max_lanes, max_k):
    out = []
    for k, n, lanes in synth.uneven_batch(seed, 4 * count):
        if k <= max_k:
            out.append((k, n, max(1, lanes * max_lanes // 8192)))
        if len(out) == count:
            break
    return out


def run_submit(ctx, cws):
    ctx.submit([ctx.encode_job(cw.src, cw.enc, cw.n) for cw in cws])
    for cw in cws:
        cw.make_recv()
    ctx.submit([ctx.decode_job(cw.loc, cw.recv, cw.dec, cw.dec_flags()) for cw in cws])
    torch.cuda.synchronize()


def test_submit_uneven_batch(ctx):
    sizes = small_uneven(seed=4, count=40, max_lanes=300, max_k=4096)
    # ragged and tiny codes, k = n, a non-power-of-two encode size
    sizes += [(1, 1, 5), (2, 2, 7), (64, 64, 33), (4, 256, 3), (1024, 2048, 130)]
    say("submit uneven", len(sizes), "codewords")
    cws = build_batch(ctx, sizes, seed=1)
    run_submit(ctx, cws)
    check_against_oracle(cws)
    check_against_singles(ctx, cws)
    for cw in cws:
        cw.loc.release()


def test_submit_full_range_sizes(ctx):
    """The workload's largest codes: k = 16384 at rate 1/4 (n = 65536, four-step decode) and rate 1/2."""
    sizes = [(16384, 65536, 40), (16384, 32768, 37), (8192, 32768, 16), (64, 128, 1000), (128, 512, 9)]
    say("submit full range", sizes)
    cws = build_batch(ctx, sizes, seed=2)
    run_submit(ctx, cws)
    check_against_oracle(cws, lanes_checked=1)
    check_against_singles(ctx, cws)
    for cw in cws:
        cw.loc.release()


def test_submit_persistent_loop(ctx):
    """Classes with many more work items than resident workgroups, several blocks per job."""
    sizes = [(256, 512, 2048), (256, 1024, 1500), (512, 1024, 777)]
    say("submit persistent", sizes)
    cws = build_batch(ctx, sizes, seed=3, blocks=6)
    run_submit(ctx, cws)
    for cw in cws:
        assert np.array_equal(host(cw.dec), cw.src_np.astype(np.int64))
    check_against_singles(ctx, cws)
    for cw in cws:
        cw.loc.release()


def test_submit_decodes_arbitrary_received_values(ctx):
    """Non-codeword received data: the exact interpolant, against the Lagrange oracle."""
    specs = [(64, 128, 5), (256, 1024, 3), (512, 1024, 4)]
    jobs, outs, refs, locs = [], [], [], []
    for i, (k, n, lanes) in enumerate(specs):
        z = synth.received_positions(500 + i, n, k)
        loc = ctx.locator(n, k, z)
        rnd = synth.residues(600 + i, (1, k, lanes))
        r = dev(rnd)
        d = torch.full((1, k, lanes), -7, dtype=torch.int32, device="cuda")
        jobs.append(ctx.decode_job(loc, r, d))
        outs.append((r, d))
        refs.append(codec.decode_lagrange(n, z, rnd[0]))
        locs.append(loc)
    ctx.submit(jobs)
    torch.cuda.synchronize()
    for (r, d), ref in zip(outs, refs):
        assert np.array_equal(host(d)[0], ref)
    for loc in locs:
        loc.release()


def test_graph_replays_match_eager(ctx):
    """A captured batch replayed several times, with new inputs and eager work between replays."""
    sizes = small_uneven(seed=9, count=12, max_lanes=200, max_k=2048) + [(16384, 65536, 8)]
    say("graph", len(sizes))
    cws = build_batch(ctx, sizes, seed=4)
    # encode graph, then decode graph over the received rows
    g_enc = ctx.graph([ctx.encode_job(cw.src, cw.enc, cw.n) for cw in cws])
    compact = [cw for cw in cws if not cw.full]
    for cw in compact:
        cw.recv = torch.zeros((cw.blocks, cw.k, cw.lanes), dtype=torch.int32, device="cuda")
    for cw in cws:
        if cw.full:
            cw.recv = cw.enc
    g_dec = ctx.graph([ctx.decode_job(cw.loc, cw.recv, cw.dec, cw.dec_flags()) for cw in cws])
    for rep in range(3):
        for cw in cws:
            cw.src_np = synth.source(7000 + 31 * rep + cw.k + cw.lanes, cw.blocks, cw.k, cw.lanes)
            cw.src.copy_(dev(cw.src_np))
        g_enc.launch()
        torch.cuda.synchronize()
        for cw in compact:
            idx = torch.from_numpy(cw.z.astype(np.int64)).cuda()
            cw.recv.copy_(cw.enc.index_select(1, idx))
        g_dec.launch()
        torch.cuda.synchronize()
        for cw in cws:
            assert np.array_equal(host(cw.dec), cw.src_np.astype(np.int64)), ("replay", rep, cw.k, cw.n)
        check_against_singles(ctx, cws)
    g_enc.destroy()
    g_dec.destroy()
    for cw in cws:
        cw.loc.release()


def test_autotune_keeps_results_exact(ctx):
    """The tuner picks one of the compiled configurations; results stay bit-exact under it."""
    from paper_0907_1788_amd.fntrs import FNTRS_OP_DECODE, FNTRS_OP_ENCODE
    say("autotune")
    for op, n, k in [(FNTRS_OP_ENCODE, 8192, 4096), (FNTRS_OP_DECODE, 8192, 4096), (FNTRS_OP_DECODE, 4096, 2048)]:
        t = ctx.autotune(op, n, k, lanes=512, batch=2, reps=2)
        assert t["ms"] > 0 and t["tile_lanes"] >= 1 and t["threads"] in (256, 512, 1024)
        L = (k - 1).bit_length() if op == FNTRS_OP_ENCODE else n.bit_length() - 1
        assert ctx.config(op, L)["tile_lanes"] == t["tile_lanes"]
    cws = build_batch(ctx, [(4096, 8192, 70), (2048, 4096, 9)], seed=5)
    run_submit(ctx, cws)
    check_against_oracle(cws, lanes_checked=1)
    check_against_singles(ctx, cws)
    for cw in cws:
        cw.loc.release()


def test_autotune_covers_every_size_and_the_direct_methods():
    """Four-step classes (2^14 points and more) are timed, any k decodes, and
    for small codes the direct methods compete; whichever wins, single calls
    stay bit-exact (their outputs are unique)."""
    from paper_0907_1788_amd.fntrs import FNTRS_OP_DECODE, FNTRS_OP_ENCODE
    with fntrs.Context(0) as c:
        for op, n, k, lanes in [(FNTRS_OP_ENCODE, 65536, 16384, 64), (FNTRS_OP_DECODE, 65536, 16384, 64),
                                (FNTRS_OP_DECODE, 32768, 9000, 32), (FNTRS_OP_DECODE, 8192, 3000, 64),
                                (FNTRS_OP_ENCODE, 128, 64, 256), (FNTRS_OP_DECODE, 128, 64, 256),
                                (FNTRS_OP_ENCODE, 512, 200, 512), (FNTRS_OP_DECODE, 512, 256, 512)]:
            say("autotune", op, n, k, lanes)
            t = c.autotune(op, n, k, lanes=lanes, batch=1, reps=3)
            assert t["ms"] > 0 and t["default_ms"] > 0
            if n >= 16384 and (op == FNTRS_OP_DECODE or k > 8192):
                assert t["method"] == "four-step"
            else:
                assert t["method"] in ("transform", "direct")
        # single calls after tuning, whatever method the tuner chose
        for n, k, lanes in [(128, 64, 256), (512, 200, 512), (512, 256, 512)]:
            src = synth.source(1300 + n, 1, k, lanes)
            e = torch.empty((1, n, lanes), dtype=torch.int32, device="cuda")
            c.encode(dev(src), e, n)
            torch.cuda.synchronize()
            rows = np.array([0, 1, n // 2, n - 1])
            assert np.array_equal(host(e)[0][rows][:, :2], codec.encode(src[0][:, :2].astype(np.int64), n, rows=rows))
            z = synth.received_positions(1400 + n, n, k)
            loc = c.locator(n, k, z)
            d = torch.empty((1, k, lanes), dtype=torch.int32, device="cuda")
            c.decode(loc, e, d, fntrs.FNTRS_RECV_FULL)
            torch.cuda.synchronize()
            assert np.array_equal(host(d), src.astype(np.int64))
            loc.release()


def test_autotune_batch_tunes_each_class_and_keeps_results_exact():
    with fntrs.Context(0) as c:
        cws = build_batch(c, [(4096, 8192, 70), (2048, 4096, 9), (256, 512, 300), (16384, 65536, 40),
                              (1000, 4096, 33)], seed=6)
        enc_jobs = [c.encode_job(cw.src, cw.enc, cw.n) for cw in cws]
        ts = c.autotune_batch(enc_jobs, reps=2)
        assert {(t["op"], t["log2_size"]) for t in ts} == {("encode", 12), ("encode", 11), ("encode", 8),
                                                           ("encode", 14), ("encode", 10)}
        assert all(t["ms"] > 0 for t in ts)
        for t in ts:
            if t["method"] == "transform":
                assert c.config(fntrs.FNTRS_OP_ENCODE, t["log2_size"])["tile_lanes"] == t["tile_lanes"]
        run_submit(c, cws)
        dec_jobs = [c.decode_job(cw.loc, cw.recv, cw.dec, cw.dec_flags()) for cw in cws]
        ts = c.autotune_batch(dec_jobs, reps=2)
        assert {t["log2_size"] for t in ts} == {13, 12, 9, 16}
        run_submit(c, cws)
        check_against_oracle(cws, lanes_checked=1)
        check_against_singles(c, cws)
        for cw in cws:
            cw.loc.release()


def test_locator_batch_state_matches_oracle(ctx):
    """Patterns built together (mixed n and k, nothing erased, k = 1, repeats) equal the oracle's locators."""
    specs = [(16, 4, 1), (64, 64, 0), (128, 1, 2), (256, 64, 3), (512, 256, 4), (1024, 128, 5), (2048, 1024, 6),
             (256, 64, 3), (4096, 2048, 7), (8192, 4096, 8), (65536, 16384, 9), (64, 32, 10), (2, 1, 11)]
    pats = []
    for n, k, seed in specs:
        z = np.arange(n, dtype=np.uint32) if k == n else synth.received_positions(900 + seed, n, k)
        pats.append((n, k, z))
    say("locator batch", len(pats))
    locs = ctx.locators(pats)
    assert locs[3].handle == locs[7].handle           # the repeated pattern is built once
    for (n, k, z), loc in zip(pats, locs):
        A, w, ahat = loc.export()
        ref = codec.locator(n, z, with_w=(k <= 4096 and k < n))
        assert np.array_equal(A.astype(np.int64), ref["A"]), (n, k)
        if k < n:
            if "w" in ref:
                assert np.array_equal(w.astype(np.int64), ref["w"]), (n, k)
            assert np.array_equal(ahat.astype(np.int64), ref["Ahat"]), (n, k)
    # cache hits on a second batch, and decoding through batch-built locators
    again = ctx.locators(pats[:4])
    assert [a.handle for a in again] == [b.handle for b in locs[:4]]
    for (n, k, z), loc in zip(pats, locs):
        lanes = 3
        src = synth.source(1000 + n + k, 1, k, lanes)
        e = torch.empty((1, n, lanes), dtype=torch.int32, device="cuda")
        ctx.encode(dev(src), e, n)
        d = torch.empty((1, k, lanes), dtype=torch.int32, device="cuda")
        ctx.decode(loc, e, d, fntrs.FNTRS_RECV_FULL)
        torch.cuda.synchronize()
        assert np.array_equal(host(d), src.astype(np.int64)), (n, k)
    for x in locs + again:
        x.release()

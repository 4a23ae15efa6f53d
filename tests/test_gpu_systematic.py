"""The systematic code (Sec. II-C) on the GPU, through the C ABI flag.

Encode: the source interpolated on positions 0..k-1 gives the intermediate
symbols, whose transform is the codeword (first k rows = source).  Decode:
the intermediate symbols from any k received symbols, transformed at the
first k positions.  Everything is integer arithmetic modulo 65537 with a
unique result, so every comparison with the oracle is exact.
"""
import numpy as np
import pytest

from oracle import codec
from paper_0907_1788_amd import fntrs, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S = fntrs.FNTRS_SYSTEMATIC


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


def sys_encode(ctx, src, n, pad=0):
    b, k, lanes = src.shape
    s = torch.zeros((b, k, lanes + pad), dtype=torch.int32, device="cuda")
    s[:, :, :lanes] = dev(src)
    e = torch.full((b, n, lanes + pad), -7, dtype=torch.int32, device="cuda")
    ctx.encode(s[:, :, :lanes], e[:, :, :lanes], n, flags=S)
    torch.cuda.synchronize()
    out = host(e)
    if pad:
        assert np.all(out[:, :, lanes:] == -7), "encode wrote outside its lanes"
    return out[:, :, :lanes]


def sys_decode(ctx, loc, recv, flags):
    b, _, lanes = recv.shape
    d = torch.full((b, loc.k, lanes), -7, dtype=torch.int32, device="cuda")
    ctx.decode(loc, dev(recv), d, flags | S)
    torch.cuda.synchronize()
    return host(d)


# n, k, lanes, batch; the oracle checks every row up to the first bound,
# sampled rows beyond
CASES = [(2, 1, 3, 1), (4, 2, 5, 2), (8, 4, 9, 1), (64, 32, 33, 1), (64, 64, 4, 1), (512, 256, 65, 2),
         (8, 3, 4, 1), (512, 200, 9, 1), (8192, 3000, 3, 1),
         (1024, 128, 7, 1), (2048, 1024, 6, 1), (8192, 4096, 5, 1), (16384, 8192, 3, 1), (65536, 16384, 2, 1)]


@pytest.mark.parametrize("n,k,lanes,batch", CASES)
def test_systematic_encode_matches_oracle(ctx, n, k, lanes, batch):
    say("systematic encode", n, k, lanes, batch)
    src = synth.residues(5000 + n + k, (batch, k, lanes))
    out = sys_encode(ctx, src, n, pad=2)
    # P16 on every lane: the first k positions are the source
    assert np.array_equal(out[:, :k], src.astype(np.int64))
    if n * k <= 2 ** 21:
        rows = None
    else:
        rows = np.unique(np.concatenate([[0, k - 1, k, n - 1], synth.stream(n + 3, 10) % np.uint64(n)])
                         .astype(np.int64))
    for b in range(batch):
        lanes_chk = [0, lanes - 1] if rows is not None else list(range(lanes))
        ref = codec.systematic_encode(src[b][:, lanes_chk], n, rows=rows)
        got = out[b][:, lanes_chk] if rows is None else out[b][rows][:, lanes_chk]
        assert np.array_equal(got, ref), b


@pytest.mark.parametrize("n,k,lanes", [(8, 4, 3), (256, 64, 17), (1024, 512, 9), (8192, 4096, 12),
                                       (16384, 4096, 5), (65536, 16384, 33), (512, 512, 4)])
def test_systematic_decode_roundtrip(ctx, n, k, lanes):
    """Every lane comes back from a random pattern, compact and full reception."""
    say("systematic roundtrip", n, k, lanes)
    src = synth.source(5100 + n + k, 2, k, lanes)
    e = sys_encode(ctx, src, n)
    z = synth.received_positions(5200 + n, n, k) if k < n else np.arange(n, dtype=np.uint32)
    loc = ctx.locator(n, k, z)
    assert np.array_equal(sys_decode(ctx, loc, e[:, z, :], fntrs.FNTRS_RECV_COMPACT), src.astype(np.int64))
    assert np.array_equal(sys_decode(ctx, loc, e, fntrs.FNTRS_RECV_FULL), src.astype(np.int64))
    loc.release()


@pytest.mark.parametrize("n,k", [(16, 4), (128, 32), (1024, 256)])
def test_systematic_decode_of_arbitrary_values_matches_oracle(ctx, n, k):
    """Received values that are not a codeword: the oracle's systematic decoder."""
    say("systematic decode arbitrary", n, k)
    z = synth.received_positions(5300 + n, n, k)
    v = synth.residues(5400 + n, (1, k, 6))
    loc = ctx.locator(n, k, z)
    got = sys_decode(ctx, loc, v, fntrs.FNTRS_RECV_COMPACT)[0]
    assert np.array_equal(got, codec.systematic_decode(n, z, v[0]))
    loc.release()


def test_systematic_identity_and_repeat_calls(ctx):
    """k = n is the identity (P17); a second call reuses the cached pattern of
    the first k positions and must give the same codeword."""
    say("systematic k = n, repeat")
    src = synth.residues(5500, (1, 256, 8))
    assert np.array_equal(sys_encode(ctx, src, 256), src.astype(np.int64))
    s2 = synth.residues(5501, (3, 64, 40))
    a = sys_encode(ctx, s2, 512)
    b = sys_encode(ctx, s2, 512)
    assert np.array_equal(a, b)
    # the systematic codeword is a codeword of the plain code: plain decoding
    # of any k symbols and plain encoding give it back
    z = synth.received_positions(5502, 512, 64)
    loc = ctx.locator(512, 64, z)
    d = torch.empty((3, 64, 40), dtype=torch.int32, device="cuda")
    ctx.decode(loc, dev(a[:, z, :]), d, fntrs.FNTRS_RECV_COMPACT)
    e = torch.empty((3, 512, 40), dtype=torch.int32, device="cuda")
    ctx.encode(d, e, 512)
    torch.cuda.synchronize()
    assert np.array_equal(host(e), a)
    loc.release()

"""The no-allocation encoder (fntrs_encode_noalloc) against fntrs_encode.

The entry point takes the arguments of fntrs_encode and must give the same
codeword bit for bit while allocating nothing: the four-step encoder
(transforms of 2^14 points or more) runs through the library's fixed device
scratch.  Two calls in a row, the second on a smaller input, so that the
second reads a scratch the first has left full of its own rows; then a short
code (no scratch) and the host-side rejection of a size beyond the scratch.
"""
import numpy as np
import pytest

from paper_0907_1788_amd import fntrs, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int32)).cuda()


def both(ctx, n, k, lanes, batch, seed, ld_pad=0):
    """dst of fntrs_encode and of fntrs_encode_noalloc on the same source."""
    src = dev(synth.source(seed, batch, k, lanes + ld_pad))
    out_ref = torch.full((batch, n, lanes + ld_pad), -7, dtype=torch.int32, device="cuda")
    out_na = torch.full((batch, n, lanes + ld_pad), -7, dtype=torch.int32, device="cuda")
    ld, st_s, st_d = lanes + ld_pad, k * (lanes + ld_pad), n * (lanes + ld_pad)
    stream = torch.cuda.current_stream().cuda_stream
    h = ctx.handle
    rc = fntrs.fntrs_encode(h, n, k, lanes, src.data_ptr(), ld, st_s, out_ref.data_ptr(), ld, st_d, batch, 0, stream)
    assert rc == fntrs.FNTRS_OK, fntrs.fntrs_last_error(h)
    rc = fntrs.fntrs_encode_noalloc(h, n, k, lanes, src.data_ptr(), ld, st_s, out_na.data_ptr(), ld, st_d, batch, 0,
                                    stream)
    assert rc == fntrs.FNTRS_OK, fntrs.fntrs_last_error(h)
    torch.cuda.synchronize()
    return out_ref, out_na


@pytest.fixture(scope="module")
def ctx():
    c = fntrs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def test_noalloc_equals_encode_two_calls_second_smaller(ctx):
    # call 1: k = 16384, n = 32768, 100 lanes x 3 blocks (four-step, scratch 32768 * 128 * 3 words)
    say("noalloc call 1: n=32768 k=16384 lanes=100 batch=3")
    ref, got = both(ctx, 32768, 16384, 100, 3, seed=501)
    assert torch.equal(ref, got)
    # call 2, smaller: k = n = 16384, 40 lanes x 1 block, rows of ld 44
    say("noalloc call 2: n=16384 k=16384 lanes=40 batch=1 ld=44")
    ref, got = both(ctx, 16384, 16384, 40, 1, seed=502, ld_pad=4)
    assert torch.equal(ref, got)
    # the pad lanes stay untouched
    assert bool((got[:, :, 40:] == -7).all())


def test_noalloc_punctured_and_short_codes(ctx):
    say("noalloc: punctured n=40000 k=20000 lanes=33")
    ref, got = both(ctx, 40000, 20000, 33, 1, seed=503)
    assert torch.equal(ref[:, :40000], got[:, :40000])
    say("noalloc: short code n=512 k=256 lanes=64 batch=2 (no scratch)")
    ref, got = both(ctx, 512, 256, 64, 2, seed=504)
    assert torch.equal(ref, got)


def test_noalloc_rejects_sizes_beyond_its_scratch(ctx):
    h = ctx.handle
    # 65536 * 544 words > 2^25: refused on the host, nothing enqueued
    rc = fntrs.fntrs_encode_noalloc(h, 65536, 32768, 513, 0x1000, 513, 32768 * 513, 0x100000000, 513,
                                    65536 * 513, 1, 0, 0)
    assert rc == fntrs.FNTRS_E_NOMEM
    assert "scratch" in fntrs.fntrs_last_error(h)
    rc = fntrs.fntrs_encode_noalloc(h, 512, 256, 4, 0x1000, 4, 1024, 0x100000000, 4, 2048, 1,
                                    fntrs.FNTRS_FLAG_VALIDATE, 0)
    assert rc == fntrs.FNTRS_E_INVAL

"""Host-side checks of the server's memory admission charge.

A request's charge must cover its input, output, locator state and the
scratch of the four-step transforms (2^14 points or more), which the library
holds for a batch while it runs: batch * N rows (decode: N + M rows, M the
low-product length max(2K, N/2)) of the lanes rounded up to 32, 4 bytes per
word.
"""
from paper_0907_1788_amd import serve


def scratch(op, n, k, lanes):
    N = 1 << (n - 1).bit_length()
    L32 = (lanes + 31) // 32 * 32
    logk = (k - 1).bit_length()
    if op == serve.ENCODE:
        return 4 * N * L32 if max(1, logk) >= 14 else 0
    if N < (1 << 14):
        return 0
    M = 1 << max(logk + 1, (n - 1).bit_length() - 1) if k < N else N
    return 4 * (N + M) * L32


def test_charge_covers_data_and_four_step_scratch():
    for op, n, k, lanes in [(serve.ENCODE, 512, 256, 100), (serve.ENCODE, 32768, 16384, 1000),
                            (serve.ENCODE, 65536, 16384, 7), (serve.ENCODE, 32768, 8192, 8192),
                            (serve.DECODE, 16384, 4096, 1000), (serve.DECODE, 16384, 8192, 2047),
                            (serve.DECODE, 32768, 8192, 300), (serve.DECODE, 65536, 16384, 8192),
                            (serve.DECODE, 8192, 4096, 2048)]:
        r = serve.Request(op, n, k, lanes, None)
        rows = k + n if op == serve.ENCODE else n + k
        assert r.device_bytes() >= 4 * lanes * rows + scratch(op, n, k, lanes), (op, n, k, lanes)
    # the largest charge of the uneven distribution: a rate-1/4 decode at n = 65536
    r = serve.Request(serve.DECODE, 65536, 16384, 8192, None)
    assert r.device_bytes() > 4 * (65536 + 32768) * 8192

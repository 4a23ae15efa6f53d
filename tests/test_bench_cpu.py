"""Host-side pieces of bench.py: the butterfly and byte accounting behind its
roofline figures, and the single-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_butterflies_of_the_default_workload():
    # k=4096, n=8192, 2048 lanes x 64 blocks: decode = inverse FNT_8192 plus two
    # FNT_8192 of the low product; encode = two twisted FNT_4096 per lane
    units = 2048 * 64
    assert bench.decode_butterflies(8192, 4096, 2048, 64) == units * (3 * 4096 * 13) == 20937965568
    assert bench.encode_butterflies(8192, 4096, 2048, 64) == units * (2 * 2048 * 12) == 6442450944


def low_product_length(n, k):
    """M as the library picks it: the least power of two >= 2k, and >= n/2."""
    m = 1
    while m < 2 * k or m < n // 2:
        m *= 2
    return m


def test_decode_butterflies_follow_the_low_product_length():
    for n, k in [(8192, 3000), (8192, 4096), (8192, 2048), (8192, 1000), (512, 100), (65536, 32768), (2, 1)]:
        m = low_product_length(n, k)
        lm = m.bit_length() - 1
        ln = n.bit_length() - 1
        assert bench.decode_butterflies(n, k, 1, 1) == (n // 2) * ln + m * lm, (n, k)


def test_encode_butterflies_pad_k_to_a_power_of_two():
    assert bench.encode_butterflies(1024, 300, 1, 1) == 2 * 256 * 9    # K = 512, two cosets
    assert bench.encode_butterflies(512, 256, 1, 1) == 2 * 128 * 8


def test_stored_traffic_is_null_for_another_workload():
    assert bench.stored_traffic("k_dec", "no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout

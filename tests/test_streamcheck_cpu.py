"""Stream ordering and memory lifetimes of the library's host logic, on the CPU.

tests/streamcheck/fake_hip.cpp stands in for the HIP runtime (same soname):
it executes no kernels, but runs every enqueued operation in a seeded random
order on simulated streams and checks each range it touches for bounds,
liveness and ordering (see its header).  tests/streamcheck/replay.py drives
the unmodified library, serve.Server and the benchmark's served request mix
through it.

The first test shows the checker reports planted mistakes (an unordered
cross-stream read, a write past an allocation, a use after a stream-ordered
free, a pinned staging buffer reused before its copy ran) and is silent on
the same sequences ordered correctly.  The others replay the served stream,
including the point where decodes draw from 16 patterns per code so that
most locators are cache hits built by earlier batches on other streams,
over several schedules, device lags, in-flight depths and cache caps (the
smallest forces evictions).
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SC = os.path.join(ROOT, "tests", "streamcheck")
LIB = os.path.join(ROOT, "paper_0907_1788_amd", "libfntrs.so")


@pytest.fixture(scope="module")
def fake(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.fail("libfntrs.so is not built (python -m paper_0907_1788_amd.build)")
    out = tmp_path_factory.mktemp("fakehip") / "libamdhip64.so.7"
    cmd = ["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "paper_0907_1788_amd", "csrc"), "-Wall", "-Wno-unused-function",
           "-Wl,-soname,libamdhip64.so.7", "-Wl,--version-script=" + os.path.join(SC, "fake_hip.map"),
           os.path.join(SC, "fake_hip.cpp"), "-o", str(out)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return str(out)


def run(fake, *args):
    res = subprocess.run([sys.executable, os.path.join(SC, "replay.py"), "--fake", fake, *map(str, args)],
                         capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert res.returncode == 0, res.stderr[-3000:]
    return json.loads(res.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("name,expect", [
    ("encode_chain_ok", None),
    ("decode_other_stream_ok", None),
    ("direct_ok", None),
    ("large_locator_ok", None),
    ("encode_chain_race", "race:"),
    ("out_of_bounds", "out of bounds:"),
    ("use_after_free", "use after free:"),
    ("pinned_reuse", "pinned staging overwritten"),
])
def test_checker_reports_planted_mistakes(fake, name, expect):
    errs = run(fake, "--scenario", name)["errors"]
    if expect is None:
        assert errs == []
    else:
        assert errs and all(e.startswith(expect) for e in errs), errs


@pytest.mark.parametrize("seed,lag,span,inflight,cap_mib,patterns", [
    (1, 0.90, 0.5, 4, 8192, 16),     # the locator-cache point of the served benchmark
    (2, 0.99, 0.3, 4, 8192, 16),
    (3, 0.995, 0.3, 16, 8192, 16),   # deep in-flight queue, device far behind
    (4, 0.99, 0.3, 12, 32, 16),      # a tiny cache cap: evictions under load
    (5, 0.50, 0.5, 4, 8192, 0),      # fresh patterns (the load sweep)
    (6, 0.99, 0.0, 8, 8192, 16),     # closed loop: large batches
    (7, 0.99, 0.0, 8, 4096, 0),      # few scratch blocks: reused across streams while pending
    (8, 0.995, 0.3, 12, 1024, 16),   # scratch larger than the blocks: stream-ordered fallback
])
def test_served_replay_is_clean(fake, seed, lag, span, inflight, cap_mib, patterns):
    r = run(fake, "--seed", seed, "--lag", lag, "--span-s", span, "--max-inflight", inflight,
            "--ctx-cap-mib", cap_mib, "--pattern-pool", patterns, "--requests", 2000)
    assert r["requests"] == 2000
    assert r["kernels"] > 1000
    assert r["errors"] == [], r["errors"][:5]


def test_served_replay_keeps_scratch_blocks(fake):
    """Under a cap that holds the batches' scratch, the context keeps and
    reuses its scratch blocks: after the first batches no call allocates
    stream-ordered memory (new device memory can make the allocating call wait
    for the GPU, which stalls a serving loop)."""
    r = run(fake, "--seed", 9, "--lag", 0.99, "--span-s", 0.0, "--max-inflight", 8, "--ctx-cap-mib", 8192,
            "--pattern-pool", 0, "--requests", 2000)
    assert r["errors"] == [], r["errors"][:5]
    assert r["batches"] > 40
    assert r["hipMallocAsync"] <= 8, r

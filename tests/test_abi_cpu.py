"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments on the host before any GPU work.

A context created on FNTRS_HOST_ONLY runs the full argument validation and
returns FNTRS_E_DEVICE for calls whose arguments pass, so every error path
below is exercised without a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0907_1788_amd import fntrs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fntrs.h")

# fake device addresses: validation never dereferences them
SRC = 0x10000000
DST = 0x90000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fntrs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert {"fntrs_create", "fntrs_destroy", "fntrs_last_error", "fntrs_encode", "fntrs_locator",
            "fntrs_locator_release", "fntrs_locator_export", "fntrs_decode", "fntrs_version"} <= set(names)
    L = fntrs.lib()
    for name in names:
        assert hasattr(L, name), name
        assert name in fntrs.SIGNATURES, name
    assert fntrs.fntrs_version().startswith("fntrs")


def test_error_codes_match_header():
    text = open(HEADER).read()
    for name, val in re.findall(r"(FNTRS_E_[A-Z]+)\s*=\s*(-\d+)", text):
        assert getattr(fntrs, name) == int(val)
    for name, val in re.findall(r"#define (FNTRS_(?:RECV|FLAG)_[A-Z]+) (\d+)u", text):
        assert getattr(fntrs, name) == int(val)


@pytest.fixture()
def hctx():
    h = fntrs.fntrs_create(-1, 0)
    yield h
    fntrs.fntrs_destroy(h)


def enc(h, n, k, lanes, ld_s=None, st_s=None, ld_d=None, st_d=None, batch=1, flags=0, src=SRC, dst=DST):
    ld_s = lanes if ld_s is None else ld_s
    ld_d = lanes if ld_d is None else ld_d
    st_s = k * ld_s if st_s is None else st_s
    st_d = n * ld_d if st_d is None else st_d
    return fntrs.fntrs_encode(h, n, k, lanes, src, ld_s, st_s, dst, ld_d, st_d, batch, flags, 0)


def test_encode_validation(hctx):
    assert enc(hctx, 512, 256, 64) == fntrs.FNTRS_E_DEVICE          # valid, no device
    assert "host-only" in fntrs.fntrs_last_error(hctx)
    assert enc(hctx, 1, 1, 1) == fntrs.FNTRS_E_DEVICE
    assert enc(hctx, 65536, 3, 1) == fntrs.FNTRS_E_DEVICE           # any k <= n
    for n, k in [(0, 1), (3, 1), (131072, 1), (96, 4), (8, 0), (8, 9)]:
        assert enc(hctx, n, k, 4) == fntrs.FNTRS_E_INVAL, (n, k)
    assert enc(hctx, 8, 4, 0) == fntrs.FNTRS_E_INVAL                # no lanes
    assert enc(hctx, 8, 4, 4, batch=0) == fntrs.FNTRS_E_INVAL
    assert enc(hctx, 8, 4, 4, ld_s=3) == fntrs.FNTRS_E_INVAL        # ld < lanes
    assert enc(hctx, 8, 4, 4, ld_d=2) == fntrs.FNTRS_E_INVAL
    assert enc(hctx, 8, 4, 4, batch=2, st_d=16) == fntrs.FNTRS_E_INVAL   # blocks overlap
    assert enc(hctx, 8, 4, 4, src=0) == fntrs.FNTRS_E_INVAL
    assert enc(hctx, 8, 4, 4, dst=SRC + 8) == fntrs.FNTRS_E_INVAL   # src/dst overlap
    assert enc(hctx, 8, 4, 4, flags=0x80) == fntrs.FNTRS_E_INVAL
    assert "flags" in fntrs.fntrs_last_error(hctx)


def test_locator_validation(hctx):
    rc, h = fntrs.fntrs_locator(hctx, 16, 4, [1, 2, 3, 9])
    assert rc == fntrs.FNTRS_E_DEVICE and h is None
    assert fntrs.fntrs_locator(hctx, 16, 4, [1, 2, 3])[0] == fntrs.FNTRS_E_TOOFEW
    assert fntrs.fntrs_locator(hctx, 16, 4, [1, 2, 2, 9])[0] == fntrs.FNTRS_E_POSITIONS
    assert fntrs.fntrs_locator(hctx, 16, 4, [3, 2, 5, 9])[0] == fntrs.FNTRS_E_POSITIONS
    assert fntrs.fntrs_locator(hctx, 16, 4, [1, 2, 3, 16])[0] == fntrs.FNTRS_E_POSITIONS
    assert fntrs.fntrs_locator(hctx, 16, 3, [1, 2, 3])[0] == fntrs.FNTRS_E_UNSUPPORTED
    assert fntrs.fntrs_locator(hctx, 12, 4, [1, 2, 3, 4])[0] == fntrs.FNTRS_E_INVAL
    assert fntrs.fntrs_locator(hctx, 16, 0, [1])[0] == fntrs.FNTRS_E_INVAL
    # more than k received: the first k are used, the rest are not checked for order
    assert fntrs.fntrs_locator(hctx, 16, 2, [1, 5, 3])[0] == fntrs.FNTRS_E_DEVICE


def test_decode_and_release_reject_null(hctx):
    L = fntrs.lib()
    assert L.fntrs_decode(hctx, None, 4, 0, SRC, 4, 16, DST, 4, 16, 1, None) == fntrs.FNTRS_E_INVAL
    assert L.fntrs_locator_release(hctx, None) == fntrs.FNTRS_E_INVAL
    assert L.fntrs_encode(None, 8, 4, 4, SRC, 4, 16, DST, 4, 32, 1, 0, None) == fntrs.FNTRS_E_INVAL
    assert fntrs.fntrs_last_error(None) == "null context"


def test_create_rejects_null_out():
    L = fntrs.lib()
    assert L.fntrs_create(0, 0, None) == fntrs.FNTRS_E_INVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fntrs, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fntrs, "_lib", None)
    with pytest.raises(ImportError):
        fntrs.lib()

"""Python binding of libfntrs (the C ABI in include/fntrs.h).

Argument marshalling only: every step of encoding and decoding runs in the
HIP library.  Loading fails loudly when the shared object is missing; there
is no fallback path.

Two layers:
* ``fntrs_*`` module functions mirror the C entry points one to one and take
  raw device pointers (ints), strides in uint32 elements and a raw
  hipStream_t handle (int, 0 = null stream);
* ``Context`` wraps them for torch tensors of dtype int32 holding residues
  (torch has no full uint32 arithmetic; residues <= 65536 have the same bit
  pattern either way).  Tensors are [batch, rows, lanes] (or [rows, lanes])
  with unit lane stride.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfntrs.so")

FNTRS_OK = 0
FNTRS_E_INVAL = -1
FNTRS_E_TOOFEW = -2
FNTRS_E_POSITIONS = -3
FNTRS_E_RANGE = -4
FNTRS_E_NOMEM = -5
FNTRS_E_DEVICE = -6
FNTRS_E_UNSUPPORTED = -7
ERROR_NAMES = {
    FNTRS_E_INVAL: "FNTRS_E_INVAL", FNTRS_E_TOOFEW: "FNTRS_E_TOOFEW",
    FNTRS_E_POSITIONS: "FNTRS_E_POSITIONS", FNTRS_E_RANGE: "FNTRS_E_RANGE",
    FNTRS_E_NOMEM: "FNTRS_E_NOMEM", FNTRS_E_DEVICE: "FNTRS_E_DEVICE",
    FNTRS_E_UNSUPPORTED: "FNTRS_E_UNSUPPORTED",
}

FNTRS_RECV_COMPACT = 0
FNTRS_RECV_FULL = 1
FNTRS_FLAG_VALIDATE = 2
FNTRS_SYSTEMATIC = 4
FNTRS_DIRECT = 8
FNTRS_TRANSFORM = 16
FNTRS_METHOD_TRANSFORM = 0
FNTRS_METHOD_DIRECT = 1
FNTRS_METHOD_FOURSTEP = 2

FNTRS_OP_ENCODE = 0
FNTRS_OP_DECODE = 1

# every symbol the header declares, with (restype, argtypes)
_u32, _sz, _vp, _int = ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int
_pu32 = ctypes.POINTER(ctypes.c_uint32)


class fntrs_job(ctypes.Structure):
    """struct fntrs_job of include/fntrs.h."""
    _fields_ = [("op", _u32), ("n", _u32), ("k", _u32), ("lanes", _u32), ("batch", _u32), ("flags", _u32),
                ("loc", _vp), ("in_", _vp), ("ld_in", _sz), ("stride_in", _sz),
                ("out", _vp), ("ld_out", _sz), ("stride_out", _sz)]


class fntrs_tuning(ctypes.Structure):
    """struct fntrs_tuning of include/fntrs.h."""
    _fields_ = [("tile_lanes", _u32), ("threads", _u32), ("lanes_per_thread", _u32), ("radix_log2", _u32),
                ("ms", ctypes.c_float), ("op", _u32), ("log2_size", _u32), ("method", _u32),
                ("default_ms", ctypes.c_float)]


_pjob = ctypes.POINTER(fntrs_job)
_ptun = ctypes.POINTER(fntrs_tuning)
SIGNATURES = {
    "fntrs_create": (_int, [_int, _sz, ctypes.POINTER(_vp)]),
    "fntrs_destroy": (None, [_vp]),
    "fntrs_last_error": (ctypes.c_char_p, [_vp]),
    "fntrs_encode": (_int, [_vp, _u32, _u32, _u32, _vp, _sz, _sz, _vp, _sz, _sz, _u32, _u32, _vp]),
    "fntrs_encode_noalloc": (_int, [_vp, _u32, _u32, _u32, _vp, _sz, _sz, _vp, _sz, _sz, _u32, _u32, _vp]),
    "fntrs_locator": (_int, [_vp, _u32, _u32, _pu32, _u32, _vp, ctypes.POINTER(_vp)]),
    "fntrs_locator_batch": (_int, [_vp, _u32, _pu32, _pu32, ctypes.POINTER(_pu32), _pu32, _vp,
                                   ctypes.POINTER(_vp)]),
    "fntrs_locator_release": (_int, [_vp, _vp]),
    "fntrs_locator_export": (_int, [_vp, _vp, _pu32, _pu32, _pu32]),
    "fntrs_decode": (_int, [_vp, _vp, _u32, _u32, _vp, _sz, _sz, _vp, _sz, _sz, _u32, _vp]),
    "fntrs_submit": (_int, [_vp, _pjob, _u32, _vp]),
    "fntrs_pack16": (_int, [_vp, _vp, _sz, _sz, _u32, _u32, _u32, _vp, _sz, _sz, _vp, _vp, _u32, _vp]),
    "fntrs_unpack16": (_int, [_vp, _vp, _sz, _sz, _u32, _u32, _u32, _vp, _vp, _u32, _vp, _sz, _sz, _vp]),
    "fntrs_graph_create": (_int, [_vp, _pjob, _u32, ctypes.POINTER(_vp)]),
    "fntrs_graph_launch": (_int, [_vp, _vp, _vp]),
    "fntrs_graph_destroy": (_int, [_vp, _vp]),
    "fntrs_autotune": (_int, [_vp, _u32, _u32, _u32, _u32, _u32, _u32, _vp, _ptun]),
    "fntrs_get_config": (_int, [_vp, _u32, _u32, _ptun]),
    "fntrs_chirp_eval": (_int, [_vp, _u32, _u32, _u32, _u32, _vp, _sz, _sz, _vp, _sz, _sz, _u32, _u32, _vp]),
    "fntrs_autotune_batch": (_int, [_vp, _pjob, _u32, _u32, _vp, _ptun, _u32, ctypes.POINTER(_u32)]),
    "fntrs_version": (ctypes.c_char_p, []),
}

_lib = None


class FntrsError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Loads libfntrs.so (built in-tree by ``paper_0907_1788_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0907_1788_amd.build`")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libfntrs bind to that copy, so the process holds one HIP
        # runtime and torch's device pointers and streams are valid here.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, rc: int) -> None:
    if rc != FNTRS_OK:
        msg = lib().fntrs_last_error(ctx)
        raise FntrsError(rc, msg.decode() if msg else "")


# ------------------------------------------------------------------ raw ABI
def fntrs_create(device: int = 0, workspace_cap_bytes: int = 0) -> int:
    out = _vp()
    rc = lib().fntrs_create(device, workspace_cap_bytes, ctypes.byref(out))
    if rc != FNTRS_OK:
        raise FntrsError(rc, f"fntrs_create(device={device}) failed")
    return out.value


def fntrs_destroy(ctx: int) -> None:
    lib().fntrs_destroy(ctx)


def fntrs_last_error(ctx: int) -> str:
    return lib().fntrs_last_error(ctx).decode()


def fntrs_encode(ctx, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, flags=0, stream=0):
    return lib().fntrs_encode(ctx, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst,
                              batch, flags, stream)


def fntrs_encode_noalloc(ctx, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, flags=0,
                         stream=0):
    return lib().fntrs_encode_noalloc(ctx, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst,
                                      batch, flags, stream)


def fntrs_locator(ctx, n, k, positions, stream=0):
    """Returns (rc, handle); positions: host sequence of received positions."""
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.uint32))
    out = _vp()
    rc = lib().fntrs_locator(ctx, n, k, pos.ctypes.data_as(_pu32), pos.size, stream, ctypes.byref(out))
    return rc, out.value


def fntrs_locator_batch(ctx, ns, ks, positions, stream=0):
    """Returns (rc, [handles]); positions: one host sequence per pattern."""
    count = len(ns)
    arrs = [np.ascontiguousarray(np.asarray(z, dtype=np.uint32)) for z in positions]
    n_arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint32))
    k_arr = np.ascontiguousarray(np.asarray(ks, dtype=np.uint32))
    npos = np.ascontiguousarray(np.asarray([a.size for a in arrs], dtype=np.uint32))
    ptrs = (_pu32 * max(1, count))(*[a.ctypes.data_as(_pu32) for a in arrs])
    out = (_vp * max(1, count))()
    rc = lib().fntrs_locator_batch(ctx, count, n_arr.ctypes.data_as(_pu32), k_arr.ctypes.data_as(_pu32), ptrs,
                                   npos.ctypes.data_as(_pu32), stream, out)
    return rc, [out[i] for i in range(count)]


def fntrs_locator_release(ctx, loc):
    return lib().fntrs_locator_release(ctx, loc)


def fntrs_locator_export(ctx, loc, k):
    A = np.zeros(k + 1, dtype=np.uint32)
    w = np.zeros(k, dtype=np.uint32)
    ahat = np.zeros(2 * k, dtype=np.uint32)
    rc = lib().fntrs_locator_export(ctx, loc, A.ctypes.data_as(_pu32), w.ctypes.data_as(_pu32),
                                    ahat.ctypes.data_as(_pu32))
    return rc, A, w, ahat


def fntrs_decode(ctx, loc, lanes, flags, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, batch, stream=0):
    return lib().fntrs_decode(ctx, loc, lanes, flags, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst,
                              batch, stream)


def fntrs_submit(ctx, jobs, stream=0):
    """jobs: a ctypes array of fntrs_job (or a list, converted here)."""
    arr = _job_array(jobs)
    return lib().fntrs_submit(ctx, arr, len(arr), stream)


def fntrs_graph_create(ctx, jobs):
    """Returns (rc, handle)."""
    arr = _job_array(jobs)
    out = _vp()
    rc = lib().fntrs_graph_create(ctx, arr, len(arr), ctypes.byref(out))
    return rc, out.value


def fntrs_graph_launch(ctx, graph, stream=0):
    return lib().fntrs_graph_launch(ctx, graph, stream)


def fntrs_graph_destroy(ctx, graph):
    return lib().fntrs_graph_destroy(ctx, graph)


def fntrs_autotune(ctx, op, n, k, lanes, batch, reps=5, stream=0):
    """Returns (rc, fntrs_tuning)."""
    t = fntrs_tuning()
    rc = lib().fntrs_autotune(ctx, op, n, k, lanes, batch, reps, stream, ctypes.byref(t))
    return rc, t


def fntrs_autotune_batch(ctx, jobs, reps=3, stream=0):
    """Returns (rc, [fntrs_tuning per class])."""
    arr = _job_array(jobs)
    cap = 64
    out = (fntrs_tuning * cap)()
    nout = _u32(0)
    rc = lib().fntrs_autotune_batch(ctx, arr, len(arr), reps, stream, out, cap, ctypes.byref(nout))
    return rc, [out[i] for i in range(nout.value)]


def fntrs_get_config(ctx, op, log2_size):
    t = fntrs_tuning()
    rc = lib().fntrs_get_config(ctx, op, log2_size, ctypes.byref(t))
    return rc, t


def fntrs_version() -> str:
    return lib().fntrs_version().decode()


def _job_array(jobs):
    if isinstance(jobs, ctypes.Array):
        return jobs
    arr = (fntrs_job * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return arr if len(jobs) else (fntrs_job * 0)()


# ------------------------------------------------------------------ tensor layer
def _geom(t, rows_expected=None):
    """(batch, rows, lanes, ld, stride) of a [batch, rows, lanes] or [rows, lanes] tensor."""
    if t.dim() == 2:
        t3 = t.unsqueeze(0)
    elif t.dim() == 3:
        t3 = t
    else:
        raise ValueError("expected a [rows, lanes] or [batch, rows, lanes] tensor")
    if t3.stride(2) != 1:
        raise ValueError("lanes must be contiguous (unit stride)")
    b, r, l = t3.shape
    if rows_expected is not None and r != rows_expected:
        raise ValueError(f"expected {rows_expected} rows, got {r}")
    stride = t3.stride(0) if b > 1 else r * t3.stride(1)
    return b, r, l, t3.stride(1), stride


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tuning_dict(t):
    method = {FNTRS_METHOD_TRANSFORM: "transform", FNTRS_METHOD_DIRECT: "direct",
              FNTRS_METHOD_FOURSTEP: "four-step"}.get(t.method, str(t.method))
    return {"op": "encode" if t.op == FNTRS_OP_ENCODE else "decode", "log2_size": t.log2_size, "method": method,
            "tile_lanes": t.tile_lanes, "threads": t.threads, "lanes_per_thread": t.lanes_per_thread,
            "radix_log2": t.radix_log2, "ms": round(t.ms, 4), "default_ms": round(t.default_ms, 4)}


class Locator:
    """A reference to the device-resident state of one erasure pattern."""

    def __init__(self, ctx: "Context", handle: int, n: int, k: int, positions):
        self.ctx, self.handle, self.n, self.k = ctx, handle, n, k
        self.positions = np.asarray(positions, dtype=np.uint32)[:k]

    def release(self) -> None:
        if self.handle:
            _check(self.ctx.handle, fntrs_locator_release(self.ctx.handle, self.handle))
            self.handle = None

    def export(self):
        rc, A, w, ahat = fntrs_locator_export(self.ctx.handle, self.handle, self.k)
        _check(self.ctx.handle, rc)
        return A, w, ahat


class Context:
    """Owns an fntrs context on one device."""

    def __init__(self, device: int = 0, workspace_cap_bytes: int = 0):
        self.device = device
        self.handle = fntrs_create(device, workspace_cap_bytes)

    def close(self) -> None:
        if self.handle:
            fntrs_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def encode(self, src, dst, n: int, flags: int = 0, stream=None) -> None:
        """dst[b, i, l] = sum_j src[b, j, l] r_n^(i j); src has k rows, dst n rows."""
        b, k, lanes, ld_s, st_s = _geom(src)
        b2, _, lanes2, ld_d, st_d = _geom(dst, n)
        if b2 != b or lanes2 != lanes:
            raise ValueError("src and dst disagree on batch or lanes")
        _check(self.handle, fntrs_encode(self.handle, n, k, lanes, src.data_ptr(), ld_s, st_s,
                                         dst.data_ptr(), ld_d, st_d, b, flags, _stream_handle(stream)))

    def locator(self, n: int, k: int, positions, stream=None) -> Locator:
        rc, h = fntrs_locator(self.handle, n, k, positions, _stream_handle(stream))
        _check(self.handle, rc)
        return Locator(self, h, n, k, positions)

    def locators(self, patterns, stream=None):
        """Locators of many patterns [(n, k, positions), ...] built together."""
        ns = [p[0] for p in patterns]
        ks = [p[1] for p in patterns]
        zs = [p[2] for p in patterns]
        rc, hs = fntrs_locator_batch(self.handle, ns, ks, zs, _stream_handle(stream))
        _check(self.handle, rc)
        return [Locator(self, h, n, k, z) for h, n, k, z in zip(hs, ns, ks, zs)]

    def decode(self, loc: Locator, recv, dst, flags: int = FNTRS_RECV_COMPACT, stream=None) -> None:
        """dst [b, k, lanes] <- source recovered from recv ([b, k, lanes] or, FULL, [b, n, lanes])."""
        rows = loc.n if flags & FNTRS_RECV_FULL else loc.k
        b, _, lanes, ld_r, st_r = _geom(recv, rows)
        b2, _, lanes2, ld_d, st_d = _geom(dst, loc.k)
        if b2 != b or lanes2 != lanes:
            raise ValueError("recv and dst disagree on batch or lanes")
        _check(self.handle, fntrs_decode(self.handle, loc.handle, lanes, flags, recv.data_ptr(), ld_r, st_r,
                                         dst.data_ptr(), ld_d, st_d, b, _stream_handle(stream)))

    # -------------------------------------------------------------- batches
    def encode_job(self, src, dst, n: int) -> fntrs_job:
        """An encode job of the batched path (see encode)."""
        b, k, lanes, ld_s, st_s = _geom(src)
        b2, _, lanes2, ld_d, st_d = _geom(dst, n)
        if b2 != b or lanes2 != lanes:
            raise ValueError("src and dst disagree on batch or lanes")
        return fntrs_job(FNTRS_OP_ENCODE, n, k, lanes, b, 0, None, src.data_ptr(), ld_s, st_s,
                         dst.data_ptr(), ld_d, st_d)

    def decode_job(self, loc: Locator, recv, dst, flags: int = FNTRS_RECV_COMPACT) -> fntrs_job:
        """A decode job of the batched path (see decode)."""
        rows = loc.n if flags & FNTRS_RECV_FULL else loc.k
        b, _, lanes, ld_r, st_r = _geom(recv, rows)
        b2, _, lanes2, ld_d, st_d = _geom(dst, loc.k)
        if b2 != b or lanes2 != lanes:
            raise ValueError("recv and dst disagree on batch or lanes")
        return fntrs_job(FNTRS_OP_DECODE, loc.n, loc.k, lanes, b, flags, loc.handle, recv.data_ptr(), ld_r, st_r,
                         dst.data_ptr(), ld_d, st_d)

    def submit(self, jobs, stream=None) -> None:
        """Enqueues a batch of jobs (encode_job / decode_job) in one call."""
        _check(self.handle, fntrs_submit(self.handle, jobs, _stream_handle(stream)))

    def chirp_eval(self, coeffs, out, a: int, q: int, stream=None) -> None:
        """out[b, i, l] = sum_j coeffs[b, j, l] (a q^i)^j for i < out rows (Sec. II-B, the chirp)."""
        b, L, lanes, ld_c, st_c = _geom(coeffs)
        b2, M, lanes2, ld_o, st_o = _geom(out)
        if (b2, lanes2) != (b, lanes):
            raise ValueError("coeffs and out disagree on batch or lanes")
        _check(self.handle, lib().fntrs_chirp_eval(self.handle, L, M, a, q, coeffs.data_ptr(), ld_c, st_c,
                                                   out.data_ptr(), ld_o, st_o, lanes, b, _stream_handle(stream)))

    # ------------------------------------------------------- 16-bit transport
    def pack16(self, src, out16, esc_count, esc_pos, stream=None) -> None:
        """out16 (int16 tensor, the same shape as src) <- src mod 65536; the
        lanes holding 65536 of row r of block b go to esc_count[b*rows + r]
        and esc_pos[b*rows + r, :] (int32 tensors; esc_pos has one row of
        capacity per symbol)."""
        b, rows, lanes, ld_s, st_s = _geom(src)
        b2, rows2, lanes2, ld_o, st_o = _geom(out16, rows)
        if (b2, lanes2) != (b, lanes):
            raise ValueError("src and out16 disagree")
        cap = esc_pos.shape[-1] if esc_pos.numel() else 0
        if esc_count.numel() < b * rows or (cap and esc_pos.numel() < b * rows * cap):
            raise ValueError("escape buffers too small")
        _check(self.handle, lib().fntrs_pack16(self.handle, src.data_ptr(), ld_s, st_s, rows, lanes, b,
                                               out16.data_ptr(), ld_o, st_o, esc_count.data_ptr(),
                                               esc_pos.data_ptr() if cap else None, cap, _stream_handle(stream)))

    def unpack16(self, in16, esc_count, esc_pos, dst, stream=None) -> None:
        """Inverse of pack16: dst (int32) <- in16 widened, listed lanes 65536."""
        b, rows, lanes, ld_i, st_i = _geom(in16)
        b2, rows2, lanes2, ld_d, st_d = _geom(dst, rows)
        if (b2, lanes2) != (b, lanes):
            raise ValueError("in16 and dst disagree")
        cap = esc_pos.shape[-1] if esc_pos.numel() else 0
        if esc_count.numel() < b * rows or (cap and esc_pos.numel() < b * rows * cap):
            raise ValueError("escape buffers too small")
        _check(self.handle, lib().fntrs_unpack16(self.handle, in16.data_ptr(), ld_i, st_i, rows, lanes, b,
                                                 esc_count.data_ptr(), esc_pos.data_ptr() if cap else None, cap,
                                                 dst.data_ptr(), ld_d, st_d, _stream_handle(stream)))

    def graph(self, jobs) -> "Graph":
        """Captures a batch into a replayable HIP graph."""
        rc, h = fntrs_graph_create(self.handle, jobs)
        _check(self.handle, rc)
        return Graph(self, h)

    def autotune(self, op: int, n: int, k: int, lanes: int, batch: int = 1, reps: int = 5, stream=None):
        """Times every configuration of the size class and keeps the fastest; returns it as a dict."""
        rc, t = fntrs_autotune(self.handle, op, n, k, lanes, batch, reps, _stream_handle(stream))
        _check(self.handle, rc)
        return _tuning_dict(t)

    def autotune_batch(self, jobs, reps: int = 3, stream=None):
        """Tunes every size class of a batch on its own jobs; returns one dict per class."""
        rc, ts = fntrs_autotune_batch(self.handle, jobs, reps, _stream_handle(stream))
        _check(self.handle, rc)
        return [_tuning_dict(t) for t in ts]

    def config(self, op: int, log2_size: int):
        rc, t = fntrs_get_config(self.handle, op, log2_size)
        _check(self.handle, rc)
        return {"tile_lanes": t.tile_lanes, "threads": t.threads, "lanes_per_thread": t.lanes_per_thread,
                "radix_log2": t.radix_log2}


class Graph:
    """A captured batch (fntrs_graph_t)."""

    def __init__(self, ctx: Context, handle: int):
        self.ctx, self.handle = ctx, handle

    def launch(self, stream=None) -> None:
        _check(self.ctx.handle, fntrs_graph_launch(self.ctx.handle, self.handle, _stream_handle(stream)))

    def destroy(self) -> None:
        if self.handle:
            _check(self.ctx.handle, fntrs_graph_destroy(self.ctx.handle, self.handle))
            self.handle = None

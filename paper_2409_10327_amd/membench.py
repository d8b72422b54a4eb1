"""ctypes binding of libhg_membench.so (include/hg_membench.h) and the
measurements bench.py reports as ceilings: random-gather rates, FP32 atomic
rates and matrix-core loop rates, each timed with events on torch's current
stream (the stream the launches go to)."""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhg_membench.so")
EXPORTS = ["hgmb_gather", "hgmb_gather_indexed", "hgmb_atomic", "hgmb_atomic_lines", "hgmb_mfma"]
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_10327_amd.build`")
        L = C.CDLL(LIB_PATH)
        for n in EXPORTS:
            getattr(L, n).restype = C.c_int
        L.hgmb_gather.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_void_p,
                                  C.c_void_p]
        L.hgmb_gather_indexed.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                          C.c_void_p]
        L.hgmb_atomic.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_void_p]
        L.hgmb_atomic_lines.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32,
                                        C.c_void_p]
        L.hgmb_mfma.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _timed(launch, reps):
    """Mean ms per launch over `reps` launches after one warm-up."""
    if launch() != 0:
        raise RuntimeError("membench launch rejected")
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        launch()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def _cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


def gather(footprint_bytes: int, item_bytes: int, reps: int = 5, rounds: int = 32):
    """Random item_bytes gathers over a table of footprint_bytes: items/s
    and useful GB/s."""
    log2_items = (footprint_bytes // item_bytes).bit_length() - 1
    table = torch.ones((1 << log2_items) * item_bytes // 4, device="cuda", dtype=torch.int32)
    blocks = _cus() * 32
    sink = torch.empty(blocks * 256, device="cuda", dtype=torch.int32)
    ms = _timed(lambda: lib().hgmb_gather(C.c_void_p(table.data_ptr()), log2_items, item_bytes, blocks, rounds, 7,
                                          C.c_void_p(sink.data_ptr()), _stream()), reps)
    n = blocks * 256 * rounds * 8
    return {"footprint_MiB": (1 << log2_items) * item_bytes / 2**20, "item_bytes": item_bytes, "ms": ms,
            "items_per_s": n / (ms * 1e-3), "useful_GBps": n * item_bytes / (ms * 1e-3) / 1e9}


def gather_indexed_ms(table: torch.Tensor, item_bytes: int, idx: torch.Tensor, reps: int = 3,
                      blocks_per_cu: int = 8) -> float:
    """Mean ms to gather table[idx] in eight-item groups over a persistent
    grid (idx: int32 item indices inside the table, checked here)."""
    assert idx.dtype == torch.int32 and idx.is_contiguous() and table.is_contiguous()
    assert int(idx.min()) >= 0 and int(idx.max()) < table.numel() * table.element_size() // item_bytes
    blocks = _cus() * blocks_per_cu
    sink = torch.empty(blocks * 256, device=table.device, dtype=torch.int32)
    return _timed(lambda: lib().hgmb_gather_indexed(C.c_void_p(table.data_ptr()), item_bytes,
                                                    C.c_void_p(idx.data_ptr()), idx.numel(), blocks,
                                                    C.c_void_p(sink.data_ptr()), _stream()), reps)


def atomic(footprint_bytes: int, lanes_per_address: int, reps: int = 5, rounds: int = 16):
    """FP32 atomic adds (lanes_per_address lanes on one address): atomics/s
    issued by the lanes."""
    log2_items = (footprint_bytes // 4).bit_length() - 1
    table = torch.zeros(1 << log2_items, device="cuda", dtype=torch.float32)
    blocks = _cus() * 32
    ms = _timed(lambda: lib().hgmb_atomic(C.c_void_p(table.data_ptr()), log2_items, blocks, rounds,
                                          lanes_per_address, 7, _stream()), reps)
    n = blocks * 256 * rounds * 4
    return {"footprint_MiB": (1 << log2_items) * 4 / 2**20, "lanes_per_address": lanes_per_address, "ms": ms,
            "lane_atomics_per_s": n / (ms * 1e-3), "addresses_per_s": n / lanes_per_address / (ms * 1e-3)}


def atomic_lines(footprint_bytes: int, lanes_per_line: int, reps: int = 5, rounds: int = 16):
    """FP32 atomic adds where groups of lanes_per_line lanes hit adjacent
    words of one line: lane atomics/s and groups (requests)/s."""
    log2_items = (footprint_bytes // 4).bit_length() - 1
    table = torch.zeros(1 << log2_items, device="cuda", dtype=torch.float32)
    blocks = _cus() * 32
    ms = _timed(lambda: lib().hgmb_atomic_lines(C.c_void_p(table.data_ptr()), log2_items, blocks, rounds,
                                                lanes_per_line, 7, _stream()), reps)
    n = blocks * 256 * rounds * 4
    return {"footprint_MiB": (1 << log2_items) * 4 / 2**20, "lanes_per_line": lanes_per_line, "ms": ms,
            "lane_atomics_per_s": n / (ms * 1e-3), "requests_per_s": n / lanes_per_line / (ms * 1e-3)}


def mfma(kind: str, chains: int, waves_per_simd: int = 2, iters: int = 4096, reps: int = 3):
    """Matrix-core loop rate in TFLOP/s: kind 'f32' (32x32x2) or 'bf16'
    (16x16x32); one block of four waves per CU per wave-per-SIMD."""
    k = {"f32": 0, "bf16": 1}[kind]
    blocks = _cus() * waves_per_simd
    sink = torch.empty(blocks * 256, device="cuda", dtype=torch.float32)
    ms = _timed(lambda: lib().hgmb_mfma(k, blocks, iters, chains, C.c_void_p(sink.data_ptr()), _stream()), reps)
    flop = blocks * 4 * iters * chains * (4096 if k == 0 else 16384)
    return {"kind": kind, "chains": chains, "waves_per_simd": waves_per_simd, "ms": ms,
            "TFLOPs": flop / (ms * 1e-3) / 1e12}

"""Thin Python binding over ``libvdmc.so`` (ctypes).

Argument marshalling only: every step of the motif count runs in the library's HIP
kernels.  PyTorch provides device memory and streams; counts come back as
``torch.int64`` tensors holding the uint64 bit patterns (all counts here stay far
below 2^63).  There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvdmc.so")

SYMBOLS = [
    "vdmc_last_error", "vdmc_num_classes", "vdmc_class_codes", "vdmc_class_table",
    "vdmc_class_codes_u32", "vdmc_class_table_u16",
    "vdmc_build_graph", "vdmc_graph_info", "vdmc_graph_export", "vdmc_free_graph",
    "vdmc_count", "vdmc_count_supported", "vdmc_count_range", "vdmc_count34", "vdmc_shape_counts", "vdmc_profile_counters",
    "vdmc_kernel_times", "vdmc_num_classes_undirected", "vdmc_undirected_classes", "vdmc_count_undirected",
    "vdmc_edge_list", "vdmc_count_edges",
    "vdmc_count_batch", "vdmc_tune", "vdmc_tuned_choice", "vdmc_set_hub_threshold",
    "vdmc_init", "vdmc_count_batch_noalloc",
    "vdmc_serve_create", "vdmc_serve_submit", "vdmc_serve_poll", "vdmc_serve_wait",
    "vdmc_serve_stats", "vdmc_serve_destroy", "vdmc_serve_counters",
]

STATUS = {
    0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "UNSUPPORTED",
    5: "BUSY", 6: "NOT_FOUND", 7: "REJECTED", 8: "TIMEOUT",
}
INPUT_ON_DEVICE = 2
UNDIRECTED = 4
SHAPES = ["(1,1)", "(1,2)", "(3,0,0)", "(2,1,0)", "(1,2,0)", "(1,1,1)"]


class VdmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2201_11655_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "vdmc_last_error": ([], ctypes.c_char_p),
        "vdmc_num_classes": ([i32], i32),
        "vdmc_class_codes": ([i32, p], i32),
        "vdmc_class_table": ([i32, p], i32),
        "vdmc_class_codes_u32": ([i32, p], i32),
        "vdmc_class_table_u16": ([i32, p], i32),
        "vdmc_build_graph": ([i64, i64, p, p, u32, p, p], i32),
        "vdmc_graph_info": ([p, p, p, p, p], i32),
        "vdmc_graph_export": ([p, p, p, p], i32),
        "vdmc_free_graph": ([p], i32),
        "vdmc_count": ([p, i32, p, p], i32),
        "vdmc_count_supported": ([p, i32], i32),
        "vdmc_count34": ([p, p, p, p], i32),
        "vdmc_count_range": ([p, i32, p, i64, i64, u32, p], i32),
        "vdmc_shape_counts": ([p, p], i32),
        "vdmc_profile_counters": ([p, p, i32], i32),
        "vdmc_kernel_times": ([p, p, i32], i32),
        "vdmc_num_classes_undirected": ([i32], i32),
        "vdmc_undirected_classes": ([i32, p], i32),
        "vdmc_count_undirected": ([p, i32, p, p], i32),
        "vdmc_edge_list": ([p, p, p], i32),
        "vdmc_count_edges": ([p, i32, p, p], i32),
        "vdmc_count_batch": ([p, i32, i32, p, p], i32),
        "vdmc_tune": ([p, i32, i32, ctypes.c_char_p], i32),
        "vdmc_tuned_choice": ([p, i32, i32, p], i32),
        "vdmc_set_hub_threshold": ([p, i32], i32),
        "vdmc_init": ([], i32),
        "vdmc_count_batch_noalloc": ([p, i32, i32, p, p], i32),
        "vdmc_serve_create": ([p, p], i32),
        "vdmc_serve_submit": ([p, p, i32, p, p], i32),
        "vdmc_serve_poll": ([p, u64, p], i32),
        "vdmc_serve_wait": ([p, u64, i64], i32),
        "vdmc_serve_stats": ([p, p, p, p, p], i32),
        "vdmc_serve_destroy": ([p], i32),
        "vdmc_serve_counters": ([p, p, i32], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load().vdmc_last_error()
        raise VdmcError(status, msg.decode() if msg else "")


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    """hipStream_t of a torch stream (None: torch's current stream)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def num_classes(k: int) -> int:
    return int(load().vdmc_num_classes(k))


def class_codes(k: int) -> np.ndarray:
    """Minimal index of every class, by class id (uint16 for k = 3, 4; uint32 for k = 5)."""
    nc = num_classes(k)
    if nc < 0:
        raise VdmcError(1, f"k={k}")
    if k == 5:
        out = np.zeros(nc, np.uint32)
        _check(load().vdmc_class_codes_u32(k, _np_ptr(out)))
        return out
    out = np.zeros(nc, np.uint16)
    _check(load().vdmc_class_codes(k, _np_ptr(out)))
    return out


def class_table(k: int) -> np.ndarray:
    """Class id of every code (uint8, 0xFF = disconnected, for k = 3, 4; uint16, 0xFFFF,
    for k = 5)."""
    if k == 5:
        out = np.zeros(1 << 20, np.uint16)
        _check(load().vdmc_class_table_u16(k, _np_ptr(out)))
        return out
    out = np.zeros(1 << (k * (k - 1)), np.uint8)
    _check(load().vdmc_class_table(k, _np_ptr(out)))
    return out


class Graph:
    """A graph resident on the current device (ranked symmetric CSR with arc bits).

    ``src``/``dst`` are numpy arrays (host) or int32 CUDA tensors (device).
    ``undirected=True`` ignores arc directions (count with ``count_undirected``)."""

    def __init__(self, n: int, src, dst, stream=None, undirected: bool = False):
        lib = load()
        self._h = ctypes.c_void_p()
        self.n = int(n)
        self.undirected = bool(undirected)
        flags = UNDIRECTED if undirected else 0
        keep = []
        if hasattr(src, "is_cuda") and src.is_cuda:
            torch = _torch()
            s = src.to(torch.int32).contiguous()
            d = dst.to(torch.int32).contiguous()
            keep = [s, d]
            ps, pd = ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr())
            m = s.numel()
            flags |= INPUT_ON_DEVICE
        else:
            s = np.ascontiguousarray(src, dtype=np.int32)
            d = np.ascontiguousarray(dst, dtype=np.int32)
            keep = [s, d]
            ps, pd = _np_ptr(s), _np_ptr(d)
            m = s.shape[0]
        if len(keep[0]) != len(keep[1]):
            raise VdmcError(1, "src and dst differ in length")
        sh = _stream_handle(stream)
        _check(lib.vdmc_build_graph(self.n, int(m), ps, pd, flags, sh, ctypes.byref(self._h)))
        n_, arcs, pairs = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        md = ctypes.c_int32()
        _check(lib.vdmc_graph_info(self._h, ctypes.byref(n_), ctypes.byref(arcs), ctypes.byref(pairs),
                                   ctypes.byref(md)))
        self.arcs, self.pairs, self.max_deg = arcs.value, pairs.value, md.value

    @property
    def handle(self):
        return self._h

    def export(self):
        """(off[n+1], adj[2*pairs], perm[n]) of the rank-space CSR, as numpy arrays."""
        off = np.zeros(self.n + 1, np.uint32)
        adj = np.zeros(max(1, 2 * self.pairs), np.uint32)
        perm = np.zeros(max(1, self.n), np.int32)
        _check(load().vdmc_graph_export(self._h, _np_ptr(off), _np_ptr(adj), _np_ptr(perm)))
        return off, adj[: 2 * self.pairs], perm[: self.n]

    def free(self):
        if self._h is not None and self._h.value:
            _check(load().vdmc_free_graph(self._h))
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _out_tensor(n: int, k: int, out):
    torch = _torch()
    C = num_classes(k)
    if out is None:
        out = torch.empty((n, C), dtype=torch.int64, device="cuda")
    if out.dtype != torch.int64 or not out.is_cuda or not out.is_contiguous() or out.numel() != n * C:
        raise VdmcError(1, f"out must be a contiguous int64 CUDA tensor of {n}x{C}")
    return out


def num_classes_undirected(k: int) -> int:
    return int(load().vdmc_num_classes_undirected(k))


def undirected_classes(k: int) -> np.ndarray:
    """Directed class id of every undirected class (ascending)."""
    nc = num_classes_undirected(k)
    if nc < 0:
        raise VdmcError(1, f"k={k}")
    out = np.zeros(nc, np.uint8)
    _check(load().vdmc_undirected_classes(k, _np_ptr(out)))
    return out


def count_undirected(g: Graph, k: int, out=None, stream=None):
    """Per-vertex undirected k-motif counts, int64[n, 2 or 6] on the device (row = original id)."""
    lib = load()
    U = num_classes_undirected(k)
    if U < 0:
        _check(lib.vdmc_count_undirected(g.handle, int(k), None, _stream_handle(stream)))
    torch = _torch()
    if out is None:
        out = torch.empty((g.n, U), dtype=torch.int64, device="cuda")
    if out.dtype != torch.int64 or not out.is_cuda or not out.is_contiguous() or out.numel() != g.n * U:
        raise VdmcError(1, f"out must be a contiguous int64 CUDA tensor of {g.n}x{U}")
    _check(lib.vdmc_count_undirected(g.handle, int(k), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def edge_list(g: Graph):
    """(lo[P], hi[P]) original-id endpoints of the G_U pairs, in per-edge output order."""
    lo = np.zeros(max(g.pairs, 1), np.int32)
    hi = np.zeros(max(g.pairs, 1), np.int32)
    _check(load().vdmc_edge_list(g.handle, _np_ptr(lo), _np_ptr(hi)))
    return lo[:g.pairs].copy(), hi[:g.pairs].copy()


def count_edges(g: Graph, k: int, out=None, stream=None):
    """Per-edge k-motif counts, int64[P, C] on the device (row order of ``edge_list``)."""
    lib = load()
    C = num_classes(k)
    if C < 0:
        _check(lib.vdmc_count_edges(g.handle, int(k), None, _stream_handle(stream)))
    torch = _torch()
    if out is None:
        out = torch.empty((g.pairs, C), dtype=torch.int64, device="cuda")
    if out.dtype != torch.int64 or not out.is_cuda or not out.is_contiguous() or out.numel() != g.pairs * C:
        raise VdmcError(1, f"out must be a contiguous int64 CUDA tensor of {g.pairs}x{C}")
    _check(lib.vdmc_count_edges(g.handle, int(k), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def count_supported(g: Graph, k: int) -> bool:
    """Whether vdmc_count can count g for this k (k = 5: n x 9364 below 2^31)."""
    return int(load().vdmc_count_supported(g.handle, int(k))) == 1


def count(g: Graph, k: int, out=None, stream=None):
    """Per-vertex k-motif counts, int64[n, C] on the device (row = original id)."""
    if k not in (3, 4, 5):
        _check(load().vdmc_count(g.handle, int(k), None, _stream_handle(stream)))
    if k == 5 and not count_supported(g, 5):
        raise VdmcError(4, f"5-vertex counts need n x 9364 below 2^31; n = {g.n}")
    out = _out_tensor(g.n, k, out)
    _check(load().vdmc_count(g.handle, int(k), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def count_range(g: Graph, k: int, out, rank_begin: int, rank_end: int, accumulate: bool, stream=None):
    """Counts contributed by roots with rank in [rank_begin, rank_end) (see vdmc.h)."""
    out = _out_tensor(g.n, k, out)
    _check(load().vdmc_count_range(g.handle, int(k), ctypes.c_void_p(out.data_ptr()), int(rank_begin),
                                   int(rank_end), 1 if accumulate else 0, _stream_handle(stream)))
    return out


def count34(g: Graph, out3=None, out4=None, stream=None):
    out3 = _out_tensor(g.n, 3, out3)
    out4 = _out_tensor(g.n, 4, out4)
    _check(load().vdmc_count34(g.handle, ctypes.c_void_p(out3.data_ptr()), ctypes.c_void_p(out4.data_ptr()),
                               _stream_handle(stream)))
    return out3, out4


def shape_counts(g: Graph) -> dict:
    out = np.zeros(6, np.uint64)
    _check(load().vdmc_shape_counts(g.handle, _np_ptr(out)))
    return {s: int(v) for s, v in zip(SHAPES, out)}


SHAPES5 = ("(4)", "(3,1)", "(2,2)", "(2,1,1)", "(1,3)", "(1,2,1)", "(1,1,2)", "(1,1,1,1)")


def shape_counts5(g: Graph) -> dict:
    """Sets visited per BFS layer shape by the last 5-vertex count on g."""
    return {s: int(v) for s, v in zip(SHAPES5, profile_counters(g))}


def profile_counters(g: Graph) -> np.ndarray:
    """Diagnostic counters of the last count (see vdmc_profile_counters in vdmc.h)."""
    out = np.zeros(8, np.uint64)
    _check(load().vdmc_profile_counters(g.handle, _np_ptr(out), 8))
    return out


def kernel_times(g: Graph) -> tuple:
    """(per-set kernel ms, hub path ms, hub kernel alone ms) of the last count call on g;
    -1 for a part that was not launched."""
    out = np.zeros(3, np.float32)
    _check(load().vdmc_kernel_times(g.handle, _np_ptr(out), 3))
    return float(out[0]), float(out[1]), float(out[2])


def count_batch(graphs, k: int, outs=None, stream=None):
    """One batched launch over many graphs; returns the list of output tensors."""
    lib = load()
    if k not in (3, 4, 5):
        _check(lib.vdmc_count_batch(None, len(graphs), int(k), None, _stream_handle(stream)))
    if k == 5:
        for i, g in enumerate(graphs):
            if not count_supported(g, 5):
                raise VdmcError(4, f"graph {i}: 5-vertex counts need n x 9364 below 2^31")
    if outs is None:
        outs = [_out_tensor(g.n, k, None) for g in graphs]
    hs = (ctypes.c_void_p * max(1, len(graphs)))(*[g.handle.value for g in graphs])
    ps = (ctypes.c_void_p * max(1, len(graphs)))(*[o.data_ptr() for o in outs])
    _check(lib.vdmc_count_batch(ctypes.cast(hs, ctypes.c_void_p), len(graphs), int(k),
                                ctypes.cast(ps, ctypes.c_void_p), _stream_handle(stream)))
    return outs


def init():
    """Per-device set-up of the library on the current device (see vdmc_init)."""
    _check(load().vdmc_init())


def count_batch_noalloc(graphs, k: int, outs, stream=None):
    """vdmc_count_batch_noalloc: the batched count into caller-owned outputs, no allocation."""
    lib = load()
    hs = (ctypes.c_void_p * max(1, len(graphs)))(*[g.handle.value for g in graphs])
    ps = (ctypes.c_void_p * max(1, len(graphs)))(*[o.data_ptr() for o in outs])
    _check(lib.vdmc_count_batch_noalloc(ctypes.cast(hs, ctypes.c_void_p), len(graphs), int(k),
                                        ctypes.cast(ps, ctypes.c_void_p), _stream_handle(stream)))
    return outs


def tune(graphs, k: int, cache_path: str | None = None):
    hs = (ctypes.c_void_p * max(1, len(graphs)))(*[g.handle.value for g in graphs])
    _check(load().vdmc_tune(ctypes.cast(hs, ctypes.c_void_p), len(graphs), int(k),
                            cache_path.encode() if cache_path else None))


def tuned_choice(graphs, k: int) -> dict:
    """Launch parameters vdmc_count_batch uses for a batch of this shape."""
    hs = (ctypes.c_void_p * max(1, len(graphs)))(*[g.handle.value for g in graphs])
    c = (ctypes.c_int32 * 5)()
    _check(load().vdmc_tuned_choice(ctypes.cast(hs, ctypes.c_void_p), len(graphs), int(k),
                                    ctypes.cast(c, ctypes.c_void_p)))
    return {"tuned": bool(c[0]), "small_threads": c[1], "threads_per_root": c[2],
            "workgroups_per_cu": c[3], "tile": c[4]}


def set_hub_threshold(g: "Graph", min_higher: int):
    """Roots with at least min_higher higher neighbours take the hub path (counts unchanged)."""
    _check(load().vdmc_set_hub_threshold(g.handle, int(min_higher)))


class ServeConfig(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32)]


class Server:
    """Continuous-batching request loop over resident graphs (see vdmc_serve_* in vdmc.h)."""

    def __init__(self, mem_budget_bytes: int, max_inflight: int):
        self._h = ctypes.c_void_p()
        cfg = ServeConfig(int(mem_budget_bytes), int(max_inflight))
        _check(load().vdmc_serve_create(ctypes.byref(cfg), ctypes.byref(self._h)))

    def submit(self, g: Graph, k: int, out) -> int:
        rid = ctypes.c_uint64()
        _check(load().vdmc_serve_submit(self._h, g.handle, int(k), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.byref(rid)))
        return rid.value

    def poll(self, rid: int) -> bool:
        done = ctypes.c_int32()
        _check(load().vdmc_serve_poll(self._h, ctypes.c_uint64(rid), ctypes.byref(done)))
        return bool(done.value)

    def wait(self, rid: int, timeout_us: int = -1):
        _check(load().vdmc_serve_wait(self._h, ctypes.c_uint64(rid), int(timeout_us)))

    def stats(self) -> dict:
        p50, p99, rps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        sets = ctypes.c_uint64()
        _check(load().vdmc_serve_stats(self._h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(rps),
                                       ctypes.byref(sets)))
        out = {"p50_us": p50.value, "p99_us": p99.value, "req_per_s": rps.value, "sets": sets.value}
        c = np.zeros(10, np.uint64)
        _check(load().vdmc_serve_counters(self._h, _np_ptr(c), 10))
        names = ["submitted", "admitted", "completed", "rejected", "failed", "deferred_by_memory",
                 "queue_depth", "max_queue_depth", "bytes_in_flight", "max_bytes_in_flight"]
        out.update({k: int(x) for k, x in zip(names, c)})
        return out

    def close(self):
        if self._h is not None and self._h.value:
            _check(load().vdmc_serve_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

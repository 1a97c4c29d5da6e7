"""Python binding of libhisalog (include/hisalog.h): argument marshalling only.

Every step of the fixpoint runs in the library's gfx950 kernels.  PyTorch
provides device memory (tensors passed to the ``*_device`` calls and the
primitives) and the stream the engine enqueues on.  There is no fallback:
if the library has not been built, importing the binding raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhisalog.so")

HL_OK = 0
HL_E_INVALID = -1
HL_E_NOMEM = -2
HL_E_DEVICE = -3
HL_E_STATE = -4
HL_E_CAPACITY = -5
HL_E_UNSUPPORTED = -6
# size of the static device scratch behind hl_sort_keys_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20
HL_FLAG_NO_EBM = 0x1
HL_FLAG_KERNEL_TIMING = 0x2
HL_FLAG_LEARNED_INDEX = 0x4
HL_FLAG_JOIN_DEDUP = 0x8
HL_FLAG_FUSED = 0x10
HL_FLAG_HIP_GRAPH = 0x20
HL_FLAG_NESTED_JOINS = 0x40
HL_FLAG_NO_LEVELS = 0x80
KERNELS = ("radix_hist", "radix_scatter", "unique_diff", "merge", "join_probe", "join_expand",
           "hisa_build", "learned_fit")
PHASES = ("index_edb", "join", "sort", "diff", "merge", "index", "fused")

# Symbols of include/hisalog.h, in declaration order.
EXPORTS = (
    "hl_options_init", "hl_create", "hl_destroy", "hl_declare", "hl_load", "hl_load_device",
    "hl_batch_layout", "hl_load_batched", "hl_batch_count", "hl_fetch_batched", "hl_index",
    "hl_program", "hl_run", "hl_autotune", "hl_count", "hl_fetch", "hl_fetch_device",
    "hl_iteration_counts", "hl_kernel_stats", "hl_rule_stats", "hl_last_error", "hl_strerror",
    "hl_sort_keys", "hl_sort_keys_noalloc",
    "hl_unique_diff", "hl_merge", "hl_hisa_query", "hl_learned_query",
)


class HlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32), ("flags", ctypes.c_uint32), ("arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_uint64), ("hbm_budget_bytes", ctypes.c_uint64),
        ("stream", ctypes.c_void_p), ("ebm_k", ctypes.c_float),
        ("hash_load_factor", ctypes.c_float), ("sort_chunk_log2", ctypes.c_uint32),
        ("fused_capacity", ctypes.c_uint32), ("expand_tile", ctypes.c_uint32),
        ("sort_tile", ctypes.c_uint32), ("diff_tile", ctypes.c_uint32),
        ("outer_slice_log2", ctypes.c_uint32), ("tail_min_bytes", ctypes.c_uint64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_uint32), ("key_bytes", ctypes.c_uint32),
        ("id_bits", ctypes.c_uint32), ("fused_iterations", ctypes.c_uint32),
        ("idb_tuples", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
        ("peak_bytes", ctypes.c_uint64), ("allocations", ctypes.c_uint64),
        ("ebm_reuses", ctypes.c_uint64), ("seconds", ctypes.c_double),
        ("phase_ms", ctypes.c_double * len(PHASES)),
        ("join_outputs", ctypes.c_uint64),
        ("fused_overflows", ctypes.c_uint32), ("graph_captures", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "phase_ms"}
        d["phase_ms"] = dict(zip(PHASES, list(self.phase_ms)))
        return d


class Tuning(ctypes.Structure):
    _fields_ = [
        ("hash_load_factor", ctypes.c_float), ("ebm_k", ctypes.c_float),
        ("flags", ctypes.c_uint32), ("trials", ctypes.c_uint32),
        ("best_seconds", ctypes.c_double), ("first_seconds", ctypes.c_double),
        ("expand_tile", ctypes.c_uint32), ("sort_tile", ctypes.c_uint32),
        ("diff_tile", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libhisalog.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2311_02206_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, cp, u64, u32, i32 = (ctypes.c_void_p, ctypes.c_char_p, ctypes.c_uint64,
                             ctypes.c_uint32, ctypes.c_int32)
    pu64, pu32 = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)
    sig = {
        "hl_options_init": [ctypes.POINTER(Options)],
        "hl_create": [ctypes.POINTER(Options), ctypes.POINTER(vp)],
        "hl_destroy": [vp],
        "hl_declare": [vp, cp, u32, i32],
        "hl_load": [vp, cp, vp, u64],
        "hl_load_device": [vp, cp, vp, u64],
        "hl_index": [vp, cp, pu32, u32],
        "hl_batch_layout": [vp, vp, u32],
        "hl_load_batched": [vp, cp, vp, vp],
        "hl_batch_count": [vp, cp, u32, pu64],
        "hl_fetch_batched": [vp, cp, u32, vp, u64, pu64],
        "hl_program": [vp, cp],
        "hl_run": [vp, ctypes.POINTER(Stats)],
        "hl_autotune": [vp, u32, ctypes.POINTER(Tuning)],
        "hl_count": [vp, cp, pu64],
        "hl_fetch": [vp, cp, vp, u64, pu64],
        "hl_fetch_device": [vp, cp, vp, u64, pu64],
        "hl_iteration_counts": [vp, cp, i32, pu64, u32, pu32],
        "hl_kernel_stats": [vp, i32, pu64, ctypes.POINTER(ctypes.c_double), pu64],
        "hl_last_error": [vp],
        "hl_strerror": [ctypes.c_int],
        "hl_sort_keys": [vp, vp, u64, u32, u32],
        "hl_sort_keys_noalloc": [vp, vp, u64, u32, u32],
        "hl_rule_stats": [vp, u32, pu64, pu64],
        "hl_unique_diff": [vp, vp, u64, vp, u64, vp, pu64, pu64, u32],
        "hl_merge": [vp, vp, u64, vp, u64, vp, u32],
        "hl_hisa_query": [vp, vp, u64, u32, u32, vp, u64, vp, vp, pu64],
        "hl_learned_query": [vp, vp, u64, u32, u32, vp, u64, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.hl_destroy.restype = None
    L.hl_last_error.restype = cp
    L.hl_strerror.restype = cp
    _lib = L
    return L


def _ptr(t) -> int:
    return int(t.data_ptr())


def _key_bytes(t) -> int:
    import torch
    if t.dtype in (torch.int32, torch.uint32):
        return 4
    if t.dtype in (torch.int64, torch.uint64):
        return 8
    raise TypeError("keys must be a 32- or 64-bit integer tensor")


@dataclass
class RunStats:
    iterations: int
    key_bytes: int
    id_bits: int
    idb_tuples: int
    candidates: int
    peak_bytes: int
    allocations: int
    ebm_reuses: int
    seconds: float
    phase_ms: dict = field(default_factory=dict)
    join_outputs: int = 0
    fused_iterations: int = 0
    fused_overflows: int = 0
    graph_captures: int = 0


class Engine:
    """One hisalog engine on one GPU (see include/hisalog.h)."""

    def __init__(self, device: int = 0, stream=None, arena=None, ebm: bool = True,
                 ebm_k: float = 8.0, load_factor: float = 0.5, budget_bytes: int = 0,
                 kernel_timing: bool = False, learned: bool = False, sort_chunk_log2: int = 0,
                 join_dedup: bool = False, fused: bool = False, hip_graph: bool = False,
                 fused_capacity: int = 0, nested_joins: bool = False, expand_tile: int = 0,
                 sort_tile: int = 0, diff_tile: int = 0, levels: bool = True,
                 tail_min_bytes: int = 0, outer_slice_log2: int = 0):
        L = lib()
        opt = Options()
        L.hl_options_init(ctypes.byref(opt))
        opt.device = device
        opt.flags = ((0 if ebm else HL_FLAG_NO_EBM) |
                     (HL_FLAG_KERNEL_TIMING if kernel_timing else 0) |
                     (HL_FLAG_LEARNED_INDEX if learned else 0) |
                     (HL_FLAG_JOIN_DEDUP if join_dedup else 0) |
                     (HL_FLAG_FUSED if fused else 0) |
                     (HL_FLAG_HIP_GRAPH if hip_graph else 0) |
                     (HL_FLAG_NESTED_JOINS if nested_joins else 0) |
                     (0 if levels else HL_FLAG_NO_LEVELS))
        opt.ebm_k = ebm_k
        opt.hash_load_factor = load_factor
        opt.hbm_budget_bytes = budget_bytes
        opt.sort_chunk_log2 = sort_chunk_log2
        opt.fused_capacity = fused_capacity
        opt.expand_tile = expand_tile
        opt.sort_tile = sort_tile
        opt.diff_tile = diff_tile
        opt.tail_min_bytes = tail_min_bytes
        opt.outer_slice_log2 = outer_slice_log2
        self._arena = arena  # keep the caller's tensor alive
        if arena is not None:
            opt.arena = _ptr(arena)
            opt.arena_bytes = arena.numel() * arena.element_size()
        if stream is not None:
            opt.stream = int(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)
        self._stream = stream
        h = ctypes.c_void_p()
        rc = L.hl_create(ctypes.byref(opt), ctypes.byref(h))
        if rc != HL_OK:
            raise HlError(rc, "hl_create: " + L.hl_strerror(rc).decode())
        self._h = h
        self._L = L
        self.arity = {}

    def close(self):
        if getattr(self, "_h", None):
            self._L.hl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc: int, what: str):
        if rc != HL_OK:
            raise HlError(rc, f"{what}: {self._L.hl_last_error(self._h).decode()}")

    # ------------------------------------------------------------- engine
    def declare(self, name: str, arity: int, edb: bool):
        self._check(self._L.hl_declare(self._h, name.encode(), arity, 1 if edb else 0),
                    "hl_declare")
        self.arity[name] = arity

    def load(self, name: str, rows):
        """Loads EDB rows from a numpy array or a CUDA tensor (n x arity)."""
        try:
            import torch
            is_tensor = isinstance(rows, torch.Tensor)
        except ImportError:
            is_tensor = False
        if is_tensor and rows.is_cuda:
            rows = rows.contiguous()
            if rows.element_size() != 4:
                raise TypeError("rows must be 32-bit")
            self._check(self._L.hl_load_device(self._h, name.encode(), _ptr(rows),
                                               rows.shape[0]), "hl_load_device")
            return
        arr = np.ascontiguousarray(np.asarray(rows), dtype=np.uint32)
        if arr.ndim == 1:
            arr = arr.reshape(-1, self.arity.get(name, 2))
        self._check(self._L.hl_load(self._h, name.encode(), arr.ctypes.data, arr.shape[0]),
                    "hl_load")

    def batch_layout(self, id_ranges):
        r = np.ascontiguousarray(id_ranges, dtype=np.uint32)
        self._check(self._L.hl_batch_layout(self._h, r.ctypes.data, len(r)), "hl_batch_layout")

    def load_batched(self, name: str, instances):
        """``instances``: list of (n, arity) uint32 arrays with instance-local
        ids, arity as declared for ``name``."""
        ar = self.arity.get(name, 2)
        parts = [np.asarray(x, dtype=np.uint32).reshape(-1, ar) for x in instances]
        rows = np.ascontiguousarray(np.concatenate(parts) if parts else
                                    np.zeros((0, ar), np.uint32), dtype=np.uint32)
        off = np.zeros(len(instances) + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(x) for x in parts])
        self._check(self._L.hl_load_batched(self._h, name.encode(),
                                            rows.ctypes.data if len(rows) else None,
                                            off.ctypes.data), "hl_load_batched")

    def batch_count(self, name: str, inst: int) -> int:
        n = ctypes.c_uint64()
        self._check(self._L.hl_batch_count(self._h, name.encode(), inst, ctypes.byref(n)),
                    "hl_batch_count")
        return n.value

    def fetch_batched(self, name: str, inst: int) -> np.ndarray:
        n = self.batch_count(name, inst)
        out = np.empty((n, self.arity.get(name, 2)), dtype=np.uint32)
        got = ctypes.c_uint64()
        self._check(self._L.hl_fetch_batched(self._h, name.encode(), inst,
                                             out.ctypes.data if n else None, n,
                                             ctypes.byref(got)), "hl_fetch_batched")
        return out

    def index(self, name: str, col: int):
        c = (ctypes.c_uint32 * 1)(col)
        self._check(self._L.hl_index(self._h, name.encode(), c, 1), "hl_index")

    def program(self, text: str):
        self._check(self._L.hl_program(self._h, text.encode()), "hl_program")

    def run(self) -> RunStats:
        st = Stats()
        self._check(self._L.hl_run(self._h, ctypes.byref(st)), "hl_run")
        d = st.as_dict()
        return RunStats(**d)

    def autotune(self, reps: int = 1) -> dict:
        """Measures the fixpoint under alternative settings (probe method and
        hash load factor, eager buffer growth, in-tile join dedup), keeps the
        fastest (see hl_autotune) and returns the choice."""
        t = Tuning()
        self._check(self._L.hl_autotune(self._h, reps, ctypes.byref(t)), "hl_autotune")
        return {"hash_load_factor": round(t.hash_load_factor, 3), "ebm_k": round(t.ebm_k, 3),
                "learned": bool(t.flags & HL_FLAG_LEARNED_INDEX),
                "join_dedup": bool(t.flags & HL_FLAG_JOIN_DEDUP),
                "nested_joins": bool(t.flags & HL_FLAG_NESTED_JOINS),
                "fused": bool(t.flags & (HL_FLAG_FUSED | HL_FLAG_HIP_GRAPH)),
                "hip_graph": bool(t.flags & HL_FLAG_HIP_GRAPH), "expand_tile": t.expand_tile,
                "sort_tile": t.sort_tile, "diff_tile": t.diff_tile, "trials": t.trials,
                "best_seconds": t.best_seconds, "first_seconds": t.first_seconds}

    def count(self, name: str) -> int:
        n = ctypes.c_uint64()
        self._check(self._L.hl_count(self._h, name.encode(), ctypes.byref(n)), "hl_count")
        return n.value

    def fetch(self, name: str) -> np.ndarray:
        n = self.count(name)
        ar = self.arity.get(name, 2)
        out = np.empty((n, ar), dtype=np.uint32)
        got = ctypes.c_uint64()
        self._check(self._L.hl_fetch(self._h, name.encode(), out.ctypes.data if n else None, n,
                                     ctypes.byref(got)), "hl_fetch")
        return out

    def fetch_device(self, name: str):
        import torch
        n = self.count(name)
        ar = self.arity.get(name, 2)
        out = torch.empty((n, ar), dtype=torch.int32, device="cuda")
        got = ctypes.c_uint64()
        self._check(self._L.hl_fetch_device(self._h, name.encode(), _ptr(out) if n else None, n,
                                            ctypes.byref(got)), "hl_fetch_device")
        return out

    def iteration_counts(self, name: str, which: int = 0) -> list:
        cap = 1 << 16
        buf = (ctypes.c_uint64 * cap)()
        n = ctypes.c_uint32()
        self._check(self._L.hl_iteration_counts(self._h, name.encode(), which, buf, cap,
                                                ctypes.byref(n)), "hl_iteration_counts")
        return [int(buf[i]) for i in range(min(n.value, cap))]

    def kernel_stats(self) -> dict:
        """Per-kernel (launches, ms, algorithmic bytes) of the last run; needs
        ``kernel_timing=True``."""
        out = {}
        for k, name in enumerate(KERNELS):
            n, ms, b = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_uint64()
            self._check(self._L.hl_kernel_stats(self._h, k, ctypes.byref(n), ctypes.byref(ms),
                                                ctypes.byref(b)), "hl_kernel_stats")
            out[name] = (n.value, ms.value, b.value)
        return out

    # --------------------------------------------------------- primitives
    def rule_stats(self) -> list:
        """Per rule of the program (text order), over the last run: (outputs
        of its last join, outputs of its earlier joins)."""
        out = []
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        k = 0
        while True:
            rc = self._L.hl_rule_stats(self._h, k, ctypes.byref(a), ctypes.byref(b))
            if rc == HL_E_INVALID:
                return out
            self._check(rc, "hl_rule_stats")
            out.append((a.value, b.value))
            k += 1

    def sort_keys(self, keys, bits: int = 0):
        """Sorts a CUDA int32/int64 tensor in place (unsigned order)."""
        self._check(self._L.hl_sort_keys(self._h, _ptr(keys), keys.numel(), _key_bytes(keys),
                                         bits), "hl_sort_keys")
        return keys

    def sort_keys_noalloc(self, keys, bits: int = 0):
        """sort_keys through the entry point that allocates nothing (its
        scratch is a static device array of NOALLOC_SCRATCH_BYTES)."""
        self._check(self._L.hl_sort_keys_noalloc(self._h, _ptr(keys), keys.numel(),
                                                 _key_bytes(keys), bits),
                    "hl_sort_keys_noalloc")
        return keys

    def unique_diff(self, sorted_keys, full):
        import torch
        kb = _key_bytes(sorted_keys)
        out = torch.empty_like(sorted_keys)
        n_out, n_uni = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.hl_unique_diff(self._h, _ptr(sorted_keys), sorted_keys.numel(),
                                           _ptr(full) if full.numel() else None, full.numel(),
                                           _ptr(out), ctypes.byref(n_out), ctypes.byref(n_uni),
                                           kb), "hl_unique_diff")
        return out[:n_out.value], n_uni.value

    def merge(self, a, b):
        import torch
        out = torch.empty(a.numel() + b.numel(), dtype=a.dtype, device=a.device)
        return self.merge_into(a, b, out)

    def merge_into(self, a, b, out):
        """Merges ascending a and b into out (a + b keys, caller-owned)."""
        if out.numel() != a.numel() + b.numel() or out.dtype != a.dtype:
            raise ValueError("out must hold a.numel() + b.numel() keys of a's type")
        self._check(self._L.hl_merge(self._h, _ptr(a) if a.numel() else None, a.numel(),
                                     _ptr(b) if b.numel() else None, b.numel(), _ptr(out),
                                     _key_bytes(a)), "hl_merge")
        return out

    def hisa_query(self, keys, shift: int, queries):
        import torch
        start = torch.empty(queries.numel(), dtype=torch.int64, device=keys.device)
        length = torch.empty(queries.numel(), dtype=torch.int32, device=keys.device)
        runs = ctypes.c_uint64()
        self._check(self._L.hl_hisa_query(self._h, _ptr(keys), keys.numel(), _key_bytes(keys),
                                          shift, _ptr(queries), queries.numel(), _ptr(start),
                                          _ptr(length), ctypes.byref(runs)), "hl_hisa_query")
        return start, length, runs.value


    def learned_query(self, keys, key_bits: int, queries):
        """lower_bound positions of ``queries`` in sorted ``keys`` (CUDA
        tensors of the same integer type) through a learned index."""
        import torch
        out = torch.empty(queries.numel(), dtype=torch.int32, device=keys.device)
        self._check(self._L.hl_learned_query(self._h, _ptr(keys) if keys.numel() else None,
                                             keys.numel(), _key_bytes(keys), key_bits,
                                             _ptr(queries) if queries.numel() else None,
                                             queries.numel(), _ptr(out) if queries.numel() else None),
                    "hl_learned_query")
        return out


def evaluate(program: str, edb: dict, idb: dict, **engine_kw):
    """Declares, loads, runs and fetches in one call.

    Returns ``(relations, deltas, stats)``: sorted uint32 arrays per IDB
    relation, per-iteration delta sizes, and the run's statistics."""
    with Engine(**engine_kw) as e:
        for name, rows in edb.items():
            e.declare(name, int(rows.shape[1]) if len(rows.shape) == 2 else 1, True)
        for name, ar in idb.items():
            e.declare(name, ar, False)
        for name, rows in edb.items():
            e.load(name, rows)
        e.program(program)
        st = e.run()
        rels = {n: e.fetch(n) for n in idb}
        deltas = {n: e.iteration_counts(n, 0) for n in idb}
        return rels, deltas, st

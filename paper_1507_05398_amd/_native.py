"""ctypes binding of libgreedy_code.so (argument marshalling only).

Every computation runs in the HIP library; if the library is missing this
module raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libgreedy_code.so")

GC_LEX, GC_GRAY, GC_GRLEX, GC_GREVLEX = 0, 1, 2, 3
ORDERINGS = {"lex": GC_LEX, "gray": GC_GRAY, "grlex": GC_GRLEX, "grevlex": GC_GREVLEX}
GC_OK, GC_EINVAL, GC_ECAPACITY, GC_EDEVICE, GC_ENOMEM, GC_ETIMEOUT = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {GC_EINVAL: "GC_EINVAL", GC_ECAPACITY: "GC_ECAPACITY", GC_EDEVICE: "GC_EDEVICE",
               GC_ENOMEM: "GC_ENOMEM", GC_ETIMEOUT: "GC_ETIMEOUT"}

# Every symbol declared in include/greedy_code.h.
EXPORTS = ["greedy_code_capacity", "greedy_code", "greedy_code_device", "greedy_code_device_ex",
           "gc_last_error", "gc_version"]


class GreedyCodeError(RuntimeError):
    def __init__(self, rc, message):
        super().__init__(f"{ERROR_NAMES.get(rc, rc)}: {message}")
        self.rc = rc


class GcStats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("windows", ctypes.c_uint64),
                ("resolve_rounds", ctypes.c_uint64), ("survivors", ctypes.c_uint64),
                ("checks_near", ctypes.c_uint64), ("checks_deep", ctypes.c_uint64),
                ("checks_pairs", ctypes.c_uint64), ("kernel_ms", ctypes.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class GcTuning(ctypes.Structure):
    _fields_ = [("near_depth", ctypes.c_uint64), ("target_survivors", ctypes.c_uint32),
                ("grid_blocks", ctypes.c_uint32), ("resolve_mode", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


_lib = None


def load():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY):
        raise ImportError(f"{LIBRARY} is missing: build it with paper_1507_05398_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIBRARY)
    u32p, u64p, vp = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p
    lib.greedy_code_capacity.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.greedy_code_capacity.restype = ctypes.c_uint64
    lib.greedy_code.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p, u64p]
    lib.greedy_code.restype = ctypes.c_int
    lib.greedy_code_device.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                       ctypes.c_uint64, vp, vp]
    lib.greedy_code_device.restype = ctypes.c_int
    lib.greedy_code_device_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                          ctypes.c_uint64, vp, vp, ctypes.POINTER(GcTuning),
                                          ctypes.POINTER(GcStats)]
    lib.greedy_code_device_ex.restype = ctypes.c_int
    lib.gc_last_error.argtypes = []
    lib.gc_last_error.restype = ctypes.c_char_p
    lib.gc_version.argtypes = []
    lib.gc_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != GC_OK:
        raise GreedyCodeError(rc, load().gc_last_error().decode())


def _ordering(ordering):
    return ORDERINGS[ordering] if isinstance(ordering, str) else int(ordering)


def greedy_code_capacity(n: int, d: int) -> int:
    return int(load().greedy_code_capacity(n, d))


def gc_last_error() -> str:
    return load().gc_last_error().decode()


def gc_version() -> str:
    return load().gc_version().decode()


def greedy_code(n: int, d: int, ordering, capacity: int = None) -> np.ndarray:
    """Host-memory entry point: returns the code as a uint32 array in
    acceptance order."""
    cap = greedy_code_capacity(n, d) if capacity is None else int(capacity)
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    count = ctypes.c_uint64(cap)
    rc = load().greedy_code(n, d, _ordering(ordering),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(count))
    _check(rc)
    return out[: count.value].copy()


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def greedy_code_device(n: int, d: int, ordering, words, count, stream=None) -> None:
    """Device entry point on torch tensors: ``words`` int32/uint32 CUDA tensor
    (capacity = numel), ``count`` one-element int64 CUDA tensor."""
    rc = load().greedy_code_device(n, d, _ordering(ordering), ctypes.c_void_p(words.data_ptr()),
                                   words.numel(), ctypes.c_void_p(count.data_ptr()),
                                   _stream_ptr(stream))
    _check(rc)


def greedy_code_device_ex(n: int, d: int, ordering, words, count, stream=None, near_depth=0,
                          target_survivors=0, grid_blocks=0, resolve_mode=0) -> dict:
    """As greedy_code_device, with tuning knobs; returns the work counters."""
    tuning = GcTuning(near_depth, target_survivors, grid_blocks, resolve_mode, 0)
    stats = GcStats()
    rc = load().greedy_code_device_ex(n, d, _ordering(ordering), ctypes.c_void_p(words.data_ptr()),
                                      words.numel(), ctypes.c_void_p(count.data_ptr()),
                                      _stream_ptr(stream), ctypes.byref(tuning), ctypes.byref(stats))
    _check(rc)
    return stats.as_dict()


def device_code(n: int, d: int, ordering, device="cuda", **tuning):
    """Convenience: allocate the output on the device, run, return
    (words tensor trimmed to |C|, stats)."""
    import torch
    cap = greedy_code_capacity(n, d)
    words = torch.empty(cap, dtype=torch.int32, device=device)
    count = torch.zeros(1, dtype=torch.int64, device=device)
    stats = greedy_code_device_ex(n, d, ordering, words, count, **tuning)
    m = int(count.item())
    return words[:m], stats

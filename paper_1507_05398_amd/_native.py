"""ctypes binding of libgreedy_code.so (argument marshalling only).

Every computation runs in the HIP library; if the library is missing this
module raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libgreedy_code.so")

GC_LEX, GC_GRAY, GC_GRLEX, GC_GREVLEX, GC_BORDER = 0, 1, 2, 3, 4
ORDERINGS = {"lex": GC_LEX, "gray": GC_GRAY, "grlex": GC_GRLEX, "grevlex": GC_GREVLEX, "border": GC_BORDER}
GC_OK, GC_EINVAL, GC_ECAPACITY, GC_EDEVICE, GC_ENOMEM, GC_ETIMEOUT, GC_EBUSY = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {GC_EINVAL: "GC_EINVAL", GC_ECAPACITY: "GC_ECAPACITY", GC_EDEVICE: "GC_EDEVICE",
               GC_ENOMEM: "GC_ENOMEM", GC_ETIMEOUT: "GC_ETIMEOUT", GC_EBUSY: "GC_EBUSY"}
GC_JOB_WAITING, GC_JOB_ADMITTED, GC_JOB_DONE, GC_JOB_FAILED = 0, 1, 2, 3

# Every symbol declared in include/greedy_code.h.
EXPORTS = ["greedy_code_capacity", "greedy_code", "greedy_code_device", "greedy_code_device_ex",
           "greedy_code_device_noalloc", "greedy_code_cw64", "gc_problem_init", "gc_problem_positions",
           "gc_problem_capacity", "greedy_code_problem", "greedy_code_problem_device",
           "greedy_code_batch", "greedy_code_tune", "greedy_code_tune_reset",
           "greedy_code_batch_tune", "gc_batch_graph_create", "gc_batch_graph_launch",
           "gc_batch_graph_results", "gc_batch_graph_destroy", "gc_probe_block_loop", "gc_probe_matrix_loop", "gc_probe_barrier",
           "gc_server_create", "gc_server_submit", "gc_server_poll",
           "gc_server_words", "gc_server_fetch", "gc_server_stats", "gc_server_release",
           "gc_server_drain", "gc_server_destroy", "gc_last_error", "gc_version"]


class GreedyCodeError(RuntimeError):
    def __init__(self, rc, message):
        super().__init__(f"{ERROR_NAMES.get(rc, rc)}: {message}")
        self.rc = rc


class GcStats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("windows", ctypes.c_uint64),
                ("resolve_rounds", ctypes.c_uint64), ("survivors", ctypes.c_uint64),
                ("checks_near", ctypes.c_uint64), ("checks_deep", ctypes.c_uint64),
                ("checks_pairs", ctypes.c_uint64), ("kernel_ms", ctypes.c_float),
                ("near_ms", ctypes.c_double), ("survivors_ms", ctypes.c_double),
                ("resolve_ms", ctypes.c_double), ("deep_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class GcTuning(ctypes.Structure):
    _fields_ = [("near_depth", ctypes.c_uint64), ("target_survivors", ctypes.c_uint32),
                ("grid_blocks", ctypes.c_uint32), ("resolve_mode", ctypes.c_uint32),
                ("deep_tile", ctypes.c_uint32), ("valu_screen", ctypes.c_uint32)]


class GcProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("d", ctypes.c_int), ("ordering", ctypes.c_int),
                ("weight", ctypes.c_int), ("self_orthogonal", ctypes.c_int),
                ("basis", ctypes.c_uint32 * 32), ("start", ctypes.c_uint64), ("stop", ctypes.c_uint64),
                ("prefix", ctypes.c_uint64)]


class GcJob(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("d", ctypes.c_int), ("ordering", ctypes.c_int),
                ("d_words", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("d_count", ctypes.c_void_p), ("status", ctypes.c_int), ("count", ctypes.c_uint64),
                ("device_ms", ctypes.c_double)]


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
    lib.greedy_code_device_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                               ctypes.c_uint64, vp, vp]
    lib.greedy_code_device_noalloc.restype = ctypes.c_int
    lib.greedy_code_cw64.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_uint64, vp, vp]
    lib.greedy_code_cw64.restype = ctypes.c_int
    pp = ctypes.POINTER(GcProblem)
    lib.gc_problem_init.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.gc_problem_init.restype = ctypes.c_int
    lib.gc_problem_positions.argtypes = [pp]
    lib.gc_problem_positions.restype = ctypes.c_uint64
    lib.gc_problem_capacity.argtypes = [pp]
    lib.gc_problem_capacity.restype = ctypes.c_uint64
    lib.greedy_code_problem.argtypes = [pp, u32p, u64p]
    lib.greedy_code_problem.restype = ctypes.c_int
    lib.greedy_code_problem_device.argtypes = [pp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(GcTuning),
                                               ctypes.POINTER(GcStats)]
    lib.greedy_code_problem_device.restype = ctypes.c_int
    lib.greedy_code_batch.argtypes = [ctypes.POINTER(GcJob), ctypes.c_int, ctypes.c_int, vp,
                                      ctypes.POINTER(ctypes.c_float)]
    lib.greedy_code_batch.restype = ctypes.c_int
    lib.greedy_code_tune.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                     ctypes.POINTER(GcTuning), ctypes.POINTER(ctypes.c_float)]
    lib.greedy_code_tune.restype = ctypes.c_int
    lib.greedy_code_tune_reset.argtypes = []
    lib.greedy_code_tune_reset.restype = None
    lib.greedy_code_batch_tune.argtypes = [ctypes.POINTER(GcJob), ctypes.c_int, vp,
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
    lib.greedy_code_batch_tune.restype = ctypes.c_int
    lib.gc_batch_graph_create.argtypes = [ctypes.POINTER(GcJob), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_void_p)]
    lib.gc_batch_graph_create.restype = ctypes.c_int
    lib.gc_batch_graph_launch.argtypes = [vp, vp]
    lib.gc_batch_graph_launch.restype = ctypes.c_int
    lib.gc_batch_graph_results.argtypes = [vp, ctypes.POINTER(GcJob)]
    lib.gc_batch_graph_results.restype = ctypes.c_int
    lib.gc_batch_graph_destroy.argtypes = [vp]
    lib.gc_batch_graph_destroy.restype = ctypes.c_int
    lib.gc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.gc_server_create.restype = ctypes.c_int
    lib.gc_server_submit.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p]
    lib.gc_server_submit.restype = ctypes.c_int
    lib.gc_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), u64p]
    lib.gc_server_poll.restype = ctypes.c_int
    lib.gc_server_words.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p), u64p]
    lib.gc_server_words.restype = ctypes.c_int
    lib.gc_server_fetch.argtypes = [vp, ctypes.c_uint64, u32p, ctypes.c_uint64, u64p]
    lib.gc_server_fetch.restype = ctypes.c_int
    lib.gc_server_stats.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(GcStats),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.gc_server_stats.restype = ctypes.c_int
    lib.gc_server_release.argtypes = [vp, ctypes.c_uint64]
    lib.gc_server_release.restype = ctypes.c_int
    lib.gc_server_drain.argtypes = [vp, ctypes.c_int]
    lib.gc_server_drain.restype = ctypes.c_int
    lib.gc_server_destroy.argtypes = [vp]
    lib.gc_server_destroy.restype = ctypes.c_int
    lib.gc_probe_block_loop.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.gc_probe_block_loop.restype = ctypes.c_int
    lib.gc_probe_matrix_loop.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.gc_probe_matrix_loop.restype = ctypes.c_int
    lib.gc_probe_barrier.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.gc_probe_barrier.restype = ctypes.c_int
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


def greedy_code_device_noalloc(n: int, d: int, ordering, words, count, stream=None) -> None:
    """As greedy_code_device, through the entry point that allocates nothing
    (its workspace is a fixed device array; overlapping calls on one device
    race)."""
    rc = load().greedy_code_device_noalloc(n, d, _ordering(ordering), ctypes.c_void_p(words.data_ptr()),
                                           words.numel(), ctypes.c_void_p(count.data_ptr()),
                                           _stream_ptr(stream))
    _check(rc)


def greedy_code_cw64(n: int, w: int, d: int, words, count, stream=None) -> None:
    """Constant-weight greedy code over uint64 words (n <= 64): the weight-w
    vectors in increasing value; ``words`` is a device int64/uint64 tensor of
    capacity words, ``count`` a device int64 tensor of one element."""
    rc = load().greedy_code_cw64(n, w, d, ctypes.c_void_p(words.data_ptr()), words.numel(),
                                 ctypes.c_void_p(count.data_ptr()), _stream_ptr(stream))
    _check(rc)


def greedy_code_device_ex(n: int, d: int, ordering, words, count, stream=None, near_depth=0,
                          target_survivors=0, grid_blocks=0, resolve_mode=0, deep_tile=0,
                          valu_screen=0) -> dict:
    """As greedy_code_device, with tuning knobs; returns the work counters."""
    tuning = GcTuning(near_depth, target_survivors, grid_blocks, resolve_mode, deep_tile, valu_screen)
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


def problem(n: int, d: int, ordering, weight: int = -1, self_orthogonal: bool = False, basis=None,
            start: int = 0, stop: int = 0, prefix: int = 0) -> GcProblem:
    """A gc_problem: ordering (name or GC_*; "border" needs `basis` = b_1..b_n),
    constant weight (-1: all weights), self-orthogonality, and the screened
    position range [start, stop) after `prefix` words (stop 0 = the end)."""
    p = GcProblem()
    _check(load().gc_problem_init(ctypes.byref(p), n, d, _ordering(ordering)))
    p.weight = int(weight)
    p.self_orthogonal = int(bool(self_orthogonal))
    if basis is not None:
        b = [int(v) for v in basis]
        if len(b) > 32:
            raise ValueError("at most 32 basis vectors")
        for j, v in enumerate(b):
            p.basis[j] = v
    p.start, p.stop, p.prefix = int(start), int(stop), int(prefix)
    return p


def problem_positions(p: GcProblem) -> int:
    """Number of candidates of the problem's walk (0 if the problem is invalid)."""
    return int(load().gc_problem_positions(ctypes.byref(p)))


def problem_capacity(p: GcProblem) -> int:
    """Capacity in words (prefix included) that always suffices (0 if invalid)."""
    return int(load().gc_problem_capacity(ctypes.byref(p)))


def greedy_code_problem(p: GcProblem, prefix_words=None, capacity: int = None) -> np.ndarray:
    """Host-memory entry point of a problem: returns the whole code (the
    prefix words first) as a uint32 array."""
    cap = problem_capacity(p) if capacity is None else int(capacity)
    if cap == 0 and problem_positions(p) == 0 and p.prefix == 0:
        _check(load().greedy_code_problem(ctypes.byref(p), None, ctypes.byref(ctypes.c_uint64(0))))
        return np.zeros(0, dtype=np.uint32)
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    if p.prefix:
        out[: p.prefix] = np.asarray(prefix_words, dtype=np.uint32)[: p.prefix]
    count = ctypes.c_uint64(cap)
    rc = load().greedy_code_problem(ctypes.byref(p), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    ctypes.byref(count))
    _check(rc)
    return out[: count.value].copy()


def greedy_code_problem_device(p: GcProblem, words, count, stream=None, near_depth=0, target_survivors=0,
                               grid_blocks=0, resolve_mode=0, deep_tile=0, valu_screen=0) -> dict:
    """Device entry point of a problem on torch tensors: ``words`` (capacity =
    numel, holding the prefix words), ``count`` one-element int64 tensor.
    Returns the work counters."""
    tuning = GcTuning(near_depth, target_survivors, grid_blocks, resolve_mode, deep_tile, valu_screen)
    stats = GcStats()
    rc = load().greedy_code_problem_device(ctypes.byref(p), ctypes.c_void_p(words.data_ptr()), words.numel(),
                                           ctypes.c_void_p(count.data_ptr()), _stream_ptr(stream),
                                           ctypes.byref(tuning), ctypes.byref(stats))
    _check(rc)
    return stats.as_dict()


def device_problem_code(p: GcProblem, device="cuda", prefix_words=None, **tuning):
    """Convenience: allocate the output on the device (capacity from the
    problem), copy the prefix words in, run, return (words tensor trimmed to
    |C|, stats)."""
    import torch
    cap = max(problem_capacity(p), 1)
    words = torch.zeros(cap, dtype=torch.int32, device=device)
    if p.prefix:
        pw = np.asarray(prefix_words, dtype=np.uint32)[: p.prefix].view(np.int32)
        words[: p.prefix] = torch.from_numpy(pw.copy()).to(device)
    count = torch.zeros(1, dtype=torch.int64, device=device)
    stats = greedy_code_problem_device(p, words, count, **tuning)
    m = int(count.item())
    return words[:m], stats


def greedy_code_batch(instances, teams=0, stream=None, device="cuda"):
    """Build several codes in one persistent launch.  ``instances``: list of
    (n, d, ordering).  Returns (list of uint32 CUDA tensors trimmed to |C|,
    list of per-job dicts with status/count/device_ms, kernel_ms)."""
    import torch
    jobs = (GcJob * len(instances))()
    bufs = []
    for i, (n, d, o) in enumerate(instances):
        cap = greedy_code_capacity(n, d)
        w = torch.empty(cap, dtype=torch.int32, device=device)
        c = torch.zeros(1, dtype=torch.int64, device=device)
        bufs.append((w, c))
        jobs[i].n, jobs[i].d, jobs[i].ordering = n, d, _ordering(o)
        jobs[i].d_words, jobs[i].capacity, jobs[i].d_count = w.data_ptr(), cap, c.data_ptr()
    ms = ctypes.c_float()
    rc = load().greedy_code_batch(jobs, len(instances), teams, _stream_ptr(stream), ctypes.byref(ms))
    _check(rc)
    out = [w[: int(jobs[i].count)] for i, (w, _) in enumerate(bufs)]
    info = [{"status": jobs[i].status, "count": int(jobs[i].count), "device_ms": jobs[i].device_ms}
            for i in range(len(instances))]
    return out, info, ms.value


def greedy_code_tune(n: int, d: int, ordering, stream=None) -> dict:
    """Autotune (n, d, ordering) on the device; the choice is remembered by the
    library for later builds of that instance.  Returns the chosen tuning and
    its device time."""
    best, ms = GcTuning(), ctypes.c_float()
    _check(load().greedy_code_tune(n, d, _ordering(ordering), _stream_ptr(stream), ctypes.byref(best),
                                   ctypes.byref(ms)))
    return {"near_depth": best.near_depth, "target_survivors": best.target_survivors,
            "grid_blocks": best.grid_blocks, "resolve_mode": best.resolve_mode, "deep_tile": best.deep_tile,
            "valu_screen": best.valu_screen, "ms": ms.value}


def greedy_code_tune_reset() -> None:
    load().greedy_code_tune_reset()


def probe_block_loop(wgs_per_cu: int = 1, iters: int = 4096) -> float:
    """Distance checks per second of the screen's block loop alone."""
    v = ctypes.c_double()
    _check(load().gc_probe_block_loop(wgs_per_cu, iters, ctypes.byref(v)))
    return v.value


def probe_matrix_loop(iters: int = 2048) -> float:
    """Distance checks per second of the matrix-core screen's segment loop alone."""
    v = ctypes.c_double()
    _check(load().gc_probe_matrix_loop(iters, ctypes.byref(v)))
    return v.value


def probe_barrier(iters: int = 20000) -> float:
    """Microseconds per team-wide barrier (one team spanning the GPU)."""
    v = ctypes.c_double()
    _check(load().gc_probe_barrier(iters, ctypes.byref(v)))
    return v.value


class BatchPlan:
    """Reusable batch: output buffers and the job table are allocated once,
    so repeated runs time only the launch."""

    def __init__(self, instances, device="cuda"):
        import torch
        self.instances = list(instances)
        self.jobs = (GcJob * len(self.instances))()
        self.bufs = []
        for i, (n, d, o) in enumerate(self.instances):
            cap = greedy_code_capacity(n, d)
            w = torch.empty(cap, dtype=torch.int32, device=device)
            c = torch.zeros(1, dtype=torch.int64, device=device)
            self.bufs.append((w, c))
            j = self.jobs[i]
            j.n, j.d, j.ordering = n, d, _ordering(o)
            j.d_words, j.capacity, j.d_count = w.data_ptr(), cap, c.data_ptr()

    def run(self, teams=0, stream=None) -> float:
        """One launch over every job; returns the device time in ms."""
        ms = ctypes.c_float()
        rc = load().greedy_code_batch(self.jobs, len(self.instances), teams, _stream_ptr(stream),
                                      ctypes.byref(ms))
        _check(rc)
        return ms.value

    def tune(self, stream=None):
        """Try 1, 2, 4 and 8 teams; returns (best team count, its device ms)."""
        best, ms = ctypes.c_int(), ctypes.c_float()
        _check(load().greedy_code_batch_tune(self.jobs, len(self.instances), _stream_ptr(stream),
                                             ctypes.byref(best), ctypes.byref(ms)))
        return best.value, ms.value

    def graph(self, teams=0):
        """Capture this batch into a replayable HIP graph (BatchGraph)."""
        return BatchGraph(self, teams)

    def results(self):
        """Per job: uint32 CUDA tensor trimmed to |C|."""
        return [w[: int(self.jobs[i].count)] for i, (w, _) in enumerate(self.bufs)]

    def info(self):
        return [{"status": self.jobs[i].status, "count": int(self.jobs[i].count),
                 "device_ms": self.jobs[i].device_ms} for i in range(len(self.instances))]


class BatchGraph:
    """A BatchPlan's launch captured into a HIP graph: launch() enqueues a
    replay, wait() synchronizes the stream and collects the job outputs."""

    def __init__(self, plan, teams=0):
        self.plan = plan
        self._h = ctypes.c_void_p()
        _check(load().gc_batch_graph_create(plan.jobs, len(plan.instances), teams, ctypes.byref(self._h)))

    def launch(self, stream=None):
        self._stream = stream
        _check(load().gc_batch_graph_launch(self._h, _stream_ptr(stream)))

    def wait(self):
        import torch
        s = getattr(self, "_stream", None)
        (s or torch.cuda.current_stream()).synchronize()
        _check(load().gc_batch_graph_results(self._h, self.plan.jobs))

    def close(self):
        if self._h:
            load().gc_batch_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Thin wrapper of the gc_server_* entry points."""

    def __init__(self, arena_bytes=1 << 30, teams=8):
        self._h = ctypes.c_void_p()
        _check(load().gc_server_create(arena_bytes, teams, ctypes.byref(self._h)))

    def submit(self, n, d, ordering) -> int:
        t = ctypes.c_uint64()
        _check(load().gc_server_submit(self._h, n, d, _ordering(ordering), ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        st, cnt = ctypes.c_int(), ctypes.c_uint64()
        _check(load().gc_server_poll(self._h, ticket, ctypes.byref(st), ctypes.byref(cnt)))
        return st.value, cnt.value

    def fetch(self, ticket) -> np.ndarray:
        st, cnt = self.poll(ticket)
        if st == GC_JOB_FAILED:
            _check(load().gc_server_words(self._h, ticket, ctypes.byref(ctypes.c_void_p()),
                                          ctypes.byref(ctypes.c_uint64())))
        out = np.zeros(max(cnt, 1), dtype=np.uint32)
        got = ctypes.c_uint64()
        _check(load().gc_server_fetch(self._h, ticket,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), out.size,
                                      ctypes.byref(got)))
        return out[: got.value].copy()

    def stats(self, ticket) -> dict:
        st, ms = GcStats(), ctypes.c_double()
        _check(load().gc_server_stats(self._h, ticket, ctypes.byref(st), ctypes.byref(ms)))
        d = st.as_dict()
        d["device_ms"] = ms.value
        return d

    def release(self, ticket):
        _check(load().gc_server_release(self._h, ticket))

    def drain(self, timeout_ms=-1):
        _check(load().gc_server_drain(self._h, timeout_ms))

    def close(self):
        if self._h:
            load().gc_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates arguments before touching the device."""
import ctypes
import math
import os
import re

import pytest

import paper_1507_05398_amd as gc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "greedy_code.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) -
                  {"if", "sizeof", "defined"})


def test_header_symbols_are_exported():
    lib = ctypes.CDLL(gc._native.LIBRARY)
    declared = header_functions()
    assert set(declared) == set(gc.EXPORTS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version():
    assert "gfx950" in gc.gc_version()


def ball(n, r):
    return sum(math.comb(n, i) for i in range(r + 1))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 15, 16, 20, 23, 24, 28, 32])
def test_capacity_is_sphere_packing_bound(n):
    for d in range(1, n + 3):
        cap = gc.greedy_code_capacity(n, d)
        if d == 1:
            assert cap == 2 ** n
        elif d > n:
            assert cap == 1
        elif d % 2:
            assert cap == 2 ** n // ball(n, (d - 1) // 2)
        else:
            assert cap == 2 ** (n - 1) // ball(n - 1, (d - 2) // 2)


def test_capacity_tight_cases():
    # perfect codes and the Golay codes meet the bound exactly
    assert gc.greedy_code_capacity(7, 3) == 16
    assert gc.greedy_code_capacity(15, 3) == 2048
    assert gc.greedy_code_capacity(23, 7) == 4096
    assert gc.greedy_code_capacity(24, 8) == 4096


@pytest.mark.parametrize("args", [(0, 3, 0), (33, 3, 0), (5, 0, 0), (5, -2, 0), (5, 3, 4), (5, 3, -1)])
def test_invalid_arguments_rejected_before_device(args):
    assert gc.greedy_code_capacity(args[0], args[1]) == 0 or args[2] not in range(4)
    with pytest.raises(gc.GreedyCodeError) as e:
        gc.greedy_code(*args, capacity=16)
    assert e.value.rc == gc.GC_EINVAL
    lib = gc.load()
    rc = lib.greedy_code_device(args[0], args[1], args[2], ctypes.c_void_p(16), 16,
                                ctypes.c_void_p(16), None)
    assert rc == gc.GC_EINVAL
    assert gc.gc_last_error()


def test_null_and_alignment_rejected():
    lib = gc.load()
    assert lib.greedy_code_device(5, 3, 0, None, 16, ctypes.c_void_p(64), None) == gc.GC_EINVAL
    assert lib.greedy_code_device(5, 3, 0, ctypes.c_void_p(64), 16, None, None) == gc.GC_EINVAL
    assert lib.greedy_code_device(5, 3, 0, ctypes.c_void_p(68), 16, ctypes.c_void_p(64), None) == gc.GC_EINVAL
    count = ctypes.c_uint64(4)
    assert lib.greedy_code(5, 3, 0, None, ctypes.byref(count)) == gc.GC_EINVAL


def test_batch_argument_validation_without_device():
    lib = gc.load()
    jobs = (gc._native.GcJob * 2)()
    jobs[0].n, jobs[0].d, jobs[0].ordering, jobs[0].d_words, jobs[0].capacity = 5, 3, 0, 64, 16
    jobs[1].n, jobs[1].d, jobs[1].ordering, jobs[1].d_words, jobs[1].capacity = 5, 0, 0, 64, 16
    assert lib.greedy_code_batch(jobs, 2, 1, None, None) == gc.GC_EINVAL
    jobs[1].d, jobs[1].d_words = 3, 68   # misaligned
    assert lib.greedy_code_batch(jobs, 2, 1, None, None) == gc.GC_EINVAL
    assert lib.greedy_code_batch(None, 3, 1, None, None) == gc.GC_EINVAL


def test_server_create_fails_cleanly_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    assert gc.load().gc_server_create(1 << 20, 8, ctypes.byref(h)) != gc.GC_OK
    assert gc.load().gc_server_create(1 << 20, 3, ctypes.byref(h)) == gc.GC_EINVAL


def test_tuner_argument_validation_without_device():
    lib = gc.load()
    best, ms = gc._native.GcTuning(), ctypes.c_float()
    for args in [(0, 3, 0), (5, 0, 0), (5, 3, 7)]:
        assert lib.greedy_code_tune(*args, None, ctypes.byref(best), ctypes.byref(ms)) == gc.GC_EINVAL
    assert lib.greedy_code_tune(5, 3, 0, None, None, None) == gc.GC_EINVAL
    # Degenerate d: the code needs no search, so there is nothing to tune.
    best.near_depth = 99
    assert lib.greedy_code_tune(5, 1, 0, None, ctypes.byref(best), ctypes.byref(ms)) == gc.GC_OK
    assert best.near_depth == 0 and ms.value == 0.0
    assert lib.greedy_code_tune(5, 6, 2, None, ctypes.byref(best), None) == gc.GC_OK
    lib.greedy_code_tune_reset()
    jobs = (gc._native.GcJob * 1)()
    assert lib.greedy_code_batch_tune(jobs, 1, None, None, None) == gc.GC_EINVAL


def test_batch_graph_argument_validation_without_device():
    lib = gc.load()
    h = ctypes.c_void_p()
    jobs = (gc._native.GcJob * 1)()
    assert lib.gc_batch_graph_create(jobs, 0, 1, ctypes.byref(h)) == gc.GC_EINVAL
    assert lib.gc_batch_graph_create(None, 1, 1, ctypes.byref(h)) == gc.GC_EINVAL
    assert lib.gc_batch_graph_create(jobs, 1, 3, ctypes.byref(h)) == gc.GC_EINVAL
    jobs[0].n, jobs[0].d, jobs[0].ordering, jobs[0].d_words, jobs[0].capacity = 5, 0, 0, 64, 16
    assert lib.gc_batch_graph_create(jobs, 1, 1, ctypes.byref(h)) == gc.GC_EINVAL
    assert lib.gc_batch_graph_create(jobs, 1, 1, None) == gc.GC_EINVAL
    assert lib.gc_batch_graph_launch(None, None) == gc.GC_EINVAL
    assert lib.gc_batch_graph_results(None, jobs) == gc.GC_EINVAL
    assert lib.gc_batch_graph_destroy(None) == gc.GC_OK


def test_empty_batch_is_a_no_op():
    lib = gc.load()
    ms = ctypes.c_float(-1.0)
    assert lib.greedy_code_batch(None, 0, 0, None, ctypes.byref(ms)) == gc.GC_OK

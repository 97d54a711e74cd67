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


# ---- generalized problems (B-ordering, constant weight, self-orthogonal, resume)

def test_problem_positions():
    assert gc.problem_positions(gc.problem(10, 3, "lex")) == 1024
    assert gc.problem_positions(gc.problem(10, 3, "grlex", self_orthogonal=True)) == 512
    assert gc.problem_positions(gc.problem(10, 3, "gray", self_orthogonal=True)) == 512
    assert gc.problem_positions(gc.problem(10, 4, "lex", weight=3)) == math.comb(10, 3)
    assert gc.problem_positions(gc.problem(10, 4, "grevlex", weight=4, self_orthogonal=True)) == math.comb(10, 4)
    assert gc.problem_positions(gc.problem(10, 4, "lex", weight=3, self_orthogonal=True)) == 0
    basis = [1 << j for j in range(12)]
    assert gc.problem_positions(gc.problem(12, 3, "border", basis=basis)) == 4096


def johnson(n, e, w):
    w = min(w, n - w)
    if w < e:
        return 1
    return min(n * johnson(n - 1, e, w - 1) // w, math.comb(n, w))


def test_problem_capacity_formulas():
    assert gc.problem_capacity(gc.problem(15, 3, "lex")) == gc.greedy_code_capacity(15, 3)
    assert gc.problem_capacity(gc.problem(12, 1, "gray")) == 4096
    assert gc.problem_capacity(gc.problem(16, 6, "lex", weight=5)) == johnson(16, 3, 5) == 48
    assert gc.problem_capacity(gc.problem(16, 5, "lex", weight=5)) == 48   # odd d: even distances
    assert gc.problem_capacity(gc.problem(24, 8, "lex", self_orthogonal=True)) == 4096
    assert gc.problem_capacity(gc.problem(20, 1, "lex", self_orthogonal=True)) == 1024
    # never more than prefix + screened positions
    assert gc.problem_capacity(gc.problem(16, 3, "lex", start=100, stop=110, prefix=7)) == 17


def test_problem_capacity_holds_the_oracle_codes():
    """The capacity bound is a bound: every code the oracle builds fits."""
    import numpy as np

    import oracle
    for n in range(4, 12):
        for d in range(1, n + 1):
            for w in range(0, n + 1, 3):
                for o in ("lex", "grevlex"):
                    cand = oracle.weight_class(n, w, oracle.ORDERINGS[o])
                    words, _, _ = oracle.greedy_list(n, d, cand)
                    assert len(words) <= gc.problem_capacity(gc.problem(n, d, o, weight=w)), (n, d, w, o)
            table = oracle.order_table(n, oracle.LEX)
            words, _, _ = oracle.greedy_list(n, d, table, self_orth=True)
            assert len(words) <= gc.problem_capacity(gc.problem(n, d, "lex", self_orthogonal=True)), (n, d)
            assert np.all(np.bitwise_count(words) % 2 == 0)


@pytest.mark.parametrize("kw,what", [
    (dict(n=8, d=3, ordering="gray", weight=3), "constant weight"),
    (dict(n=8, d=3, ordering="border", weight=3, basis=[1 << j for j in range(8)]), "constant weight"),
    (dict(n=8, d=3, ordering="border", self_orthogonal=True, basis=[1 << j for j in range(8)]), "self_orthogonal"),
    (dict(n=8, d=3, ordering="border", basis=[1, 2, 3, 8, 16, 32, 64, 128]), "depends"),
    (dict(n=8, d=3, ordering="border", basis=[1, 2, 4, 8, 16, 32, 64, 256]), "bits above"),
    (dict(n=8, d=3, ordering="lex", weight=9), "weight"),
    (dict(n=8, d=3, ordering="lex", stop=257), "stop"),
    (dict(n=8, d=3, ordering="lex", start=20, stop=10), "start"),
])
def test_problem_validation(kw, what):
    n, d, o = kw.pop("n"), kw.pop("d"), kw.pop("ordering")
    p = gc.problem(n, d, o, **kw)
    assert gc.problem_positions(p) == 0 and gc.problem_capacity(p) == 0
    assert what in gc.gc_last_error()
    with pytest.raises(gc.GreedyCodeError) as e:
        gc.greedy_code_problem(p, capacity=16)
    assert e.value.rc == gc.GC_EINVAL


def test_self_orthogonal_flag_must_be_boolean():
    p = gc.problem(8, 3, "lex")
    p.self_orthogonal = 2
    assert gc.problem_capacity(p) == 0


def test_plain_entry_points_reject_border():
    with pytest.raises(gc.GreedyCodeError) as e:
        gc.greedy_code(8, 3, "border", capacity=16)
    assert e.value.rc == gc.GC_EINVAL


def test_tuning_deep_tile_is_validated():
    lib = gc.load()
    t = gc._native.GcTuning(0, 0, 0, 0, 300)
    rc = lib.greedy_code_device_ex(8, 3, 0, ctypes.c_void_p(64), 16, ctypes.c_void_p(64), None,
                                   ctypes.byref(t), None)
    assert rc == gc.GC_EINVAL and "deep_tile" in gc.gc_last_error()


def test_tuning_valu_screen_is_validated():
    lib = gc.load()
    t = gc._native.GcTuning(0, 0, 0, 0, 0, 2)
    rc = lib.greedy_code_device_ex(8, 3, 0, ctypes.c_void_p(64), 16, ctypes.c_void_p(64), None,
                                   ctypes.byref(t), None)
    assert rc == gc.GC_EINVAL and "valu_screen" in gc.gc_last_error()


@pytest.mark.parametrize("n,w,d,words,cap", [
    (0, 1, 2, 64, 16), (65, 1, 2, 64, 16),       # length outside 1..64
    (35, -1, 2, 64, 16), (35, 36, 2, 64, 16),     # weight outside 0..n
    (35, 3, 0, 64, 16),                           # d below 1
    (35, 3, 4, None, 16),                         # no output with room for words
    (35, 3, 4, 68, 16),                           # output not 8-byte aligned
    (64, 32, 4, 64, 16), (40, 20, 4, 64, 16),     # more than 2^32 candidates
])
def test_cw64_arguments_rejected_before_device(n, w, d, words, cap):
    lib = gc.load()
    ptr = None if words is None else ctypes.c_void_p(words)
    assert lib.greedy_code_cw64(n, w, d, ptr, cap, None, None) == gc.GC_EINVAL
    assert gc.gc_last_error()


def test_header_is_plain_c(tmp_path):
    # The boundary is a C ABI: the header compiles as strict C99 (plain
    # pointers and sizes, no C++ or framework types).
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "use_header.c"
    src.write_text('#include "greedy_code.h"\nint main(void) { return GC_OK; }\n')
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([gcc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", include,
                        "-c", str(src), "-o", str(tmp_path / "use_header.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

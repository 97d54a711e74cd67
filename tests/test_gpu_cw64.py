"""Constant-weight codes over uint64 words (n up to 64) on the GPU against the
oracle: the same words in the same order as the oracle's plain scan over the
weight-w vectors in increasing value (bit-exact)."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
gc = pytest.importorskip("paper_1507_05398_amd")


def gpu_code(n, w, d, cap=None):
    cap = math.comb(n, w) if cap is None else cap
    words = torch.zeros(cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    gc.greedy_code_cw64(n, w, d, words, count)
    m = int(count.item())
    return words[:m].cpu().numpy().view(np.uint64)


def oracle_code(n, w, d):
    return oracle.greedy_list64(n, d, oracle.weight_class64(n, w))[0]


@pytest.mark.parametrize("n,w,d", [
    (33, 5, 6), (34, 0, 3), (34, 34, 3), (35, 1, 2), (35, 2, 4), (35, 3, 1), (35, 3, 2), (35, 3, 4),
    (35, 4, 6), (35, 5, 8), (36, 4, 4), (40, 3, 6), (63, 3, 4), (64, 1, 2), (64, 2, 4), (20, 5, 4),
])
def test_cw64_matches_the_oracle(n, w, d):
    print(f"cw64 n={n} w={w} d={d}", flush=True)
    got = gpu_code(n, w, d)
    ref = oracle_code(n, w, d)
    assert got.size == ref.size
    assert np.array_equal(got, ref)


def test_cw64_triple_system_at_63():
    got = gpu_code(63, 3, 4)
    assert got.size == 63 * 62 // 6
    assert oracle.verify_certificate64(63, 4, oracle.weight_class64(63, 3), got) == 0


def test_cw64_capacity_error_keeps_the_prefix():
    ref = oracle_code(35, 3, 4)
    cap = ref.size // 2
    words = torch.zeros(cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(gc.GreedyCodeError) as e:
        gc.greedy_code_cw64(35, 3, 4, words, count)
    assert e.value.rc == gc.GC_ECAPACITY
    assert int(count.item()) == cap
    assert np.array_equal(words.cpu().numpy().view(np.uint64), ref[:cap])


def test_cw64_repeated_calls_agree():
    a = gpu_code(35, 4, 6)
    b = gpu_code(35, 4, 6)
    assert np.array_equal(a, b)

"""GPU test of greedy_code_device_noalloc, the entry point that allocates
nothing: through the C ABI, its output must equal greedy_code_device's word
for word, on two calls in a row (the second with a smaller input, so that
state left in the shared device array by the first call cannot leak into the
second)."""
import sys

import numpy as np
import pytest

import paper_1507_05398_amd as gc

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    gc.load()
    return torch


def build(torch, fn, n, d, o):
    cap = gc.greedy_code_capacity(n, d)
    words = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    fn(n, d, o, words, count)
    torch.cuda.synchronize()
    m = int(count.item())
    return words[:m].cpu().numpy().view(np.uint32).copy()


@pytest.mark.parametrize("first,second", [((20, 3, "lex"), (16, 4, "gray")),
                                          ((18, 5, "grlex"), (12, 3, "grevlex")),
                                          ((22, 4, "gray"), (9, 2, "lex"))])
def test_noalloc_matches_device_entry_point(cuda, first, second):
    for n, d, o in (first, second):
        log(f"[noalloc] n={n} d={d} ord={o}")
        ref = build(cuda, gc.greedy_code_device, n, d, o)
        got = build(cuda, gc.greedy_code_device_noalloc, n, d, o)
        assert len(got) == len(ref), (n, d, o)
        assert np.array_equal(got, ref), (n, d, o)


def test_noalloc_capacity_error_keeps_prefix(cuda):
    ref = build(cuda, gc.greedy_code_device, 16, 3, "lex")
    words = cuda.zeros(1000, dtype=cuda.int32, device="cuda")
    count = cuda.zeros(1, dtype=cuda.int64, device="cuda")
    with pytest.raises(gc.GreedyCodeError) as e:
        gc.greedy_code_device_noalloc(16, 3, "lex", words, count)
    assert e.value.rc == gc.GC_ECAPACITY
    assert int(count.item()) == 1000
    assert np.array_equal(words.cpu().numpy().view(np.uint32), ref[:1000])

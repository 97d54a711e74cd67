"""GPU parity of the paper's other problems against the CPU oracle, word for
word: the B-ordering with a user basis, constant-weight codes,
self-orthogonal codes, and checkpoint/resume of a construction.

The oracle side builds each walk by its definition (oracle.border_table,
oracle.weight_class, oracle.order_table) and runs the plain greedy scan over
it (oracle.greedy_list, with the self-orthogonality rule when asked)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1507_05398_amd as gc

pytestmark = pytest.mark.gpu
ORDS = ["lex", "gray", "grlex", "grevlex"]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    gc.load()
    return torch


def gpu(p, **tuning):
    words, stats = gc.device_problem_code(p, **tuning)
    return words.cpu().numpy().view(np.uint32).copy(), stats


def random_basis(n, rng):
    """A random invertible n x n matrix over F_2, as n column words."""
    while True:
        basis = [int(v) for v in rng.integers(1, 1 << n, size=n)]
        piv = {}
        ok = True
        for v in basis:
            for b in range(n - 1, -1, -1):
                if not (v >> b) & 1:
                    continue
                if b in piv:
                    v ^= piv[b]
                else:
                    piv[b] = v
                    break
            else:
                ok = False
            if v == 0:
                ok = False
        if ok:
            return basis


# ---- B-ordering -------------------------------------------------------------

@pytest.mark.parametrize("n,d", [(8, 3), (12, 4), (14, 3), (16, 5), (18, 4), (20, 6)])
def test_border_random_basis_matches_oracle(n, d):
    rng = np.random.default_rng(1000 + n * 10 + d)
    basis = random_basis(n, rng)
    log(f"[border] n={n} d={d}")
    ref, _, _ = oracle.greedy_list(n, d, oracle.border_table(n, basis))
    got, _ = gpu(gc.problem(n, d, "border", basis=basis))
    assert np.array_equal(got, ref), (n, d, len(got), len(ref))


def test_border_unit_and_gray_bases_give_lex_and_gray():
    n = 20
    unit = [1 << j for j in range(n)]
    gray = [1] + [(1 << j) | (1 << (j - 1)) for j in range(1, n)]
    for d in (3, 5):
        lex_code, _ = gc.device_code(n, d, "lex")
        gray_code, _ = gc.device_code(n, d, "gray")
        got_unit, _ = gpu(gc.problem(n, d, "border", basis=unit))
        got_gray, _ = gpu(gc.problem(n, d, "border", basis=gray))
        assert np.array_equal(got_unit, lex_code.cpu().numpy().view(np.uint32))
        assert np.array_equal(got_gray, gray_code.cpu().numpy().view(np.uint32))


def test_border_code_is_linear():
    """B-greedy codes are linear (Brualdi and Pless): closed under XOR."""
    n, d = 16, 4
    basis = random_basis(n, np.random.default_rng(77))
    got, _ = gpu(gc.problem(n, d, "border", basis=basis))
    s = set(got.tolist())
    assert len(got) & (len(got) - 1) == 0
    for a in got[:64]:
        for b in got[:: max(1, len(got) // 64)]:
            assert int(a) ^ int(b) in s


# ---- constant weight --------------------------------------------------------

@pytest.mark.parametrize("o", ["lex", "grlex", "grevlex"])
@pytest.mark.parametrize("n,w,d", [(10, 3, 4), (12, 4, 4), (14, 5, 6), (16, 6, 4), (18, 5, 6), (20, 4, 4),
                                   (20, 8, 6), (22, 3, 4), (12, 0, 3), (9, 9, 2), (11, 5, 1)])
def test_constant_weight_matches_oracle(o, n, w, d):
    log(f"[weight] n={n} w={w} d={d} {o}")
    ref, _, _ = oracle.greedy_list(n, d, oracle.weight_class(n, w, oracle.ORDERINGS[o]))
    got, _ = gpu(gc.problem(n, d, o, weight=w))
    assert np.array_equal(got, ref), (n, w, d, o, len(got), len(ref))
    assert np.all(np.bitwise_count(got) == w)


# ---- self-orthogonal ----------------------------------------------------------

@pytest.mark.parametrize("o", ORDS)
@pytest.mark.parametrize("n,d", [(6, 2), (8, 4), (10, 1), (12, 4), (14, 3), (16, 4), (18, 6), (20, 4)])
def test_self_orthogonal_matches_oracle(o, n, d):
    log(f"[so] n={n} d={d} {o}")
    ref, _, _ = oracle.greedy_list(n, d, oracle.order_table(n, oracle.ORDERINGS[o]), self_orth=True)
    got, _ = gpu(gc.problem(n, d, o, self_orthogonal=True))
    assert np.array_equal(got, ref), (n, d, o, len(got), len(ref))


def test_self_orthogonal_lex_24_8_is_the_extended_golay_code():
    """Section "Some Examples": the self-orthogonal lexicode of length 24 and
    distance 8 is the extended Golay [24,12,8] code (weight enumerator
    1, 759, 2576, 759, 1); the oracle gives the same list."""
    got, _ = gpu(gc.problem(24, 8, "lex", self_orthogonal=True))
    assert len(got) == 4096
    wt = np.bincount(np.bitwise_count(got), minlength=25)
    assert {k: int(v) for k, v in enumerate(wt) if v} == {0: 1, 8: 759, 12: 2576, 16: 759, 24: 1}
    ref, _, _ = oracle.greedy_list(24, 8, oracle.order_table(24, oracle.LEX), self_orth=True)
    assert np.array_equal(got, ref)


def test_self_orthogonal_with_weight():
    for n, w, d in [(12, 4, 4), (14, 6, 4), (10, 3, 2)]:
        ref, _, _ = oracle.greedy_list(n, d, oracle.weight_class(n, w, oracle.GREVLEX), self_orth=True)
        got = gc.greedy_code_problem(gc.problem(n, d, "grevlex", weight=w, self_orthogonal=True))
        assert np.array_equal(got, ref), (n, w, d)


# ---- checkpoint / resume ------------------------------------------------------

@pytest.mark.parametrize("kw", [dict(n=20, d=3, ordering="lex"), dict(n=18, d=5, ordering="gray"),
                                dict(n=16, d=4, ordering="grlex"), dict(n=17, d=3, ordering="grevlex"),
                                dict(n=16, d=6, ordering="lex", weight=7),
                                dict(n=16, d=4, ordering="gray", self_orthogonal=True)],
                         ids=["lex", "gray", "grlex", "grevlex", "weight", "so"])
def test_resume_gives_the_same_code(kw):
    n, d, o = kw.pop("n"), kw.pop("d"), kw.pop("ordering")
    whole = gc.problem(n, d, o, **kw)
    full, _ = gpu(whole)
    total = gc.problem_positions(whole)
    cuts = sorted({1, total // 3 + 17, total // 2, total - 5})
    prev, words = 0, np.zeros(0, dtype=np.uint32)
    for cut in cuts + [total]:
        part = gc.problem(n, d, o, start=prev, stop=cut, prefix=len(words), **kw)
        log(f"[resume] {o} n={n} d={d} [{prev}, {cut}) after {len(words)} words")
        t, _ = gc.device_problem_code(part, prefix_words=words)
        words = t.cpu().numpy().view(np.uint32).copy()
        prev = cut
    assert np.array_equal(words, full)


def test_resume_through_host_entry_point():
    n, d = 18, 4
    ref = oracle.greedy_ball(n, d, oracle.GRAY)[0]
    first = gc.greedy_code_problem(gc.problem(n, d, "gray", stop=100000))
    assert np.array_equal(first, ref[: len(first)])
    rest = gc.greedy_code_problem(gc.problem(n, d, "gray", start=100000, prefix=len(first)), prefix_words=first)
    assert np.array_equal(rest, ref)


def test_empty_range_returns_the_prefix():
    pre = np.array([0, 7, 25], dtype=np.uint32)
    got = gc.greedy_code_problem(gc.problem(8, 3, "lex", start=40, stop=40, prefix=3), prefix_words=pre)
    assert np.array_equal(got, pre)
    assert len(gc.greedy_code_problem(gc.problem(10, 4, "lex", weight=3, self_orthogonal=True))) == 0

"""Pins for the oracle's uint64 functions (constant-weight walks of length up
to 64; section "Some Examples" reports constant-weight codes up to length 35).

As for the 32-bit oracle, no expected value comes from the oracle itself:
weight classes are checked against subsets listed by itertools, small greedy
codes against a plain Python greedy, and the codes past 32 bits against closed
forms of coding theory (disjoint supports, all words at d = 2, the projective
triple system at n = 2^k - 1) and the independent certificate.
"""
import itertools
import math

import numpy as np
import pytest

import oracle


def subsets_in_value_order(n, w):
    return sorted(sum(1 << b for b in c) for c in itertools.combinations(range(n), w))


def python_greedy(cands, d):
    """The greedy rule with its work counts: checks done newest first up to
    the first clash (W_ee), and every candidate against every word accepted
    before it (W_full)."""
    code, w_ee, w_full = [], 0, 0
    for x in cands:
        w_full += len(code)
        accept = True
        for c in reversed(code):
            w_ee += 1
            if bin(x ^ c).count("1") < d:
                accept = False
                break
        if accept:
            code.append(x)
    return code, w_ee, w_full


@pytest.mark.parametrize("n,w", [(1, 0), (1, 1), (6, 3), (12, 5), (20, 2), (33, 1), (35, 2), (35, 3), (64, 1),
                                 (64, 2), (64, 63), (64, 64)])
def test_weight_class64_is_every_subset_in_increasing_value(n, w):
    got = [int(x) for x in oracle.weight_class64(n, w)]
    assert len(got) == math.comb(n, w)
    if math.comb(n, w) <= 5000:
        assert got == subsets_in_value_order(n, w)
    else:
        assert all(a < b for a, b in zip(got, got[1:]))
        assert all(bin(x).count("1") == w for x in got)


def test_weight_class64_extremes():
    assert [int(x) for x in oracle.weight_class64(64, 0)] == [0]
    assert [int(x) for x in oracle.weight_class64(64, 64)] == [(1 << 64) - 1]
    units = [int(x) for x in oracle.weight_class64(64, 1)]
    assert units == [1 << b for b in range(64)]
    with pytest.raises(oracle.OracleError):
        oracle.weight_class64(65, 1)
    with pytest.raises(oracle.OracleError):
        oracle.weight_class64(10, 11)


@pytest.mark.parametrize("n,w,d", [(10, 3, 4), (12, 4, 4), (12, 4, 6), (14, 5, 4), (16, 3, 4), (16, 6, 6)])
def test_greedy_list64_is_the_plain_greedy(n, w, d):
    cands = subsets_in_value_order(n, w)
    words, w_ee, w_full = oracle.greedy_list64(n, d, np.array(cands, dtype=np.uint64))
    expect, expect_ee, expect_full = python_greedy(cands, d)
    assert [int(x) for x in words] == expect
    assert (w_ee, w_full) == (expect_ee, expect_full)


@pytest.mark.parametrize("n,w", [(35, 2), (35, 3), (40, 4), (64, 5), (64, 7)])
def test_disjoint_supports_past_32_bits(n, w):
    # At d = 2w two weight-w words may share no coordinate: the greedy in
    # increasing value takes the blocks {0..w-1}, {w..2w-1}, ... and stops.
    words = [int(x) for x in oracle.greedy_list64(n, 2 * w, oracle.weight_class64(n, w))[0]]
    block = (1 << w) - 1
    assert words == [block << (w * k) for k in range(n // w)]


@pytest.mark.parametrize("n,w", [(35, 1), (35, 3), (40, 2)])
def test_distance_two_takes_every_word_past_32_bits(n, w):
    cands = oracle.weight_class64(n, w)
    words, _, _ = oracle.greedy_list64(n, 2, cands)
    assert len(words) == math.comb(n, w)
    assert np.array_equal(words, cands)


def test_triple_system_at_63():
    # For n = 2^k - 1 the weight-3, distance-4 greedy code in increasing value
    # is the set of lines of the projective geometry PG(k-1, 2): with the
    # points labelled 1..n by their coordinate index plus one, every triple
    # {a < b < c} has a XOR b = c, and there are n(n-1)/6 of them (a Steiner
    # triple system: every pair of points on exactly one triple).
    n = 63
    cands = oracle.weight_class64(n, 3)
    words = [int(x) for x in oracle.greedy_list64(n, 4, cands)[0]]
    assert len(words) == n * (n - 1) // 6
    pairs = set()
    for x in words:
        a, b, c = (i + 1 for i in range(n) if (x >> i) & 1)
        assert a ^ b == c
        for p in ((a, b), (a, c), (b, c)):
            assert p not in pairs
            pairs.add(p)
    assert len(pairs) == n * (n - 1) // 2
    assert oracle.verify_certificate64(n, 4, cands, words) == 0


def test_certificate64_rejects_mutations():
    n, w, d = 35, 3, 4
    cands = oracle.weight_class64(n, w)
    words = oracle.greedy_list64(n, d, cands)[0]
    assert oracle.verify_certificate64(n, d, cands, words) == 0
    dropped = np.delete(words, 5)
    assert oracle.verify_certificate64(n, d, cands, dropped) == 3
    swapped = words.copy()
    swapped[[3, 4]] = swapped[[4, 3]]
    assert oracle.verify_certificate64(n, d, cands, swapped) != 0
    # A candidate the greedy rejected, put in its place, clashes or breaks maximality.
    rejected = [int(x) for x in cands if int(x) not in set(int(y) for y in words)]
    extra = np.sort(np.append(words, np.uint64(rejected[10])))
    assert oracle.verify_certificate64(n, d, cands, extra) in (2, 3)


def test_distance64():
    assert oracle.distance64(0, (1 << 64) - 1) == 64
    assert oracle.distance64(1 << 63, 1) == 2

"""Pins for the CPU oracle against what the paper and coding theory fix.

None of these tests compares the oracle with itself: every expected value is a
number printed in the paper, a textbook closed form or code property, a
listing written out by hand, or brute force on tiny inputs.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ORDS = [oracle.LEX, oracle.GRAY, oracle.GRLEX, oracle.GREVLEX]
NAMES = {v: k for k, v in oracle.ORDERINGS.items()}


def bits(s):
    return int(s, 2)


def weight_distribution(words):
    w = np.array([bin(int(x)).count("1") for x in words])
    vals, counts = np.unique(w, return_counts=True)
    return {int(a): int(b) for a, b in zip(vals, counts)}


def ball_volume(n, r):
    return sum(math.comb(n, i) for i in range(0, r + 1))


# --------------------------------------------------------------------------
# Paper's worked example (section "Parallel Implementation", Example 1)
# --------------------------------------------------------------------------

def load_example1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "example1_n3_d2_lex.txt"))
            if l.strip() and not l.startswith("#")]
    n, d, name = int(rows[0][0]), int(rows[0][1]), rows[0][2]
    return n, d, oracle.ORDERINGS[name], [bits(r[0]) for r in rows[1:]]


def test_worked_example_1():
    n, d, ordering, expected = load_example1()
    words, w_ee, w_full = oracle.greedy_scan(n, d, ordering)
    assert words.tolist() == expected
    # Example 1 compares each candidate with every output word: 1+1+1+2+2+3+4
    # comparisons over steps 2..8 (the paper's per-step thread counts).
    assert w_full == 1 + 1 + 1 + 2 + 2 + 3 + 4
    words2, _ = oracle.greedy_ball(n, d, ordering)
    assert words2.tolist() == expected


def test_example1_other_orderings_by_hand():
    # Derived by hand: Gray lists 000,001,011,010,110,111,101,100 -> keeps
    # 000, 011, 110, 101.  Both graded orders list 000 | 001 010 100 | 011 101
    # 110 | 111 (grevlex tie-break agrees with grlex at n=3, weight 2).
    assert oracle.greedy_scan(3, 2, oracle.GRAY)[0].tolist() == [0b000, 0b011, 0b110, 0b101]
    for o in (oracle.GRLEX, oracle.GREVLEX):
        assert oracle.greedy_scan(3, 2, o)[0].tolist() == [0b000, 0b011, 0b101, 0b110]


# --------------------------------------------------------------------------
# Orderings (section "Ordering Implementation")
# --------------------------------------------------------------------------

def test_orderings_n4_listing_by_hand():
    for line in open(os.path.join(GOLDEN, "orderings_n4.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        name, *listing = line.split()
        table = oracle.order_table(4, oracle.ORDERINGS[name])
        assert table.tolist() == [bits(s) for s in listing], name


@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n", [1, 2, 5, 9, 12])
def test_orderings_are_bijections_starting_at_zero(n, ordering):
    t = oracle.order_table(n, ordering)
    assert t[0] == 0
    assert np.array_equal(np.sort(t), np.arange(1 << n, dtype=np.uint32))
    if ordering in (oracle.GRLEX, oracle.GREVLEX):
        w = np.array([bin(int(x)).count("1") for x in t])
        assert np.all(np.diff(w) >= 0)


@pytest.mark.parametrize("n", [1, 3, 8, 13])
def test_gray_consecutive_words_differ_in_one_coordinate(n):
    t = oracle.order_table(n, oracle.GRAY).astype(np.int64)
    d = np.bitwise_xor(t[1:], t[:-1])
    assert np.all([bin(int(x)).count("1") == 1 for x in d])
    # Textbook closed form of the reflected code: g(p) = p xor (p >> 1).
    p = np.arange(1 << n, dtype=np.int64)
    assert np.array_equal(t, p ^ (p >> 1))


@pytest.mark.parametrize("n", [5, 10])
def test_grlex_is_weight_then_value(n):
    t = oracle.order_table(n, oracle.GRLEX)
    key = sorted(range(1 << n), key=lambda x: (bin(x).count("1"), x))
    assert t.tolist() == key


@pytest.mark.parametrize("n", [4, 7, 11])
def test_grevlex_complement_bitreversal_form(n):
    # Independent characterisation: inside weight w, grevlex ascending equals
    # bit-reverse of the complement of the weight-(n-w) integers taken in
    # increasing order (complement maps the weight-(n-w) list, increasing, to
    # the weight-w list, decreasing; bit-reversal turns "highest differing
    # bit is 0" into "lowest differing bit is 0").
    def rev(x):
        return int(format(x, f"0{n}b")[::-1], 2)
    mask = (1 << n) - 1
    expected = []
    for w in range(n + 1):
        ys = [y for y in range(1 << n) if bin(y).count("1") == n - w]
        expected += [rev(~y & mask) for y in ys]
    assert oracle.order_table(n, oracle.GREVLEX).tolist() == expected


def test_distance_is_count_of_differing_coordinates():
    rng = np.random.default_rng(5)
    for a, b in rng.integers(0, 1 << 32, size=(200, 2), dtype=np.uint64):
        a, b = int(a), int(b)
        naive = sum(((a >> i) & 1) != ((b >> i) & 1) for i in range(32))
        assert oracle.distance(a, b) == naive


# --------------------------------------------------------------------------
# Degenerate parameters (closed forms)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n", [1, 4, 9])
def test_degenerate_distances(n, ordering):
    table = oracle.order_table(n, ordering)
    assert np.array_equal(oracle.greedy_scan(n, 1, ordering)[0], table)
    assert oracle.greedy_scan(n, n + 1, ordering)[0].tolist() == [0]
    assert oracle.greedy_scan(n, n + 7, ordering)[0].tolist() == [0]
    assert oracle.greedy_scan(n, n, ordering)[0].tolist() == [0, (1 << n) - 1]


def test_invalid_arguments():
    for bad in [(0, 3, 0), (33, 3, 0), (5, 0, 0), (5, 3, 4), (5, 3, -1)]:
        with pytest.raises(oracle.OracleError):
            oracle.greedy_scan(*bad)


def test_capacity_error():
    with pytest.raises(oracle.OracleError) as e:
        oracle.greedy_scan(10, 3, oracle.LEX, cap=5)
    assert e.value.rc == oracle.ECAPACITY
    with pytest.raises(oracle.OracleError) as e:
        oracle.greedy_ball(10, 3, oracle.LEX, cap=5)
    assert e.value.rc == oracle.ECAPACITY


# --------------------------------------------------------------------------
# Classical codes (paper, section "Some Examples"; textbook enumerators)
# --------------------------------------------------------------------------

def load_enumerators():
    out = []
    for line in open(os.path.join(GOLDEN, "weight_enumerators.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        head, tail = line.split("|")
        n, d, name = head.split()
        dist = {int(a): int(b) for a, b in (t.split(":") for t in tail.split())}
        out.append((int(n), int(d), name, dist))
    return out


@pytest.mark.parametrize("n,d,name,dist", load_enumerators(), ids=lambda v: str(v))
def test_lexicodes_are_classical_codes(n, d, name, dist):
    words, _, _ = oracle.greedy_scan(n, d, oracle.LEX)
    assert len(words) == sum(dist.values())
    assert weight_distribution(words) == dist
    # Gray is a B-ordering, so its greedy code is linear too; the same classical
    # codes appear (checked here by weight distribution).
    gwords, _ = oracle.greedy_ball(n, d, oracle.GRAY)
    assert weight_distribution(gwords) == dist


@pytest.mark.parametrize("n", list(range(3, 21)))
def test_lex_d3_size_is_shortened_hamming(n):
    # The d=3 lexicode of length n is a shortened Hamming code of redundancy
    # r = ceil(log2(n+1)): 2^(n-r) words; perfect when n = 2^r - 1.
    r = math.ceil(math.log2(n + 1))
    words, _ = oracle.greedy_ball(n, 3, oracle.LEX)
    assert len(words) == 1 << (n - r)
    if n + 1 == 1 << r:
        assert len(words) * (n + 1) == 1 << n  # sphere-packing equality


@pytest.mark.parametrize("ordering", [oracle.LEX, oracle.GRAY])
@pytest.mark.parametrize("n,d", [(6, 2), (9, 3), (10, 4), (12, 5), (13, 6), (14, 7), (15, 8)])
def test_lex_and_gray_codes_are_linear(n, d, ordering):
    # Lexicodes and, more generally, B-greedy codes are linear (Brualdi-Pless):
    # closed under XOR, size a power of two (paper, caption of the figure on
    # time vs distance: "M = 2^k"), and word i is the XOR of the basis words at
    # the 1-bits of i.
    words, _ = oracle.greedy_ball(n, d, ordering)
    s = set(int(w) for w in words)
    k = len(words).bit_length() - 1
    assert len(words) == 1 << k
    for a in list(s)[:64]:
        for b in s:
            assert (a ^ b) in s
    basis = [int(words[1 << j]) for j in range(k)]
    for i, w in enumerate(words):
        acc = 0
        for j in range(k):
            if (i >> j) & 1:
                acc ^= basis[j]
        assert acc == int(w)


@pytest.mark.parametrize("n", list(range(5, 17)))
@pytest.mark.parametrize("d", [2, 4, 8])
def test_lex_equals_grlex_as_sets_for_power_of_two_distance(n, d):
    # Paper, section "Some Examples": for d a power of two the lexicographic and
    # graded-lexicographic greedy codes contain exactly the same words.
    lex, _ = oracle.greedy_ball(n, d, oracle.LEX)
    grl, _ = oracle.greedy_ball(n, d, oracle.GRLEX)
    assert sorted(lex.tolist()) == sorted(grl.tolist())


@pytest.mark.parametrize("n,t", [(10, 2), (14, 2), (12, 3), (18, 2), (16, 4)])
def test_even_distance_size_equals_punctured_odd(n, t):
    # For lexicodes |L(n, 2t)| = |L(n-1, 2t-1)| (extension by a parity bit).
    a, _ = oracle.greedy_ball(n, 2 * t, oracle.LEX)
    b, _ = oracle.greedy_ball(n - 1, 2 * t - 1, oracle.LEX)
    assert len(a) == len(b)


# --------------------------------------------------------------------------
# Bounds, certificate and brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n,d", [(8, 3), (11, 4), (13, 5), (14, 3), (12, 6), (15, 7)])
def test_gilbert_varshamov_and_hamming_bounds(n, d, ordering):
    words, _ = oracle.greedy_ball(n, d, ordering)
    m = len(words)
    # maximal code: the radius-(d-1) balls cover the space
    assert m * ball_volume(n, d - 1) >= 1 << n
    # packing: the radius-floor((d-1)/2) balls are disjoint
    assert m * ball_volume(n, (d - 1) // 2) <= 1 << n


@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_outputs_satisfy_certificate(n, ordering):
    for d in range(1, n + 2):
        words, _, _ = oracle.greedy_scan(n, d, ordering)
        assert oracle.verify_certificate(n, d, ordering, words) == 0, (n, d)


def test_certificate_rejects_wrong_outputs():
    n, d = 8, 3
    for ordering in ORDS:
        words, _, _ = oracle.greedy_scan(n, d, ordering)
        w = words.tolist()
        assert oracle.verify_certificate(n, d, ordering, w[:-1]) == 3        # missing word
        assert oracle.verify_certificate(n, d, ordering, w[1:]) == 3
        assert oracle.verify_certificate(n, d, ordering, w[:3] + [w[3] ^ 1] + w[4:]) != 0
        assert oracle.verify_certificate(n, d, ordering, [w[1], w[0]] + w[2:]) == 1
        assert oracle.verify_certificate(n, d + 1, ordering, w) != 0
        assert oracle.verify_certificate(n, d - 1, ordering, w) != 0


def max_code_size(n, d):
    """A(n, d) by exhaustive branch and bound (tiny n).  The distance graph is
    vertex transitive under XOR translation, so the search may keep 0."""
    size = 1 << n
    conflict = [0] * size
    for a in range(size):
        for b in range(size):
            if a != b and bin(a ^ b).count("1") < d:
                conflict[a] |= 1 << b
    best = 1

    def rec(cand, k):
        nonlocal best
        if k > best:
            best = k
        while cand:
            if k + bin(cand).count("1") <= best:
                return
            v = (cand & -cand).bit_length() - 1
            cand &= ~(1 << v)
            rec(cand & ~conflict[v], k + 1)

    rec(((1 << size) - 1) & ~conflict[0] & ~1, 1)
    return best


# Textbook values of A(n, d) (MacWilliams-Sloane table) confirm the search.
KNOWN_A = {(3, 3): 2, (4, 3): 2, (5, 3): 4, (5, 4): 2, (4, 2): 8, (5, 2): 16, (6, 3): 8,
           (6, 4): 4, (6, 5): 2}


@pytest.mark.parametrize("n,d", sorted(KNOWN_A))
def test_brute_force_optimal_sizes_bound_greedy(n, d):
    a = max_code_size(n, d)
    assert a == KNOWN_A[(n, d)]
    for ordering in ORDS:
        words, _, _ = oracle.greedy_scan(n, d, ordering)
        assert len(words) <= a
        if ordering == oracle.LEX:
            # lexicodes reach A(n, d) at these small parameters
            assert len(words) == a


def python_greedy(n, d, table):
    """Tiny-n brute force used only to check the work counters."""
    code, ee, full = [], 0, 0
    for x in table:
        ok = True
        full += len(code)
        for c in reversed(code):
            ee += 1
            if bin(int(x) ^ c).count("1") < d:
                ok = False
                break
        if ok:
            code.append(int(x))
    return code, ee, full


@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n,d", [(5, 2), (6, 3), (7, 3), (8, 4), (8, 5)])
def test_work_counters_brute_force(n, d, ordering):
    table = oracle.order_table(n, ordering)
    code, ee, full = python_greedy(n, d, table)
    words, w_ee, w_full = oracle.greedy_scan(n, d, ordering)
    assert words.tolist() == code
    assert (w_ee, w_full) == (ee, full)
    # W_full closed form: sum over accepted words of the candidates after them.
    pos = {int(x): p for p, x in enumerate(table)}
    assert w_full == sum((1 << n) - 1 - pos[w] for w in code)


@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n,d", [(10, 2), (12, 3), (13, 4), (14, 5), (15, 3), (16, 6), (16, 3)])
def test_plain_scan_equals_ball_marking(n, d, ordering):
    words, w_ee, w_full = oracle.greedy_scan(n, d, ordering)
    words2, w_ee2, w_full2 = oracle.greedy_ball(n, d, ordering, want_w_ee=True, want_w_full=True)
    assert np.array_equal(words, words2)
    assert (w_ee, w_full) == (w_ee2, w_full2)

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


# --------------------------------------------------------------------------
# Wide ball marking (LEX/GRAY up to n = 32): same output as the plain scan
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ordering", [oracle.LEX, oracle.GRAY])
@pytest.mark.parametrize("n,d", [(1, 1), (4, 2), (9, 3), (10, 4), (12, 5), (13, 8), (15, 3), (16, 6)])
def test_wide_ball_marking_equals_plain_scan(n, d, ordering):
    words, _, w_full = oracle.greedy_scan(n, d, ordering)
    wide, full2 = oracle.greedy_ball_wide(n, d, ordering)
    assert np.array_equal(words, wide)
    assert full2 == w_full


def test_wide_ball_marking_extended_golay_lex():
    # the n=24 d=8 lexicode is the extended Golay code (section "Some Examples")
    words, _ = oracle.greedy_ball_wide(24, 8, oracle.LEX)
    assert weight_distribution(words) == {0: 1, 8: 759, 12: 2576, 16: 759, 24: 1}


# --------------------------------------------------------------------------
# B-ordering (section "B-ordering Implementation")
# --------------------------------------------------------------------------

def gf2_rank(vectors):
    rows, rank = [int(v) for v in vectors], 0
    for bit in range(32):
        piv = next((i for i in range(rank, len(rows)) if (rows[i] >> bit) & 1), None)
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and (rows[i] >> bit) & 1:
                rows[i] ^= rows[rank]
        rank += 1
    return rank


def random_basis(n, seed):
    rng = np.random.default_rng(seed)
    while True:
        b = rng.integers(1, 1 << n, size=n, dtype=np.uint64).astype(np.uint32)
        if gf2_rank(b) == n:
            return b


def test_border_listing_of_the_paper():
    # 0, b1, b2, b2+b1, b3, b3+b1, b3+b2, b3+b2+b1 for n = 3
    b = [0b011, 0b110, 0b100]
    t = oracle.border_table(3, b)
    b1, b2, b3 = b
    assert t.tolist() == [0, b1, b2, b2 ^ b1, b3, b3 ^ b1, b3 ^ b2, b3 ^ b2 ^ b1]


@pytest.mark.parametrize("n", [1, 3, 8, 14])
def test_border_unit_basis_is_lex_and_gray_basis_is_gray(n):
    unit = [1 << j for j in range(n)]
    assert np.array_equal(oracle.border_table(n, unit), oracle.order_table(n, oracle.LEX))
    # b_1 = 1, b_j = 2^(j-1) + 2^(j-2): the reflected Gray code (built by reflection)
    gray = [1] + [(1 << j) | (1 << (j - 1)) for j in range(1, n)]
    assert np.array_equal(oracle.border_table(n, gray), oracle.order_table(n, oracle.GRAY))


@pytest.mark.parametrize("n", [5, 11, 16])
def test_border_independent_basis_is_a_bijection(n):
    t = oracle.border_table(n, random_basis(n, n))
    assert t[0] == 0
    assert np.array_equal(np.sort(t), np.arange(1 << n, dtype=np.uint32))


@pytest.mark.parametrize("n,d", [(10, 3), (13, 4), (15, 3), (16, 5)])
def test_border_with_permuted_unit_basis_is_permuted_lexicode(n, d):
    # b_j = 2^sigma(j): position p lists sigma applied to the bits of p, and a
    # permutation of coordinates keeps distances, so the code is sigma(lexicode)
    sigma = np.random.default_rng(n * 31 + d).permutation(n)
    basis = [1 << int(sigma[j]) for j in range(n)]
    words, _, _ = oracle.greedy_list(n, d, oracle.border_table(n, basis))
    lexi, _, _ = oracle.greedy_scan(n, d, oracle.LEX)

    def permute(x):
        return sum(1 << int(sigma[j]) for j in range(n) if (int(x) >> j) & 1)

    assert [int(w) for w in words] == [permute(x) for x in lexi]


@pytest.mark.parametrize("n,d", [(9, 3), (11, 4), (12, 5), (14, 3), (14, 6)])
def test_border_greedy_codes_are_linear(n, d):
    # B-greedy codes are linear (Brualdi and Pless, cited in the B-ordering
    # section): |C| = 2^k and the code is closed under XOR
    for seed in range(3):
        words, _, _ = oracle.greedy_list(n, d, oracle.border_table(n, random_basis(n, 100 * n + seed)))
        k = int(math.log2(len(words)))
        assert len(words) == 1 << k
        s = set(int(w) for w in words)
        assert all((int(a) ^ int(b)) in s for a in words[:40] for b in words)


@pytest.mark.parametrize("n,d", [(8, 3), (10, 4), (12, 3)])
def test_border_greedy_satisfies_certificate(n, d):
    table = oracle.border_table(n, random_basis(n, 7 * n + d))
    words, _, _ = oracle.greedy_list(n, d, table)
    assert oracle.verify_certificate_list(n, d, table, words) == 0
    bad = words.copy()
    bad[-1] ^= 1
    assert oracle.verify_certificate_list(n, d, table, bad) != 0


# --------------------------------------------------------------------------
# Constant-weight codes (section "Brief overview ...": given n, d and w)
# --------------------------------------------------------------------------

def test_weight_class_listings_by_hand():
    assert [format(int(x), "04b") for x in oracle.weight_class(4, 2, oracle.LEX)] == \
        ["0011", "0101", "0110", "1001", "1010", "1100"]
    assert [format(int(x), "04b") for x in oracle.weight_class(4, 2, oracle.GREVLEX)] == \
        ["0011", "0101", "1001", "0110", "1010", "1100"]
    assert oracle.weight_class(5, 0, oracle.LEX).tolist() == [0]
    assert oracle.weight_class(5, 5, oracle.GRLEX).tolist() == [31]


@pytest.mark.parametrize("n,w", [(6, 3), (10, 4), (12, 1), (13, 6)])
def test_weight_class_sizes_and_weights(n, w):
    c = oracle.weight_class(n, w, oracle.LEX)
    assert len(c) == math.comb(n, w)
    assert all(bin(int(x)).count("1") == w for x in c)
    assert np.all(np.diff(c.astype(np.int64)) > 0)


@pytest.mark.parametrize("n,w", [(8, 3), (11, 4), (12, 5), (9, 2)])
def test_constant_weight_closed_forms(n, w):
    c = oracle.weight_class(n, w, oracle.LEX)
    # distinct words of one weight differ in at least 2 places: d <= 2 keeps all
    assert len(oracle.greedy_list(n, 2, c)[0]) == len(c)
    # distance 2w means disjoint supports: the greedy takes consecutive blocks
    words = oracle.greedy_list(n, 2 * w, c)[0]
    assert [int(x) for x in words] == [((1 << w) - 1) << (w * i) for i in range(n // w)]
    # odd d behaves as d + 1 (distances between equal-weight words are even)
    assert np.array_equal(oracle.greedy_list(n, 2 * w - 1, c)[0], words)
    # above 2w only the first word fits
    assert oracle.greedy_list(n, 2 * w + 1, c)[0].tolist() == [(1 << w) - 1]


@pytest.mark.parametrize("n", [7, 15, 31])
def test_constant_weight_triples_are_projective_steiner_systems(n):
    # n = 2^m - 1, w = 3, d = 4: the lexicographic code is the Steiner triple
    # system of points and lines of PG(m-1, 2), n(n-1)/6 triples, every pair
    # of points in exactly one triple
    words = oracle.greedy_list(n, 4, oracle.weight_class(n, 3, oracle.LEX))[0]
    assert len(words) == n * (n - 1) // 6
    pairs = set()
    for x in words:
        pts = [j for j in range(n) if (int(x) >> j) & 1]
        for a, b in itertools.combinations(pts, 2):
            assert (a, b) not in pairs
            pairs.add((a, b))
    assert len(pairs) == n * (n - 1) // 2


def johnson_bound(n, d, w):
    # A(n, 2t, w) <= floor(n/w * A(n-1, 2t, w-1)), with A = 1 once w < t
    t = (d + 1) // 2
    if w < t:
        return 1
    return n * johnson_bound(n - 1, d, w - 1) // w


@pytest.mark.parametrize("ordering", [oracle.LEX, oracle.GREVLEX])
@pytest.mark.parametrize("n,d,w", [(10, 4, 4), (12, 6, 5), (13, 4, 3), (14, 6, 4), (11, 8, 5)])
def test_constant_weight_bounds_and_certificate(n, d, w, ordering):
    c = oracle.weight_class(n, w, ordering)
    words = oracle.greedy_list(n, d, c)[0]
    assert len(words) <= johnson_bound(n, d, w)
    assert oracle.verify_certificate_list(n, d, c, words) == 0


# --------------------------------------------------------------------------
# Self-orthogonal greedy codes (section "Self Orthogonal Greedy Codes
# Implementation"; section "Some Examples")
# --------------------------------------------------------------------------

def macwilliams_self_dual(dist, n):
    # weight enumerator of the dual: B_j = 2^-k sum_i A_i K_j(i), with the
    # Krawtchouk polynomial K_j(i) = sum_s (-1)^s C(i, s) C(n - i, j - s)
    size = sum(dist.values())
    out = {}
    for j in range(n + 1):
        tot = 0
        for i, a in dist.items():
            tot += a * sum((-1) ** s * math.comb(i, s) * math.comb(n - i, j - s) for s in range(j + 1))
        assert tot % size == 0
        if tot:
            out[j] = tot // size
    return out


@pytest.mark.parametrize("n,d,dist", [
    (8, 4, {0: 1, 4: 14, 8: 1}),                          # extended Hamming [8,4,4]
    (22, 6, {0: 1, 6: 77, 8: 330, 10: 616, 12: 616, 14: 330, 16: 77, 22: 1}),  # self-dual [22,11,6]
    (24, 8, {0: 1, 8: 759, 12: 2576, 16: 759, 24: 1}),   # extended Golay [24,12,8]
])
def test_self_orthogonal_lexicodes_are_the_classical_self_dual_codes(n, d, dist):
    # the paper: self-orthogonal greedy generation gives the extended Golay
    # code [24,12,8]; Monroe's codes include the [22,11,6] one
    words = oracle.greedy_list(n, d, oracle.order_table(n, oracle.LEX), self_orth=True)[0]
    assert weight_distribution(words) == dist
    # self-dual: |C| = 2^(n/2) and the enumerator is its own MacWilliams transform
    assert len(words) == 1 << (n // 2)
    assert macwilliams_self_dual(dist, n) == dist


@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n,d", [(10, 2), (12, 4), (13, 3), (14, 6)])
def test_self_orthogonal_outputs_are_orthogonal_and_certified(n, d, ordering):
    table = oracle.order_table(n, ordering)
    words = oracle.greedy_list(n, d, table, self_orth=True)[0]
    assert all(bin(int(x)).count("1") % 2 == 0 for x in words)
    for a in words:
        for b in words:
            assert bin(int(a) & int(b)).count("1") % 2 == 0
    assert len(words) <= 1 << (n // 2)
    assert oracle.verify_certificate_list(n, d, table, words, self_orth=True) == 0
    bad = words.copy()
    bad[-1] ^= 3
    assert oracle.verify_certificate_list(n, d, table, bad, self_orth=True) != 0


@pytest.mark.parametrize("ordering", ORDS)
@pytest.mark.parametrize("n,d", [(9, 3), (12, 4), (14, 5)])
def test_list_scan_without_constraint_is_the_plain_scan(n, d, ordering):
    a, ee, full = oracle.greedy_scan(n, d, ordering)
    b, ee2, full2 = oracle.greedy_list(n, d, oracle.order_table(n, ordering))
    assert np.array_equal(a, b) and ee == ee2 and full == full2

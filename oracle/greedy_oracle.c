/*
 * greedy_oracle.c -- plain CPU oracle for greedy binary code construction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * HIP library; the two are compared output against output.
 *
 * What it computes (Paliwal, Tiwary, Chaudhury, Gupta, "Generating Binary
 * Optimal Codes Using Heterogeneous Parallel Computing", arXiv:1507.05398):
 *
 *   Section "Greedy Algorithms and Different Orderings": order all 2^n vectors
 *   of F_2^n, start from the zero vector, and append each vector in turn to
 *   the code C if its Hamming distance to every codeword already in C is at
 *   least d.  Stop when all 2^n vectors have been examined.
 *
 *   Section "Hamming Distance": the distance of two words is the number of
 *   coordinates where they differ = popcount(a XOR b).
 *
 *   Section "Ordering Implementation": four orderings -- lexicographic, Gray,
 *   graded-lexicographic and graded-reverse-lexicographic.  The paper names
 *   but does not define the last three; the readings used here are:
 *     LEX      vectors as binary numbers, increasing from 0 (the listing of
 *              Example 1: 000, 001, 010, ..., 111).
 *     GRAY     the binary-reflected Gray code, built by reflection.
 *     GRLEX    weight ascending; inside one weight, the lexicographic order
 *              (leftmost coordinate most significant), i.e. increasing value.
 *     GREVLEX  weight ascending; inside one weight, the graded reverse
 *              lexicographic monomial order of Cox, Little and O'Shea
 *              (exponent vectors alpha, beta of equal weight: alpha > beta iff
 *              the rightmost non-zero entry of alpha - beta is negative),
 *              listed from smallest to largest.
 *   Bit convention: coordinate x_1 (leftmost character of the paper's
 *   strings) is bit n-1 of the word, x_n is bit 0.
 *
 * Two exact algorithms are provided:
 *   gco_greedy_scan  -- the definition itself: for every position, compare the
 *                       candidate with the accepted words, newest first, and
 *                       stop at the first word closer than d.  It also counts
 *                       the distance checks it performs (W_ee) and the checks
 *                       an exhaustive scan would perform (W_full).
 *   gco_greedy_ball  -- ball marking: a vector is rejected exactly when it lies
 *                       within distance d-1 of an earlier accepted word, so on
 *                       acceptance every vector of the radius-(d-1) ball is
 *                       marked.  Same output; used where the scan is too slow.
 *
 * Extensions (the paper's other problems, same greedy rule):
 *   gco_border_table   -- section "B-ordering Implementation": an ordered basis
 *                         b_1..b_n induces the list 0, b_1, b_2, b_2+b_1, b_3,
 *                         ..., built here by its recursive definition (the list
 *                         for b_1..b_k is the list for b_1..b_{k-1} followed by
 *                         b_k added to each of its entries).
 *   gco_weight_class   -- section "Brief overview of the Greedy Algorithm and
 *                         Codes": constant-weight codes take only the weight-w
 *                         vectors as candidates, here in increasing value or
 *                         in the graded reverse lexicographic order.
 *   gco_greedy_list    -- the plain scan over an explicit candidate list, with
 *                         the optional self-orthogonality constraint of section
 *                         "Self Orthogonal Greedy Codes Implementation": a
 *                         candidate must also have an even number of common
 *                         ones (popcount of the AND) with itself and with every
 *                         accepted word.
 *   gco_verify_certificate_list -- the certificate below for a candidate list.
 *   gco_greedy_ball_wide -- ball marking for the two positional orderings up to
 *                         n = 32 (a 2^n-bit covered set, no per-vector index);
 *                         it reports no W_ee.
 *   gco_weight_class64, gco_greedy_list64, gco_verify_certificate64 -- the
 *                         constant-weight walk, the plain scan and the
 *                         certificate over uint64 words, n <= 64 (section
 *                         "Some Examples" reports constant-weight codes up to
 *                         length 35).
 *
 * Parity status: every function here is pinned by the CPU tests against the
 * paper's worked example (Example 1), closed forms (Hamming, extended Hamming
 * and Golay lexicodes, degenerate d), invariants (linearity of LEX/GRAY
 * lexicodes, LEX = GRLEX as sets for d a power of two), an independent
 * certificate check, and brute force on tiny n -- except the GREVLEX
 * within-weight tie-break, for which the paper prints no example or property:
 * parity unpinned beyond the textbook definition (checked against the n=4
 * listing written out by hand in the tests).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GCO_LEX 0
#define GCO_GRAY 1
#define GCO_GRLEX 2
#define GCO_GREVLEX 3

#define GCO_OK 0
#define GCO_EINVAL (-1)
#define GCO_ECAPACITY (-2)
#define GCO_ENOMEM (-4)
#define GCO_EFAIL (-5)

/* Largest n for which an ordering table of 2^n words is materialised. */
#define GCO_TABLE_MAX_N 28

/* ------------------------------------------------------------------ */
/* Hamming distance and weight (section "Hamming Distance")           */
/* ------------------------------------------------------------------ */

/* Number of coordinates in which a and b differ: XOR, then count ones. */
unsigned gco_distance(uint32_t a, uint32_t b)
{
    return (unsigned)__builtin_popcount(a ^ b);
}

/* Number of non-zero coordinates (the weight of a word). */
unsigned gco_weight(uint32_t x)
{
    return (unsigned)__builtin_popcount(x);
}

/* ------------------------------------------------------------------ */
/* Orderings of F_2^n (section "Ordering Implementation")             */
/* ------------------------------------------------------------------ */

/* Binary-reflected Gray code, from its recursive definition: the list for
 * k coordinates is the list for k-1 coordinates with a leading 0, followed by
 * the same list reversed with a leading 1.  Returns the word at position p. */
static uint32_t gray_reflected(uint64_t p, int k)
{
    uint32_t word = 0;
    while (k > 0) {
        uint64_t half = 1ull << (k - 1);
        if (p >= half) {               /* second half: leading 1, reversed */
            word |= (uint32_t)half;
            p = (half - 1) - (p - half);
        }
        --k;
    }
    return word;
}

/* Cox-Little-O'Shea graded reverse lexicographic comparison of two words of
 * equal weight, read as exponent vectors (x_1 .. x_n) with x_1 = bit n-1.
 * alpha > beta iff the rightmost non-zero entry of alpha - beta is negative.
 * "Rightmost" coordinate x_n is bit 0, so walk from bit 0 upwards. */
static int grevlex_greater(uint32_t alpha, uint32_t beta, int n)
{
    for (int bit = 0; bit < n; ++bit) {
        int a = (alpha >> bit) & 1, b = (beta >> bit) & 1;
        if (a != b)
            return (a - b) < 0; /* entry of alpha - beta is a - b */
    }
    return 0; /* equal */
}

static int g_sort_n; /* qsort has no context argument in plain C */

static int cmp_grevlex_ascending(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    if (grevlex_greater(a, b, g_sort_n)) return 1;
    if (grevlex_greater(b, a, g_sort_n)) return -1;
    return 0;
}

/* Fill table[0 .. 2^n) with the ordering, straight from its definition.
 * Graded orders go through the space once per weight, collecting the words of
 * that weight, then order that class by the chosen tie-break. */
int gco_order_table(int n, int ordering, uint32_t *table)
{
    if (n < 1 || n > GCO_TABLE_MAX_N || !table) return GCO_EINVAL;
    uint64_t size = 1ull << n;
    switch (ordering) {
    case GCO_LEX:
        for (uint64_t p = 0; p < size; ++p) table[p] = (uint32_t)p;
        return GCO_OK;
    case GCO_GRAY:
        for (uint64_t p = 0; p < size; ++p) table[p] = gray_reflected(p, n);
        return GCO_OK;
    case GCO_GRLEX:
    case GCO_GREVLEX: {
        uint64_t at = 0;
        for (int w = 0; w <= n; ++w) {
            uint64_t start = at;
            for (uint64_t x = 0; x < size; ++x)      /* increasing value */
                if (gco_weight((uint32_t)x) == (unsigned)w) table[at++] = (uint32_t)x;
            if (ordering == GCO_GREVLEX) {
                g_sort_n = n;
                qsort(table + start, at - start, sizeof(uint32_t), cmp_grevlex_ascending);
            }
        }
        return at == size ? GCO_OK : GCO_EFAIL;
    }
    default:
        return GCO_EINVAL;
    }
}

/* Word at position p without a table, for the two orderings whose definition
 * is positional. */
static int positional(int ordering) { return ordering == GCO_LEX || ordering == GCO_GRAY; }

static uint32_t position_word(int n, int ordering, uint64_t p)
{
    return ordering == GCO_LEX ? (uint32_t)p : gray_reflected(p, n);
}

/* Position -> word via the table when n allows, else positionally. */
typedef struct {
    int n, ordering;
    uint32_t *table; /* NULL when positional */
} order_t;

static int order_open(order_t *o, int n, int ordering)
{
    o->n = n; o->ordering = ordering; o->table = NULL;
    if (ordering < GCO_LEX || ordering > GCO_GREVLEX) return GCO_EINVAL;
    if (positional(ordering)) return GCO_OK;
    if (n <= GCO_TABLE_MAX_N) {
        o->table = (uint32_t *)malloc(sizeof(uint32_t) << n);
        if (!o->table) return GCO_ENOMEM;
        int rc = gco_order_table(n, ordering, o->table);
        if (rc) { free(o->table); o->table = NULL; return rc; }
        return GCO_OK;
    }
    return GCO_EINVAL; /* graded orders need a table */
}

static inline uint32_t order_at(const order_t *o, uint64_t p)
{
    return o->table ? o->table[p] : position_word(o->n, o->ordering, p);
}

static void order_close(order_t *o) { free(o->table); o->table = NULL; }

/* ------------------------------------------------------------------ */
/* The greedy algorithm, by definition (section "Greedy Algorithms ...") */
/* ------------------------------------------------------------------ */

static int check_args(int n, int d, int ordering, const uint64_t *count)
{
    if (n < 1 || n > 32 || d < 1 || ordering < GCO_LEX || ordering > GCO_GREVLEX || !count)
        return GCO_EINVAL;
    return GCO_OK;
}

/* Plain scan.  out has room for cap words; on success *count holds |C| and
 * out[0 .. |C|) the codewords in acceptance order.  w_ee (may be NULL)
 * receives the number of distance checks performed when each candidate is
 * compared with the accepted words newest first and stops at the first word
 * closer than d; w_full (may be NULL) receives sum over candidates of |C| at
 * that moment (every candidate compared with every accepted word).
 * Returns GCO_ECAPACITY if more than cap words would be accepted. */
int gco_greedy_scan(int n, int d, int ordering, uint32_t *out, uint64_t cap,
                    uint64_t *count, uint64_t *w_ee, uint64_t *w_full)
{
    int rc = check_args(n, d, ordering, count);
    if (rc) return rc;
    if (!out && cap) return GCO_EINVAL;
    order_t o;
    if ((rc = order_open(&o, n, ordering))) return rc;

    uint64_t m = 0, ee = 0, full = 0, size = 1ull << n;
    for (uint64_t p = 0; p < size; ++p) {
        uint32_t x = order_at(&o, p);
        int accept = 1;
        for (uint64_t i = m; i-- > 0;) {            /* newest accepted word first */
            ++ee;
            if (gco_distance(x, out[i]) < (unsigned)d) { accept = 0; break; }
        }
        full += m;
        if (accept) {
            if (m == cap) { order_close(&o); *count = m; return GCO_ECAPACITY; }
            out[m++] = x;
        }
    }
    order_close(&o);
    *count = m;
    if (w_ee) *w_ee = ee;
    if (w_full) *w_full = full;
    return GCO_OK;
}

/* Visit every word within distance r of x (all sets of at most r coordinates
 * flipped), marking it covered and, when last is given, recording that the
 * newest accepted word covering it is number idx. */
static void mark_ball(uint32_t x, int n, int r, uint8_t *covered, uint32_t *last, uint32_t idx)
{
    int pos[33];
    /* flip-set of size k, as strictly increasing coordinate lists */
    for (int k = 0; k <= r && k <= n; ++k) {
        for (int i = 0; i < k; ++i) pos[i] = i;
        for (;;) {
            uint32_t y = x;
            for (int i = 0; i < k; ++i) y ^= 1u << pos[i];
            covered[y >> 3] |= (uint8_t)(1u << (y & 7));
            if (last) last[y] = idx;
            /* next combination of k out of n */
            int i = k - 1;
            while (i >= 0 && pos[i] == n - k + i) --i;
            if (i < 0) break;
            ++pos[i];
            for (int j = i + 1; j < k; ++j) pos[j] = pos[j - 1] + 1;
        }
    }
}

/* Ball marking: same output as the plain scan.  w_ee (may be NULL) receives
 * the same newest-first check count the plain scan would report: for a
 * rejected candidate that is |C| minus the index of the newest accepted word
 * within d-1, for an accepted one it is |C|.  w_full (may be NULL) receives
 * the sum over candidates of |C| at that moment.  Needs 2^n/8 bytes, plus
 * 4*2^n bytes when w_ee is requested; n <= GCO_TABLE_MAX_N. */
int gco_greedy_ball(int n, int d, int ordering, uint32_t *out, uint64_t cap,
                    uint64_t *count, uint64_t *w_ee, uint64_t *w_full)
{
    int rc = check_args(n, d, ordering, count);
    if (rc) return rc;
    if (n > GCO_TABLE_MAX_N || (!out && cap)) return GCO_EINVAL;
    order_t o;
    if ((rc = order_open(&o, n, ordering))) return rc;
    uint64_t size = 1ull << n;
    uint8_t *covered = (uint8_t *)calloc(size / 8 + 1, 1);
    uint32_t *last = w_ee ? (uint32_t *)malloc(sizeof(uint32_t) * size) : NULL;
    if (!covered || (w_ee && !last)) {
        free(covered); free(last); order_close(&o);
        return GCO_ENOMEM;
    }
    uint64_t m = 0, ee = 0, full = 0;
    int r = d - 1;
    for (uint64_t p = 0; p < size; ++p) {
        uint32_t x = order_at(&o, p);
        full += m;
        if (covered[x >> 3] & (1u << (x & 7))) {
            if (last) ee += m - last[x];
            continue;
        }
        if (m == cap) { rc = GCO_ECAPACITY; break; }
        ee += m;
        out[m] = x;
        mark_ball(x, n, r, covered, last, (uint32_t)m);
        ++m;
    }
    free(covered); free(last); order_close(&o);
    *count = m;
    if (rc) return rc;
    if (w_ee) *w_ee = ee;
    if (w_full) *w_full = full;
    return GCO_OK;
}

/* ------------------------------------------------------------------ */
/* Certificate: an independent characterisation of the greedy output   */
/* ------------------------------------------------------------------ */

/* words[0 .. count) is the greedy code for (n, d, ordering) iff
 *   (a) the words appear in strictly increasing position order,
 *   (b) every two of them are at distance >= d, and
 *   (c) every vector not in the list is within distance d-1 of a listed word
 *       that comes earlier in the ordering.
 * (By induction over positions: (b) says no listed word should have been
 * rejected, (c) says every unlisted word was.)  Brute force; for small n.
 * Returns 0 if the certificate holds, else 1 + the index of the failed rule. */
int gco_verify_certificate(int n, int d, int ordering, const uint32_t *words, uint64_t count)
{
    if (n < 1 || n > 20 || d < 1 || !words) return GCO_EINVAL;
    order_t o;
    if (order_open(&o, n, ordering)) return GCO_EINVAL;
    uint64_t size = 1ull << n;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * size);
    int8_t *member = (int8_t *)calloc(size, 1);
    if (!pos || !member) { free(pos); free(member); order_close(&o); return GCO_ENOMEM; }
    for (uint64_t p = 0; p < size; ++p) pos[order_at(&o, p)] = (int64_t)p;
    int fail = 0;
    for (uint64_t i = 0; i < count && !fail; ++i) {
        if (words[i] >= size) fail = 1;
        else if (i && pos[words[i]] <= pos[words[i - 1]]) fail = 1;
        else member[words[i]] = 1;
    }
    for (uint64_t i = 0; i < count && !fail; ++i)
        for (uint64_t j = i + 1; j < count; ++j)
            if (gco_distance(words[i], words[j]) < (unsigned)d) { fail = 2; break; }
    for (uint64_t y = 0; y < size && !fail; ++y) {
        if (member[y]) continue;
        int covered = 0;
        for (uint64_t i = 0; i < count && !covered; ++i)
            if (pos[words[i]] < pos[y] && gco_distance((uint32_t)y, words[i]) < (unsigned)d)
                covered = 1;
        if (!covered) fail = 3;
    }
    free(pos); free(member); order_close(&o);
    return fail;
}

/* ------------------------------------------------------------------ */
/* Ball marking up to n = 32 for LEX and GRAY                          */
/* ------------------------------------------------------------------ */

/* Same rule as gco_greedy_ball (a vector is rejected exactly when it lies
 * within d-1 of an earlier accepted word), for the positional orderings at
 * any n <= 32, with a covered set of 2^n bits and no W_ee.  The ball around an
 * accepted word is visited as (flips among the coordinates above the lowest
 * L) x (flips among the lowest L), so that the inner loop stays inside one
 * 64-byte stretch of the covered set; the set of marked vectors is the ball
 * all the same.  w_full (may be NULL) = sum over candidates of |C| then. */
int gco_greedy_ball_wide(int n, int d, int ordering, uint32_t *out, uint64_t cap,
                         uint64_t *count, uint64_t *w_full)
{
    if (n < 1 || n > 32 || d < 1 || !count || (!out && cap)) return GCO_EINVAL;
    if (!positional(ordering)) return GCO_EINVAL;
    uint64_t size = 1ull << n;
    uint8_t *covered = (uint8_t *)calloc(size / 8 + 1, 1);
    if (!covered) return GCO_ENOMEM;
    int r = d - 1;
    int L = n < 9 ? n : 9;                 /* 2^9 bits = 64 bytes */
    int H = n - L;
    /* low flip patterns, grouped by weight */
    uint32_t low[512];
    int low_start[11], nlow = 0;
    for (int k = 0; k <= L; ++k) {
        low_start[k] = nlow;
        for (uint32_t e = 0; e < (1u << L); ++e)
            if (gco_weight(e) == (unsigned)k) low[nlow++] = e;
    }
    low_start[L + 1] = nlow;
    uint64_t m = 0, full = 0;
    int rc = GCO_OK;
    for (uint64_t p = 0; p < size; ++p) {
        uint32_t x = position_word(n, ordering, p);
        full += m;
        if (covered[x >> 3] & (1u << (x & 7))) continue;
        if (m == cap) { rc = GCO_ECAPACITY; break; }
        out[m++] = x;
        /* every flip set = high part of size kh <= r, low part of size <= r - kh */
        int pos[33];
        for (int kh = 0; kh <= r && kh <= H; ++kh) {
            for (int i = 0; i < kh; ++i) pos[i] = i;
            for (;;) {
                uint32_t y = x;
                for (int i = 0; i < kh; ++i) y ^= 1u << (L + pos[i]);
                int kl = r - kh < L ? r - kh : L;
                for (int j = 0; j < low_start[kl + 1]; ++j) {
                    uint32_t z = y ^ low[j];
                    covered[z >> 3] |= (uint8_t)(1u << (z & 7));
                }
                int i = kh - 1;
                while (i >= 0 && pos[i] == H - kh + i) --i;
                if (i < 0) break;
                ++pos[i];
                for (int j = i + 1; j < kh; ++j) pos[j] = pos[j - 1] + 1;
            }
        }
    }
    free(covered);
    *count = m;
    if (rc) return rc;
    if (w_full) *w_full = full;
    return GCO_OK;
}

/* ------------------------------------------------------------------ */
/* B-ordering (section "B-ordering Implementation")                    */
/* ------------------------------------------------------------------ */

/* table[0 .. 2^n) = the ordering induced by the ordered basis b_1..b_n
 * (basis[0] = b_1), by its recursive definition: start from (0); for
 * k = 1..n append b_k + v for every entry v of the list so far, in order.
 * The basis is not checked for independence (a dependent one repeats
 * vectors). */
int gco_border_table(int n, const uint32_t *basis, uint32_t *table)
{
    if (n < 1 || n > GCO_TABLE_MAX_N || !basis || !table) return GCO_EINVAL;
    uint64_t len = 1;
    table[0] = 0;
    for (int k = 1; k <= n; ++k) {
        for (uint64_t i = 0; i < len; ++i) table[len + i] = basis[k - 1] ^ table[i];
        len *= 2;
    }
    return GCO_OK;
}

/* ------------------------------------------------------------------ */
/* Constant weight candidates                                          */
/* ------------------------------------------------------------------ */

/* The vectors of weight w in F_2^n, in increasing value (ordering LEX or
 * GRLEX) or in the Cox-Little-O'Shea graded reverse lexicographic order
 * (GREVLEX), into table (room for cap entries).  *len = their number.
 * Walks every vector of F_2^n once. */
int gco_weight_class(int n, int w, int ordering, uint32_t *table, uint64_t cap, uint64_t *len)
{
    if (n < 1 || n > 32 || w < 0 || w > n || !len) return GCO_EINVAL;
    if (ordering != GCO_LEX && ordering != GCO_GRLEX && ordering != GCO_GREVLEX) return GCO_EINVAL;
    uint64_t size = 1ull << n, at = 0;
    for (uint64_t x = 0; x < size; ++x) {
        if (gco_weight((uint32_t)x) != (unsigned)w) continue;
        if (at == cap) return GCO_ECAPACITY;
        table[at++] = (uint32_t)x;
    }
    if (ordering == GCO_GREVLEX) {
        g_sort_n = n;
        qsort(table, at, sizeof(uint32_t), cmp_grevlex_ascending);
    }
    *len = at;
    return GCO_OK;
}

/* ------------------------------------------------------------------ */
/* Plain scan over an explicit candidate list                          */
/* ------------------------------------------------------------------ */

/* Does candidate x clash with accepted word c?  Distance below d, or, with
 * the self-orthogonality constraint, an odd number of common ones. */
static int clash(uint32_t x, uint32_t c, int d, int self_orth)
{
    if (gco_distance(x, c) < (unsigned)d) return 1;
    if (self_orth && (gco_weight(x & c) & 1u)) return 1;
    return 0;
}

/* The greedy algorithm over cand[0 .. ncand): every candidate is compared
 * with the accepted words newest first and appended when it clashes with
 * none; with self_orth it must also be orthogonal to itself (even weight).
 * Counters as in gco_greedy_scan. */
int gco_greedy_list(int n, int d, int self_orth, const uint32_t *cand, uint64_t ncand,
                    uint32_t *out, uint64_t cap, uint64_t *count, uint64_t *w_ee, uint64_t *w_full)
{
    if (n < 1 || n > 32 || d < 1 || !count || (!cand && ncand) || (!out && cap)) return GCO_EINVAL;
    uint64_t m = 0, ee = 0, full = 0;
    for (uint64_t p = 0; p < ncand; ++p) {
        uint32_t x = cand[p];
        int accept = !(self_orth && (gco_weight(x) & 1u));
        for (uint64_t i = m; accept && i-- > 0;) {
            ++ee;
            if (clash(x, out[i], d, self_orth)) accept = 0;
        }
        full += m;
        if (accept) {
            if (m == cap) { *count = m; return GCO_ECAPACITY; }
            out[m++] = x;
        }
    }
    *count = m;
    if (w_ee) *w_ee = ee;
    if (w_full) *w_full = full;
    return GCO_OK;
}

/* Certificate for a candidate list: words[0 .. count) is the greedy output
 * over cand[0 .. ncand) iff (a) the words are candidates, listed in candidate
 * order, (b) no two of them clash and, with self_orth, each has even weight,
 * and (c) every other candidate clashes with a listed word that comes earlier
 * in the list of candidates (or, with self_orth, has odd weight).  Brute
 * force; candidates must be distinct and below 2^20.  Returns 0 if it holds,
 * else 1 + the index of the failed rule. */
int gco_verify_certificate_list(int n, int d, int self_orth, const uint32_t *cand, uint64_t ncand,
                                const uint32_t *words, uint64_t count)
{
    if (n < 1 || n > 20 || d < 1 || !cand || (!words && count)) return GCO_EINVAL;
    uint64_t size = 1ull << n;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * size);
    int8_t *member = (int8_t *)calloc(size, 1);
    if (!pos || !member) { free(pos); free(member); return GCO_ENOMEM; }
    for (uint64_t y = 0; y < size; ++y) pos[y] = -1;
    for (uint64_t p = 0; p < ncand; ++p) pos[cand[p]] = (int64_t)p;
    int fail = 0;
    for (uint64_t i = 0; i < count && !fail; ++i) {
        if (words[i] >= size || pos[words[i]] < 0) fail = 1;
        else if (i && pos[words[i]] <= pos[words[i - 1]]) fail = 1;
        else member[words[i]] = 1;
    }
    for (uint64_t i = 0; i < count && !fail; ++i) {
        if (self_orth && (gco_weight(words[i]) & 1u)) { fail = 2; break; }
        for (uint64_t j = i + 1; j < count; ++j)
            if (clash(words[j], words[i], d, self_orth)) { fail = 2; break; }
    }
    for (uint64_t p = 0; p < ncand && !fail; ++p) {
        uint32_t y = cand[p];
        if (member[y]) continue;
        int rejected = self_orth && (gco_weight(y) & 1u);
        for (uint64_t i = 0; i < count && !rejected; ++i)
            if (pos[words[i]] < (int64_t)p && clash(y, words[i], d, self_orth)) rejected = 1;
        if (!rejected) fail = 3;
    }
    free(pos); free(member);
    return fail;
}

/* ------------------------------------------------------------------ */
/* Words of up to 64 coordinates (constant-weight walks past n = 32)   */
/* ------------------------------------------------------------------ */
/* Section "Some Examples" reports constant-weight codes up to length 35,
 * beyond 32-bit words.  The same rule over uint64 words: the weight-w
 * vectors of length n <= 64 in increasing value, and the plain newest-first
 * scan over them.  The 2^n walk is never materialised: the weight class is
 * listed directly, one w-subset of the coordinates at a time. */

unsigned gco_distance64(uint64_t a, uint64_t b)
{
    return (unsigned)__builtin_popcountll(a ^ b);
}

/* The weight-w vectors of length n in increasing value.  A vector is its set
 * of one-coordinates c_0 < c_1 < ... < c_{w-1}; increasing value is the order
 * that compares the largest coordinate first (then the next largest, ...).
 * The successor of a set: the first position i whose coordinate can move up
 * by one without meeting c_{i+1} (or n, for the last) moves up, and the
 * positions below it go back to 0, 1, ..., i-1. */
int gco_weight_class64(int n, int w, uint64_t *table, uint64_t cap, uint64_t *len)
{
    if (n < 1 || n > 64 || w < 0 || w > n || !len || (!table && cap)) return GCO_EINVAL;
    int c[64];
    for (int i = 0; i < w; ++i) c[i] = i;
    uint64_t at = 0;
    for (;;) {
        uint64_t x = 0;
        for (int i = 0; i < w; ++i) x |= 1ull << c[i];
        if (at == cap) { *len = at; return GCO_ECAPACITY; }
        table[at++] = x;
        int i = 0;
        while (i < w && c[i] + 1 == (i + 1 < w ? c[i + 1] : n)) ++i;
        if (i == w) break;  /* the last set: coordinates n-w .. n-1 */
        c[i] += 1;
        for (int k = 0; k < i; ++k) c[k] = k;
    }
    *len = at;
    return GCO_OK;
}

/* The plain scan over a list of uint64 candidates: each candidate is compared
 * with the accepted words newest first and accepted when none is closer than
 * d.  Counts the checks performed (W_ee) and those of the exhaustive scan
 * (W_full), as gco_greedy_list does for 32-bit words. */
int gco_greedy_list64(int n, int d, const uint64_t *cand, uint64_t ncand, uint64_t *out, uint64_t cap,
                      uint64_t *count, uint64_t *w_ee, uint64_t *w_full)
{
    if (n < 1 || n > 64 || d < 1 || !count || (!cand && ncand) || (!out && cap)) return GCO_EINVAL;
    uint64_t m = 0, ee = 0, full = 0;
    for (uint64_t p = 0; p < ncand; ++p) {
        uint64_t x = cand[p];
        int accept = 1;
        for (uint64_t i = m; accept && i-- > 0;) {
            ++ee;
            if (gco_distance64(x, out[i]) < (unsigned)d) accept = 0;
        }
        full += m;
        if (accept) {
            if (m == cap) { *count = m; return GCO_ECAPACITY; }
            out[m++] = x;
        }
    }
    *count = m;
    if (w_ee) *w_ee = ee;
    if (w_full) *w_full = full;
    return GCO_OK;
}

/* Certificate for uint64 words over a candidate list: 0 iff (a) the words are
 * candidates listed in candidate order, (b) no two are closer than d, and
 * (c) every other candidate is closer than d to a word that precedes it in
 * the list.  (1, 2 and 3 name the part that fails.)  O(ncand x count). */
int gco_verify_certificate64(int n, int d, const uint64_t *cand, uint64_t ncand, const uint64_t *words,
                             uint64_t count)
{
    if (n < 1 || n > 64 || d < 1 || (!cand && ncand) || (!words && count)) return GCO_EINVAL;
    uint64_t i = 0;
    for (uint64_t p = 0; p < ncand; ++p) {
        const uint64_t y = cand[p];
        if (i < count && y == words[i]) {
            for (uint64_t j = 0; j < i; ++j)
                if (gco_distance64(y, words[j]) < (unsigned)d) return 2;
            ++i;
            continue;
        }
        int rejected = 0;
        for (uint64_t j = 0; j < i && !rejected; ++j)
            if (gco_distance64(y, words[j]) < (unsigned)d) rejected = 1;
        if (!rejected) return 3;
    }
    return i == count ? 0 : 1;
}

"""CPU oracle for greedy binary code construction (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``greedy_oracle.c`` (plain C,
built with gcc) through ctypes and shares nothing with the HIP library.

Functions follow Paliwal et al., arXiv:1507.05398:
  * ``greedy_scan``   -- the greedy algorithm as defined in section "Greedy
    Algorithms and Different Orderings": candidates in order, each compared
    with every accepted word (newest first, stop at the first word closer than
    d), appended when none is closer than d.  Reports the checks performed
    (``w_ee``) and the exhaustive count (``w_full``).
  * ``greedy_ball``   -- the same output by ball marking (rejected exactly when
    within d-1 of an earlier accepted word); reports the same ``w_ee``.
  * ``order_table``   -- the four orderings of section "Ordering
    Implementation" (readings in ``greedy_oracle.c``).
  * ``verify_certificate`` -- independent characterisation of the output.
  * ``greedy_ball_wide`` -- ball marking for LEX/GRAY up to n = 32 (no W_ee).
  * ``border_table`` -- section "B-ordering Implementation": the ordering an
    ordered basis induces, by its recursive definition.
  * ``weight_class`` -- the weight-w vectors (constant-weight candidates).
  * ``greedy_list`` -- the plain scan over an explicit candidate list, with the
    optional self-orthogonality constraint of section "Self Orthogonal Greedy
    Codes Implementation".
  * ``verify_certificate_list`` -- the certificate for a candidate list.
  * ``weight_class64``, ``greedy_list64``, ``verify_certificate64`` -- the
    same for uint64 words of length n <= 64 (section "Some Examples" reports
    constant-weight codes up to length 35): weight classes listed subset by
    subset in increasing value, never through the 2^n walk.
  * ``distance`` -- Hamming distance, section "Hamming Distance".

Parity: the GREVLEX tie-break is "parity unpinned" beyond the textbook
definition; everything else is pinned by the CPU tests.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

LEX, GRAY, GRLEX, GREVLEX = 0, 1, 2, 3
ORDERINGS = {"lex": LEX, "gray": GRAY, "grlex": GRLEX, "grevlex": GREVLEX}

OK, EINVAL, ECAPACITY, ENOMEM, EFAIL = 0, -1, -2, -4, -5

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIBRARY
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SOURCE):
        _build.build()
    lib = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.gco_distance.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.gco_distance.restype = ctypes.c_uint
    lib.gco_weight.argtypes = [ctypes.c_uint32]
    lib.gco_weight.restype = ctypes.c_uint
    lib.gco_order_table.argtypes = [ctypes.c_int, ctypes.c_int, u32p]
    lib.gco_order_table.restype = ctypes.c_int
    lib.gco_greedy_scan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p,
                                    ctypes.c_uint64, u64p, u64p, u64p]
    lib.gco_greedy_scan.restype = ctypes.c_int
    lib.gco_greedy_ball.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p,
                                    ctypes.c_uint64, u64p, u64p, u64p]
    lib.gco_greedy_ball.restype = ctypes.c_int
    lib.gco_verify_certificate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p,
                                           ctypes.c_uint64]
    lib.gco_verify_certificate.restype = ctypes.c_int
    lib.gco_greedy_ball_wide.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p,
                                         ctypes.c_uint64, u64p, u64p]
    lib.gco_greedy_ball_wide.restype = ctypes.c_int
    lib.gco_border_table.argtypes = [ctypes.c_int, u32p, u32p]
    lib.gco_border_table.restype = ctypes.c_int
    lib.gco_weight_class.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p, ctypes.c_uint64, u64p]
    lib.gco_weight_class.restype = ctypes.c_int
    lib.gco_greedy_list.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p, ctypes.c_uint64,
                                    u32p, ctypes.c_uint64, u64p, u64p, u64p]
    lib.gco_greedy_list.restype = ctypes.c_int
    lib.gco_verify_certificate_list.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p,
                                                ctypes.c_uint64, u32p, ctypes.c_uint64]
    lib.gco_verify_certificate_list.restype = ctypes.c_int
    lib.gco_distance64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gco_distance64.restype = ctypes.c_uint
    lib.gco_weight_class64.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64, u64p]
    lib.gco_weight_class64.restype = ctypes.c_int
    lib.gco_greedy_list64.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64, u64p, ctypes.c_uint64,
                                      u64p, u64p, u64p]
    lib.gco_greedy_list64.restype = ctypes.c_int
    lib.gco_verify_certificate64.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64, u64p,
                                             ctypes.c_uint64]
    lib.gco_verify_certificate64.restype = ctypes.c_int
    _lib = lib
    return lib


def _u32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"{what} failed with code {rc}")
        self.rc = rc


def distance(a: int, b: int) -> int:
    """Hamming distance: popcount(a XOR b)."""
    return int(_load().gco_distance(a, b))


def order_table(n: int, ordering: int) -> np.ndarray:
    """All 2^n words of F_2^n in the given ordering (n <= 28)."""
    out = np.zeros(1 << n, dtype=np.uint32)
    rc = _load().gco_order_table(n, ordering, _u32(out))
    if rc:
        raise OracleError(rc, "order_table")
    return out


def _bound(n: int) -> int:
    # Worst case: d = 1 keeps every vector.
    return 1 << n


def greedy_scan(n: int, d: int, ordering: int, cap: int = None):
    """Plain-scan greedy.  Returns (words uint32[|C|], w_ee, w_full)."""
    cap = _bound(n) if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    count, ee, full = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = _load().gco_greedy_scan(n, d, ordering, _u32(out), cap, ctypes.byref(count),
                                 ctypes.byref(ee), ctypes.byref(full))
    if rc:
        raise OracleError(rc, "greedy_scan")
    return out[: count.value].copy(), ee.value, full.value


def greedy_ball(n: int, d: int, ordering: int, cap: int = None, want_w_ee: bool = False,
                want_w_full: bool = False):
    """Ball-marking greedy.  Returns (words, w_ee or None), or
    (words, w_ee or None, w_full) when want_w_full."""
    cap = _bound(n) if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    count, ee, full = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = _load().gco_greedy_ball(n, d, ordering, _u32(out), cap, ctypes.byref(count),
                                 ctypes.byref(ee) if want_w_ee else None, ctypes.byref(full))
    if rc:
        raise OracleError(rc, "greedy_ball")
    words = out[: count.value].copy()
    if want_w_full:
        return words, (ee.value if want_w_ee else None), full.value
    return words, (ee.value if want_w_ee else None)


def verify_certificate(n: int, d: int, ordering: int, words) -> int:
    """0 if ``words`` is the greedy code for (n, d, ordering), else 1/2/3 =
    order / distance / maximality rule failed (n <= 20, brute force)."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.size == 0:
        w = np.zeros(1, dtype=np.uint32)
        return int(_load().gco_verify_certificate(n, d, ordering, _u32(w), 0))
    return int(_load().gco_verify_certificate(n, d, ordering, _u32(w), w.size))


def greedy_ball_wide(n: int, d: int, ordering: int, cap: int = 1 << 22):
    """Ball marking for LEX or GRAY at any n <= 32.  Returns (words, w_full)."""
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    count, full = ctypes.c_uint64(), ctypes.c_uint64()
    rc = _load().gco_greedy_ball_wide(n, d, ordering, _u32(out), cap, ctypes.byref(count),
                                      ctypes.byref(full))
    if rc:
        raise OracleError(rc, "greedy_ball_wide")
    return out[: count.value].copy(), full.value


def border_table(n: int, basis) -> np.ndarray:
    """The 2^n vectors in the order the basis b_1..b_n (basis[0] = b_1)
    induces: 0, b_1, b_2, b_2+b_1, b_3, ... (n <= 28)."""
    b = np.ascontiguousarray(basis, dtype=np.uint32)
    if b.size != n:
        raise ValueError("basis needs n words")
    out = np.zeros(1 << n, dtype=np.uint32)
    rc = _load().gco_border_table(n, _u32(b), _u32(out))
    if rc:
        raise OracleError(rc, "border_table")
    return out


def weight_class(n: int, w: int, ordering: int) -> np.ndarray:
    """The weight-w vectors of F_2^n in increasing value (LEX, GRLEX) or in
    graded reverse lexicographic order (GREVLEX)."""
    cap = max(1, math.comb(n, w)) if 0 <= w <= n else 1
    out = np.zeros(cap, dtype=np.uint32)
    ln = ctypes.c_uint64()
    rc = _load().gco_weight_class(n, w, ordering, _u32(out), cap, ctypes.byref(ln))
    if rc:
        raise OracleError(rc, "weight_class")
    return out[: ln.value].copy()


def greedy_list(n: int, d: int, candidates, self_orth: bool = False, cap: int = None):
    """Plain-scan greedy over an explicit candidate list (optionally
    self-orthogonal).  Returns (words, w_ee, w_full)."""
    cand = np.ascontiguousarray(candidates, dtype=np.uint32)
    cap = max(cand.size, 1) if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    count, ee, full = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = _load().gco_greedy_list(n, d, int(bool(self_orth)), _u32(cand) if cand.size else None,
                                 cand.size, _u32(out), cap, ctypes.byref(count), ctypes.byref(ee),
                                 ctypes.byref(full))
    if rc:
        raise OracleError(rc, "greedy_list")
    return out[: count.value].copy(), ee.value, full.value


def verify_certificate_list(n: int, d: int, candidates, words, self_orth: bool = False) -> int:
    """0 if ``words`` is the greedy output over ``candidates``; else 1/2/3 =
    order / clash / maximality rule failed (n <= 20)."""
    cand = np.ascontiguousarray(candidates, dtype=np.uint32)
    w = np.ascontiguousarray(words, dtype=np.uint32)
    wp = _u32(w) if w.size else None
    return int(_load().gco_verify_certificate_list(n, d, int(bool(self_orth)), _u32(cand), cand.size,
                                                   wp, w.size))


def distance64(a: int, b: int) -> int:
    """Hamming distance of two words of up to 64 coordinates."""
    return int(_load().gco_distance64(a, b))


def weight_class64(n: int, w: int) -> np.ndarray:
    """The weight-w vectors of length n <= 64 in increasing value (uint64)."""
    cap = max(1, math.comb(n, w)) if 0 <= w <= n else 1
    out = np.zeros(cap, dtype=np.uint64)
    ln = ctypes.c_uint64()
    rc = _load().gco_weight_class64(n, w, _u64(out), cap, ctypes.byref(ln))
    if rc:
        raise OracleError(rc, "weight_class64")
    return out[: ln.value].copy()


def greedy_list64(n: int, d: int, candidates, cap: int = None):
    """Plain-scan greedy over a list of uint64 candidates (n <= 64).  Returns
    (words, w_ee, w_full)."""
    cand = np.ascontiguousarray(candidates, dtype=np.uint64)
    cap = max(cand.size, 1) if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    count, ee, full = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = _load().gco_greedy_list64(n, d, _u64(cand) if cand.size else None, cand.size, _u64(out), cap,
                                   ctypes.byref(count), ctypes.byref(ee), ctypes.byref(full))
    if rc:
        raise OracleError(rc, "greedy_list64")
    return out[: count.value].copy(), ee.value, full.value


def verify_certificate64(n: int, d: int, candidates, words) -> int:
    """0 if ``words`` is the greedy output over ``candidates`` (uint64, n <=
    64); else 1/2/3 = order / clash / maximality rule failed."""
    cand = np.ascontiguousarray(candidates, dtype=np.uint64)
    w = np.ascontiguousarray(words, dtype=np.uint64)
    return int(_load().gco_verify_certificate64(n, d, _u64(cand) if cand.size else None, cand.size,
                                                _u64(w) if w.size else None, w.size))

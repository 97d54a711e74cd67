"""The stored oracle references cover every workload instance (CPU only).

The references themselves are written by tests/golden/make_expected.py, which
calls only the oracle; these checks make a missing reference a failure rather
than a silently skipped parity case."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_expected  # noqa: E402  (instance lists only)
from paper_1507_05398_amd import workloads  # noqa: E402


def rows(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def test_every_workload_instance_has_a_reference():
    have = {r[0] for r in rows("expected_codes.txt")}
    want = [f"{n}_{d}_{o}" for n, d, o in make_expected.instances()]
    missing = [k for k in want if k not in have]
    assert not missing, missing
    assert len(want) == 75


def test_served_references_cover_the_stream():
    have = {r[0] for r in rows("expected_served.txt")}
    want = {f"{n}_{d}_{o}" for _, n, d, o in workloads.served_jobs(seed=1507, count=10000, rate=1.0)}
    assert have == want
    assert sum(int(k.split("_")[0]) > 20 for k in want) == 105


def test_batch_references_match_the_instances():
    got = [(int(r[0]), r[1]) for r in rows("expected_batch.txt")]
    want = [(i, f"{n}_{d}_{o}") for i, (n, d, o) in enumerate(workloads.batched_instances())]
    assert got == want

"""GPU parity of the batched launch and the job server against the oracle.

Every code built in a batch or through the server must be the exact list the
oracle produces for its (n, d, ordering); a job's result must not depend on
what else shares the GPU with it.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1507_05398_amd as gc
from paper_1507_05398_amd import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    gc.load()
    return torch


def ref(n, d, o):
    return oracle.greedy_ball(n, d, oracle.ORDERINGS[o])[0]


SMALL = workloads.batched_instances(seed=7, count=48, n_lo=8, n_hi=17, d_lo=2, d_hi=9)


@pytest.mark.parametrize("teams", [1, 2, 4, 8])
def test_batch_matches_oracle(teams):
    log(f"[gpu] batch teams={teams} jobs={len(SMALL)}")
    words, info, ms = gc.greedy_code_batch(SMALL, teams=teams)
    for (n, d, o), w, inf in zip(SMALL, words, info):
        assert inf["status"] == 0
        assert np.array_equal(w.cpu().numpy().view(np.uint32), ref(n, d, o)), (n, d, o)


def test_batch_with_degenerate_and_single_jobs():
    inst = [(5, 1, "gray"), (6, 7, "lex"), (10, 10, "grevlex"), (1, 1, "lex"), (12, 3, "grlex")]
    words, info, _ = gc.greedy_code_batch(inst, teams=8)
    for (n, d, o), w in zip(inst, words):
        assert np.array_equal(w.cpu().numpy().view(np.uint32), ref(n, d, o)), (n, d, o)
    words, info, _ = gc.greedy_code_batch([(16, 4, "grlex")], teams=1)
    assert np.array_equal(words[0].cpu().numpy().view(np.uint32), ref(16, 4, "grlex"))


def load_expected():
    path = os.path.join(HERE, "golden", "expected_batch.txt")
    out = {}
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and not line.startswith("#"):
                idx, key, m, digest = line.split()[:4]
                out[int(idx)] = (key, int(m), digest)
    return out


def test_batched_workload_256_instances():
    import hashlib
    exp = load_expected()
    inst = workloads.batched_instances()
    assert len(exp) == len(inst), "tests/golden/expected_batch.txt is incomplete"
    t = time.time()
    words, info, ms = gc.greedy_code_batch(inst, teams=8)
    log(f"[gpu] 256-instance batch: {ms:.1f} ms kernel, {time.time() - t:.1f} s wall")
    for i, ((n, d, o), w) in enumerate(zip(inst, words)):
        key, m, digest = exp[i]
        assert key == f"{n}_{d}_{o}"
        got = w.cpu().numpy().astype("<u4")
        assert len(got) == m and hashlib.sha256(got.tobytes()).hexdigest() == digest, (i, key)


JOBS = [(14, 3, "lex"), (16, 5, "gray"), (12, 4, "grlex"), (15, 6, "grevlex"), (18, 3, "gray"),
        (10, 2, "lex"), (17, 8, "grlex"), (13, 7, "lex"), (20, 4, "grevlex"), (11, 3, "gray")]
# wide jobs (2^n * capacity >= 2^38) for the servers with a wide team
WIDE_JOBS = [(22, 3, "grlex"), (23, 4, "lex")]


def wait_all(srv, tickets, timeout=120.0):
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            st, _ = srv.poll(t)
            if st in (gc.GC_JOB_DONE, gc.GC_JOB_FAILED):
                pending.discard(t)
        assert time.time() - t0 < timeout, "server jobs did not finish"
        time.sleep(0.001)


@pytest.mark.parametrize("teams", [8, 2])
def test_server_alone_and_in_the_mix_match_oracle(teams):
    expected = [ref(*j) for j in JOBS + WIDE_JOBS]
    with gc.Server(arena_bytes=64 << 20, teams=teams) as srv:
        # alone: one job at a time
        for j, e in zip(JOBS + WIDE_JOBS, expected):
            log(f"[gpu] server alone {j}")
            t = srv.submit(*j)
            wait_all(srv, [t])
            assert np.array_equal(srv.fetch(t), e), j
            srv.release(t)
        # in the mix: everything at once, twice over
        tickets = [srv.submit(*j) for j in JOBS + WIDE_JOBS + JOBS + WIDE_JOBS]
        wait_all(srv, tickets)
        for t, e in zip(tickets, expected + expected):
            assert np.array_equal(srv.fetch(t), e)
            st = srv.stats(t)
            assert st["count"] == len(e)
            srv.release(t)


def test_server_admission_waits_for_memory():
    # An arena that holds one n=16 d=3 code at a time: later jobs wait until
    # earlier ones are released.
    cap_bytes = gc.greedy_code_capacity(16, 3) * 4
    jobs = [(16, 3, "lex"), (16, 3, "gray"), (16, 3, "grlex"), (16, 3, "grevlex")]
    with gc.Server(arena_bytes=cap_bytes + 256, teams=4) as srv:
        tickets = [srv.submit(*j) for j in jobs]
        states = [srv.poll(t)[0] for t in tickets]
        assert states[1:] == [gc.GC_JOB_WAITING] * 3
        done = {}
        t0 = time.time()
        while len(done) < len(jobs):
            for t, j in zip(tickets, jobs):
                if t in done:
                    continue
                st, _ = srv.poll(t)
                if st == gc.GC_JOB_DONE:
                    done[t] = srv.fetch(t)
                    srv.release(t)
            assert time.time() - t0 < 120
            time.sleep(0.001)
        for t, j in zip(tickets, jobs):
            assert np.array_equal(done[t], ref(*j)), j


def test_server_relaunches_after_idle():
    with gc.Server(arena_bytes=16 << 20, teams=2) as srv:
        t = srv.submit(15, 3, "lex")
        wait_all(srv, [t])
        time.sleep(0.5)  # longer than the kernel's idle period
        t2 = srv.submit(13, 4, "gray")
        wait_all(srv, [t2])
        assert np.array_equal(srv.fetch(t), ref(15, 3, "lex"))
        assert np.array_equal(srv.fetch(t2), ref(13, 4, "gray"))


def test_batch_graph_replays_match_oracle():
    """A captured batch replayed three times, with eager work and cleared
    outputs between the replays: every replay rebuilds every code."""
    import torch
    ords = ["lex", "gray", "grlex", "grevlex"]
    insts = [(10 + (i % 7), 3 + (i % 5), ords[i % 4]) for i in range(20)]
    refs = [oracle.greedy_ball(n, d, oracle.ORDERINGS[o])[0] for n, d, o in insts]
    plan = gc.BatchPlan(insts)
    print(f"[graph] capture {len(insts)} jobs", flush=True)
    with plan.graph() as g:
        for rep in range(3):
            for w, c in plan.bufs:
                w.fill_(-1)
                c.zero_()
            words, _ = gc.device_code(12, 3, "gray")   # eager work between replays
            np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32),
                                          oracle.greedy_ball(12, 3, oracle.ORDERINGS["gray"])[0])
            torch.cuda.synchronize()
            print(f"[graph] replay {rep}", flush=True)
            g.launch()
            g.wait()
            for (n, d, o), ref, t, (w, c), inf in zip(insts, refs, plan.results(), plan.bufs, plan.info()):
                assert inf["status"] == gc.GC_OK and inf["count"] == len(ref)
                assert int(c.item()) == len(ref)
                np.testing.assert_array_equal(t.cpu().numpy().view(np.uint32), ref)


def test_served_workload_sample_matches_oracle():
    """The served workload (seeded Poisson stream: n in [10, 26] skewed small,
    d in [3, 10], random ordering): its first 400 jobs with n <= 20, all
    submitted at once to an 8-team server whose 512 KiB arena holds only part
    of their worst-case codes (admission by memory binds: jobs wait until
    finished ones are released); every result is compared with the oracle."""
    jobs = [j for j in workloads.served_jobs(seed=1507, count=2000, rate=1.0) if j[1] <= 20][:400]
    log(f"[served] {len(jobs)} jobs")
    got = {}
    waited = 0
    with gc.Server(arena_bytes=512 << 10, teams=8) as srv:
        open_tickets = {srv.submit(n, d, o): i for i, (_, n, d, o) in enumerate(jobs)}
        deadline = time.time() + 90
        while open_tickets and time.time() < deadline:
            for tk in list(open_tickets):
                st, _ = srv.poll(tk)
                waited += st == gc.GC_JOB_WAITING
                if st >= gc.GC_JOB_DONE:
                    got[open_tickets.pop(tk)] = srv.fetch(tk)
                    srv.release(tk)
        assert not open_tickets, f"{len(open_tickets)} jobs unfinished"
    assert waited > 0  # some jobs did wait for memory
    for i, (_, n, d, o) in enumerate(jobs):
        np.testing.assert_array_equal(got[i], ref(n, d, o))


def load_served_digests():
    path = os.path.join(HERE, "golden", "expected_served.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, m, digest = line.split()
            out[key] = (int(m), digest)
    return out


def test_served_triples_match_oracle_digests():
    """Every distinct (n, d, ordering) of the served workload's stream (seed
    1507, 10,000 jobs: n in [10, 26], d in [3, 10], all four orderings)
    through a server with a wide team (6 XCDs) and two narrow teams and a
    16 MiB arena (admission binds; narrow jobs pass waiting wide ones), each
    result against the oracle's digest."""
    import hashlib
    exp = load_served_digests()
    triples = sorted({(n, d, o) for _, n, d, o in workloads.served_jobs(seed=1507, count=10000, rate=1.0)},
                     key=lambda t: (-t[0], t[1], t[2]))
    keys = [f"{n}_{d}_{o}" for n, d, o in triples]
    assert set(keys) == set(exp), "tests/golden/expected_served.txt does not match the served stream"
    log(f"[served] {len(triples)} distinct triples, {sum(t[0] > 20 for t in triples)} with n > 20")
    got, waited = {}, 0
    with gc.Server(arena_bytes=16 << 20, teams=2) as srv:
        open_tickets = {srv.submit(n, d, o): k for (n, d, o), k in zip(triples, keys)}
        deadline = time.time() + 300
        while open_tickets and time.time() < deadline:
            for tk in list(open_tickets):
                st, _ = srv.poll(tk)
                waited += st == gc.GC_JOB_WAITING
                if st >= gc.GC_JOB_DONE:
                    w = srv.fetch(tk)
                    got[open_tickets.pop(tk)] = (len(w), hashlib.sha256(w.astype("<u4").tobytes()).hexdigest())
                    srv.release(tk)
            time.sleep(0.0005)
        assert not open_tickets, f"{len(open_tickets)} jobs unfinished"
    assert waited > 0
    bad = [k for k in keys if got[k] != exp[k]]
    assert not bad, f"served results differ from the oracle for {bad[:10]}"


def test_server_wait_expiry_fails_jobs_and_drains():
    """With a zero spin limit every device-side wait expires at once: the
    server's jobs must end FAILED with GC_ETIMEOUT, drain must return, and the
    server must refuse further jobs (no endless relaunch)."""
    os.environ["GC_SPIN_LIMIT"] = "0"
    try:
        with gc.Server(arena_bytes=16 << 20, teams=4) as srv:
            jobs = [(14, 3, "lex"), (13, 4, "gray"), (12, 5, "grlex"), (24, 4, "gray")]
            tickets = [srv.submit(*j) for j in jobs]
            srv.drain(timeout_ms=60000)
            states = [srv.poll(t)[0] for t in tickets]
            assert all(s in (gc.GC_JOB_DONE, gc.GC_JOB_FAILED) for s in states), states
            assert gc.GC_JOB_FAILED in states
            for t, j, s in zip(tickets, jobs, states):
                if s == gc.GC_JOB_FAILED:
                    with pytest.raises(gc.GreedyCodeError) as e:
                        srv.fetch(t)
                    assert e.value.rc == gc.GC_ETIMEOUT
                else:
                    assert np.array_equal(srv.fetch(t), ref(*j))
                srv.release(t)
            with pytest.raises(gc.GreedyCodeError) as e:
                srv.submit(10, 3, "lex")
            assert e.value.rc == gc.GC_ETIMEOUT
    finally:
        del os.environ["GC_SPIN_LIMIT"]
    # the library keeps working afterwards
    with gc.Server(arena_bytes=16 << 20, teams=4) as srv:
        t = srv.submit(13, 3, "gray")
        wait_all(srv, [t])
        assert np.array_equal(srv.fetch(t), ref(13, 3, "gray"))

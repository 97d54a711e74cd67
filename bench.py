#!/usr/bin/env python3
"""Benchmark: greedy code construction on one MI355X.

A step is one pass of the whole construction over the workload: every
instance (n, d, ordering) is built from scratch on the GPU (all 2^n candidate
positions screened, resolved and committed).  The default workload is the
screens at n = 24..28: the four orderings x d in {3, 4, 5, 6, 8} at n=24 (the
n=24 part of the sweep) plus lex and Gray at n in {26, 28} with d=3 (24
instances).  ``--workload sweep`` runs the whole sweep (four orderings x n in
{20, 22, 24} x d in {3, 4, 5, 6, 8}, plus n=23 with d=7: 64 instances),
``--workload large`` only the n=26/28 screens.

The headline value is algorithmic distance checks per second: the sum over
instances of W_ee (checks done by a sequential newest-first scan with early
exit, counted by the CPU oracle and stored in tests/golden/expected_codes.txt)
divided by the wall time of the step.

Also measured (one JSON line in all):
  * roofline of greedy_code_kernel, the single-code kernel, over every timed
    launch of the workload: algorithmic checks (W_ee) per launch over the
    launch's duration (HIP events on the launch stream, recorded by the
    library);
  * batched: the 256-instance workload (seed 1507) as one persistent launch,
    as a captured graph and as a loop of plain per-instance calls on the same
    buffers, with the built-in defaults and then autotuned;
  * served: a seeded Poisson stream of 10,000 jobs through the job server
    (continuous batching) with p50/p99/max latency, next to the same jobs one
    at a time and all at once;
  * cpu_baseline: the oracle on a bounded sample of the workload, one host
    thread.
Every code built is compared with the oracle's stored digest.

``--copy-calibration`` only runs a device copy of known size (for scaling
the FETCH_SIZE / WRITE_SIZE counters) and prints its bytes.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ORDS = ["lex", "gray", "grlex", "grevlex"]
# MI355X: 256 CUs x 64 int32 lanes per clock x 2.4 GHz.  The vector-ALU screen
# costs 2.5 lane-ops per distance check (v_xor_b32 + v_bcnt_u32_b32 + half a
# v_min3_u32): PEAK_GCHECKS is that screen's ceiling.
VALU_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_CHECK = 2.5
PEAK_GCHECKS = VALU_LANE_OPS / OPS_PER_CHECK / 1e9
# The default screen runs on the matrix cores: bits as signed bytes, a check is
# an int8 dot product.  Its roofline is MI355X's dense int8 MFMA peak, with 2n
# int8 operations (n multiply-adds) per check of n-bit words.  Two check-rate
# ceilings bound it: the instruction's 32-byte rows (64 operations per check
# whatever n is) and the max-fold of the products on the vector ALU (half a
# lane-op per check: v_max3_i32 folds two products).
INT8_PEAK_TOPS = 5000.0
MFMA_CHECKS_PEAK_G = INT8_PEAK_TOPS * 1e12 / 64 / 1e9
FOLD_CHECKS_PEAK_G = VALU_LANE_OPS / 0.5 / 1e9


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_instances():
    out = []
    for o in ORDS:
        for n in (20, 22, 24):
            for d in (3, 4, 5, 6, 8):
                out.append((n, d, o))
        out.append((23, 7, o))
    return out


def large_instances():
    return [(n, 3, o) for n in (26, 28) for o in ("lex", "gray")]


def screens_24_28():
    return [i for i in sweep_instances() if i[0] == 24] + large_instances()


def load_expected():
    path = os.path.join(ROOT, "tests", "golden", "expected_codes.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, m, digest, w_ee, w_full = line.split()
            out[key] = (int(m), digest, int(w_ee), int(w_full))
    return out


def load_expected_batch():
    path = os.path.join(ROOT, "tests", "golden", "expected_batch.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            idx, key, m, digest, w_ee, w_full = line.split()
            out[int(idx)] = (key, int(m), digest, int(w_ee), int(w_full))
    return out


def digest_of(t):
    return hashlib.sha256(t.cpu().numpy().astype("<u4").tobytes()).hexdigest()


def measured_traffic():
    """HBM bytes per greedy_code_kernel launch from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "greedy_code_kernel_screens24_28_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    h = hashlib.sha256()
    for name in ("greedy_code.hip", "gc_internal.h"):
        with open(os.path.join(ROOT, "paper_1507_05398_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Bounded sample of the n=24..28 screens for the CPU baseline: instances the
# plain scan finishes in about 20 s together on one host core (6.2e9 checks).
CPU_SAMPLE = [(24, 8, "lex"), (24, 8, "gray"), (24, 8, "grlex"), (24, 8, "grevlex"), (24, 6, "grlex")]


def cpu_baseline(expected, gpu_ms):
    """The CPU oracle as it stands, one host thread: the plain newest-first
    scan (the definition) on CPU_SAMPLE, in algorithmic checks per second,
    next to the GPU's time for the same instances; plus the oracle's ball
    marking (a different exact algorithm) on n=26 d=3 lex."""
    import oracle
    t_all, checks, rows = 0.0, 0, []
    for n, d, o in CPU_SAMPLE:
        t0 = time.perf_counter()
        _, w_ee, _ = oracle.greedy_scan(n, d, oracle.ORDERINGS[o])
        dt = time.perf_counter() - t0
        key = f"{n}_{d}_{o}"
        assert w_ee == expected[key][2]
        t_all += dt
        checks += w_ee
        rows.append({"instance": key, "cpu_s": round(dt, 3), "gpu_ms": gpu_ms.get(key)})
    t0 = time.perf_counter()
    oracle.greedy_ball(26, 3, oracle.LEX)
    ball_s = time.perf_counter() - t0
    return {"value": round(checks / t_all / 1e9, 4), "unit": "Gchecks/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "plain newest-first scan (one thread) on 5 of the 24 screens: n=24 d=8 (4 orderings) "
                      f"and d=6 grlex; {checks:.3e} checks in {t_all:.1f} s",
            "per_instance": rows,
            "ball_marking_26_3_lex_s": round(ball_s, 3),
            "ball_marking_note": "exact, but a different algorithm (marks the radius d-1 ball of each "
                                 "accepted word) with no distance checks; GPU time for the same code: "
                                 f"{gpu_ms.get('26_3_lex')} ms"}


def _oracle_time(task):
    import oracle
    how, (n, d, o) = task
    t0 = time.perf_counter()
    if how == "scan":
        words, w_ee, _ = oracle.greedy_scan(n, d, oracle.ORDERINGS[o])
    else:
        words, w_ee = oracle.greedy_ball(n, d, oracle.ORDERINGS[o], want_w_ee=True)
    return how, f"{n}_{d}_{o}", time.perf_counter() - t0, len(words), w_ee


def oracle_times(expected, workers):
    """Every screen of the n=24..28 workload on the host CPU, each instance on
    one thread (`workers` instances at a time): the plain scan (the
    definition) on the n=24 instances, ball marking on n=26/28 (the scan
    would take hours there).  Prints one JSON line per instance."""
    from concurrent.futures import ProcessPoolExecutor
    tasks = [("scan", i) for i in screens_24_28() if i[0] == 24] + [("ball", i) for i in large_instances()]
    tasks.sort(key=lambda t: -expected[f"{t[1][0]}_{t[1][1]}_{t[1][2]}"][2])
    from concurrent.futures import as_completed
    with ProcessPoolExecutor(workers) as ex:
        for fut in as_completed([ex.submit(_oracle_time, t) for t in tasks]):
            how, key, dt, m, w_ee = fut.result()
            ok = m == expected[key][0] and w_ee == expected[key][2]
            print(json.dumps({"instance": key, "algorithm": how, "cpu_s": round(dt, 3), "threads": 1,
                              "checks_per_s": round(w_ee / dt, 1), "matches_reference": ok,
                              "cpu": cpu_model()}), flush=True)


class LaunchLog:
    """Kernel time and algorithmic checks of every timed greedy_code_kernel
    launch, and each instance's launch times."""

    def __init__(self):
        self.ms, self.w_ee, self.executed, self.launches = 0.0, 0, 0, 0
        self.ops = 0  # int8 operations: 2n per algorithmic check
        self.per_key = {}

    def add(self, key, stats, w_ee):
        self.ms += stats["kernel_ms"]
        self.w_ee += w_ee
        self.ops += 2 * int(key.split("_")[0]) * w_ee
        self.executed += stats["checks_near"] + stats["checks_deep"] + stats["checks_pairs"]
        self.launches += 1
        self.per_key.setdefault(key, []).append(stats["kernel_ms"])

    def median_ms(self):
        return {k: round(sorted(v)[len(v) // 2], 3) for k, v in self.per_key.items()}

    def gchecks(self):
        return self.w_ee / (self.ms / 1e3) / 1e9 if self.ms else 0.0

    def tops(self):
        return self.ops / (self.ms / 1e3) / 1e12 if self.ms else 0.0


def bench_sweep(gc, torch, insts, expected, steps, warmup):
    bufs = []
    for n, d, o in insts:
        cap = gc.greedy_code_capacity(n, d)
        bufs.append((torch.empty(cap, dtype=torch.int32, device="cuda"),
                     torch.zeros(1, dtype=torch.int64, device="cuda")))
    stream = torch.cuda.current_stream()
    own = LaunchLog()

    def one_step(record):
        for (n, d, o), (w, c) in zip(insts, bufs):
            st = gc.greedy_code_device_ex(n, d, o, w, c, stream=stream)
            if record:
                own.add(f"{n}_{d}_{o}", st, expected[f"{n}_{d}_{o}"][2])

    for _ in range(warmup):
        one_step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        one_step(True)
        progress(f"step {k + 1}/{steps}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # Bit-exact check of the last step's output (outside the timed region).
    for (n, d, o), (w, c) in zip(insts, bufs):
        m, dig, _, _ = expected[f"{n}_{d}_{o}"]
        got = w[: int(c.item())]
        if len(got) != m or digest_of(got) != dig:
            raise SystemExit(f"MISMATCH n={n} d={d} {o}: {len(got)} words vs {m}")
    return wall, own


def bench_batched(gc, torch, steps, warmup):
    """The 256-instance batched workload (seed 1507): one persistent launch
    over every instance (teams pull jobs longest first) against a loop of
    plain per-instance calls on the same preallocated buffers, first with the
    built-in defaults, then autotuned (outside the timed region: the
    team-count tuner of the batch with the built-in per-instance defaults
    and again after the per-instance tuner ran on every distinct instance;
    the faster of the two on the batch is kept).  Every result is compared
    with the oracle's digest."""
    from paper_1507_05398_amd import workloads
    insts = workloads.batched_instances()
    expected = load_expected_batch()
    plan = gc.BatchPlan(insts)
    stream = torch.cuda.current_stream()

    def verify(what):
        for i, (w, c) in enumerate(plan.bufs):
            key, m, dig, _, _ = expected[i]
            if int(c.item()) != m or digest_of(w[:m]) != dig:
                raise SystemExit(f"{what} MISMATCH job {i} ({key})")

    def median(v):
        return sorted(v)[len(v) // 2]

    def measure(teams):
        for _ in range(warmup):
            plan.run(teams=teams, stream=stream)
        torch.cuda.synchronize()
        walls, kms = [], []
        for _ in range(steps):
            for w, c in plan.bufs:
                c.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            kms.append(plan.run(teams=teams, stream=stream))
            walls.append(time.perf_counter() - t0)
        verify("BATCH")
        # The same batch captured once into a HIP graph and replayed.
        gwalls = []
        with plan.graph(teams=teams) as g:
            g.launch(stream)
            g.wait()
            for _ in range(steps):
                for w, c in plan.bufs:
                    c.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.launch(stream)
                g.wait()
                gwalls.append(time.perf_counter() - t0)
        verify("GRAPH")

        def plain():
            for (n, d, o), (w, c) in zip(insts, plan.bufs):
                gc.greedy_code_device_ex(n, d, o, w, c, stream=stream)
        for _ in range(warmup):
            plain()
        torch.cuda.synchronize()
        pwalls = []
        for _ in range(steps):
            for w, c in plan.bufs:
                c.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plain()
            torch.cuda.synchronize()
            pwalls.append(time.perf_counter() - t0)
        verify("PLAIN")
        tb, tg, tp = median(walls), median(gwalls), median(pwalls)
        return {"teams": teams or "default", "batched_codes_per_s": round(len(insts) / tb, 2),
                "batched_ms": round(tb * 1e3, 3), "batched_kernel_ms": round(median(kms), 3),
                "graph_codes_per_s": round(len(insts) / tg, 2),
                "plain_codes_per_s": round(len(insts) / tp, 2), "plain_ms": round(tp * 1e3, 3),
                "speedup_vs_plain": round(tp / tb, 3)}

    gc.greedy_code_tune_reset()
    default = measure(0)
    progress(f"batched (defaults): {default['batched_ms']} ms")
    # Two candidates, each with its best team count on this batch: the
    # built-in per-instance defaults, and the per-instance tunings (picked on
    # each instance alone, where a job has the whole GPU).  The faster on the
    # batch itself is kept.
    t0 = time.perf_counter()
    teams_def, ms_def = plan.tune(stream=stream)
    for n, d, o in sorted(set(insts)):
        gc.greedy_code_tune(n, d, o, stream=stream)
    teams_inst, ms_inst = plan.tune(stream=stream)
    instance_tunings = ms_inst < ms_def
    if not instance_tunings:
        gc.greedy_code_tune_reset()
    teams = teams_inst if instance_tunings else teams_def
    tuning_s = time.perf_counter() - t0
    tuned = measure(teams)
    tuned["instance_tunings"] = instance_tunings
    progress(f"batched (tuned, {teams} teams, instance tunings {instance_tunings}): {tuned['batched_ms']} ms")
    gc.greedy_code_tune_reset()
    w_ee = sum(v[3] for v in expected.values())
    return {"instances": len(insts), "seed": 1507, "default": default, "tuned": tuned,
            "tuner_ms": {"defaults": {"teams": teams_def, "ms": round(ms_def, 3)},
                         "instance_tunings": {"teams": teams_inst, "ms": round(ms_inst, 3)}},
            "tuning_s": round(tuning_s, 2),
            "tuned_over_default": round(default["batched_ms"] / tuned["batched_ms"], 3),
            "batched_gchecks_per_s": round(w_ee / (min(default["batched_ms"], tuned["batched_ms"]) / 1e3) / 1e9, 3),
            "checked": "every result against the oracle digest"}


def load_expected_served():
    path = os.path.join(ROOT, "tests", "golden", "expected_served.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, m, digest = line.split()
            out[key] = (int(m), digest)
    return out


def bench_served(gc, njobs, arena_bytes, teams, load_frac):
    """The served workload: seeded Poisson stream of `njobs` jobs (n in
    [10, 26] skewed small, d in [3, 10], random ordering).  Three passes:
    one job in flight at a time (serial: one team spanning the GPU), all
    jobs submitted at once (burst: its makespan gives the capacity), then
    the Poisson stream offered at `load_frac` of that capacity.  Latency =
    arrival -> words in host memory.  Every result of every pass is compared
    with the oracle's digest for its (n, d, ordering)."""
    from paper_1507_05398_amd import workloads
    unit = workloads.served_jobs(seed=1507, count=njobs, rate=1.0)
    expected = load_expected_served()

    def check(i, words):
        _, n, d, o = unit[i]
        m, dig = expected[f"{n}_{d}_{o}"]
        if len(words) != m or hashlib.sha256(words.astype("<u4").tobytes()).hexdigest() != dig:
            raise SystemExit(f"SERVED MISMATCH job {i} {unit[i][1:]}: {len(words)} words vs {m}")

    t0 = time.perf_counter()
    with gc.Server(arena_bytes=arena_bytes, teams=1) as srv:
        for i, (_, n, d, o) in enumerate(unit):
            tk = srv.submit(n, d, o)
            while srv.poll(tk)[0] < gc.GC_JOB_DONE:
                pass
            check(i, srv.fetch(tk))
            srv.release(tk)
    serial_s = time.perf_counter() - t0
    progress(f"served: serial pass {serial_s:.2f} s")

    def serve(arrivals):
        lat = [0.0] * njobs
        waiting_polls = 0
        with gc.Server(arena_bytes=arena_bytes, teams=teams) as srv:
            nxt, inflight, done = 0, {}, 0
            t0 = time.perf_counter()
            while done < njobs:
                now = time.perf_counter() - t0
                while nxt < njobs and arrivals[nxt] <= now:
                    _, n, d, o = unit[nxt]
                    inflight[srv.submit(n, d, o)] = nxt
                    nxt += 1
                progressed = False
                for tk in list(inflight):
                    st, _ = srv.poll(tk)
                    if st == gc.GC_JOB_WAITING:
                        waiting_polls += 1
                    if st < gc.GC_JOB_DONE:
                        continue
                    i = inflight.pop(tk)
                    words = srv.fetch(tk)
                    lat[i] = time.perf_counter() - t0 - arrivals[i]
                    srv.release(tk)
                    check(i, words)
                    done += 1
                    progressed = True
                if not progressed and nxt < njobs:
                    wait = arrivals[nxt] - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(min(wait, 1e-3))
            span = time.perf_counter() - t0
        lat.sort()
        return span, lat, waiting_polls

    # Capacity: jobs over the makespan of the whole burst.
    burst_span, burst_lat, burst_waits = serve([0.0] * njobs)
    progress(f"served: burst pass {burst_span:.2f} s")
    capacity = njobs / burst_span
    rate = load_frac * capacity
    arrivals = [a / rate for a, _, _, _ in unit]
    span, lat, waits = serve(arrivals)
    q = lambda v, f: v[min(njobs - 1, int(f * njobs))]
    return {"jobs": njobs, "seed": 1507, "arena_bytes": arena_bytes, "teams": teams,
            "wide_jobs": ("2^n * capacity(n, d) >= 2^38: wide queue, one team of 8 - teams XCDs; "
                          "other jobs: teams teams of one XCD (and the wide team when idle)"
                          if teams in (2, 4) else "one queue, equal teams"),
            "serial_makespan_s": round(serial_s, 3), "serial_jobs_per_s": round(njobs / serial_s, 2),
            "burst_makespan_s": round(burst_span, 3), "capacity_jobs_per_s": round(capacity, 2),
            "burst_p99_ms": round(q(burst_lat, 0.99) * 1e3, 3),
            "burst_polls_waiting_for_memory": burst_waits,
            "offered_rate_jobs_per_s": round(rate, 2), "load_fraction": load_frac,
            "served_jobs_per_s": round(njobs / span, 2),
            "p50_ms": round(q(lat, 0.50) * 1e3, 3), "p99_ms": round(q(lat, 0.99) * 1e3, 3),
            "max_ms": round(lat[-1] * 1e3, 3),
            "polls_waiting_for_memory": waits,
            "checked": "every result of every pass against the oracle digest"}


def copy_calibration(torch, mib):
    """A plain device copy of `mib` MiB, five times (the FETCH_SIZE and
    WRITE_SIZE of this kernel scale the counters of the others)."""
    n = (mib << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 4, "launches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["screens", "sweep", "large"], default="screens")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-jobs", type=int, default=10000)
    ap.add_argument("--served-arena-mib", type=int, default=32)
    ap.add_argument("--served-teams", type=int, default=2)
    ap.add_argument("--served-load", type=float, default=0.7)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--probe", action="store_true",
                    help="only run the measurement probes (block-loop VALU rate, team barrier) and exit")
    ap.add_argument("--oracle-times", type=int, default=0, metavar="WORKERS",
                    help="only time the CPU oracle on every screen instance (one thread each, "
                         "WORKERS at a time) and exit")
    ap.add_argument("--host-api", action="store_true",
                    help="also time one step through the host-memory entry point")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.oracle_times:
        oracle_times(load_expected(), args.oracle_times)
        return

    import torch
    import paper_1507_05398_amd as gc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return
    if args.probe:
        gc.load()
        out = {"peak_gchecks_per_s": round(PEAK_GCHECKS, 1)}
        for k in (1, 2):
            try:
                v = gc.probe_block_loop(wgs_per_cu=k, iters=4096) / 1e9
            except gc.GreedyCodeError as e:  # two screen workgroups no longer fit a CU's LDS
                out[f"block_loop_{k}wg_per_cu"] = str(e)
                continue
            out[f"block_loop_{k}wg_per_cu_gchecks_per_s"] = round(v, 1)
            out[f"block_loop_{k}wg_per_cu_frac_of_peak"] = round(v / PEAK_GCHECKS, 4)
        v = gc.probe_matrix_loop(iters=2048) / 1e9
        out["matrix_loop_gchecks_per_s"] = round(v, 1)
        out["matrix_loop_frac_of_mfma_checks_ceiling"] = round(v / MFMA_CHECKS_PEAK_G, 4)
        out["matrix_loop_tops_at_n28"] = round(v * 56 / 1e3, 1)
        out["team_barrier_us"] = round(gc.probe_barrier(iters=20000), 3)
        print(json.dumps(out), flush=True)
        return
    gc.load()
    expected = load_expected()
    insts = {"screens": screens_24_28, "sweep": sweep_instances, "large": large_instances}[args.workload]()
    missing = [i for i in insts if f"{i[0]}_{i[1]}_{i[2]}" not in expected]
    if missing:
        raise SystemExit(f"no oracle reference for {missing}")

    wall, sweep = bench_sweep(gc, torch, insts, expected, args.steps, args.warmup)
    progress(f"{args.workload} done: {wall:.2f} s for {args.steps} steps")
    w_ee = sum(expected[f"{n}_{d}_{o}"][2] for n, d, o in insts)
    w_full = sum(expected[f"{n}_{d}_{o}"][3] for n, d, o in insts)
    name = {"screens": "screens n=24..28: lex/gray/grlex/grevlex x n24 x d{3,4,5,6,8} + lex/gray x n{26,28} x d3 "
                       "(24 instances)",
            "sweep": "sweep: lex/gray/grlex/grevlex x n{20,22,24} x d{3,4,5,6,8} + n23 d7 (64 instances)",
            "large": "large: lex/gray x n{26,28} x d3 (4 instances)"}[args.workload]
    line = {
        "metric": "Gdist-checks/s (algorithmic W_ee checks per second)",
        "value": round(args.steps * w_ee / wall / 1e9, 3),
        "unit": "Gchecks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",  # the distance checks are int8 products (int32 sums) on the matrix cores
        "data": "synthetic: the full space F_2^n in each ordering (no dataset)",
        "config": {"workload": name, "instances": len(insts), "w_ee_per_step": w_ee,
                   "w_full_per_step": w_full},
    }
    if args.host_api:
        # The same step through the host-memory entry point (device
        # allocation, build and copy of the words over PCIe).  Off by default:
        # its launches are not in the roofline's launch log.
        t0 = time.perf_counter()
        for n, d, o in insts:
            gc.greedy_code(n, d, o)
        host_wall = time.perf_counter() - t0
        line["host_api_gchecks_per_s"] = round(w_ee / host_wall / 1e9, 3)
    batched = None
    if not args.no_batched:
        batched = bench_batched(gc, torch, max(args.steps, 3), args.warmup)
        progress("batched done")
    line["roofline"] = {
        "bound": "mfma",
        "kernel": "greedy_code_kernel",
        "achieved": round(sweep.tops(), 3),
        "peak": INT8_PEAK_TOPS,
        "unit": "TOP/s (int8: 2n operations per check of n-bit words)",
        "frac": round(sweep.tops() / INT8_PEAK_TOPS, 5),
        "achieved_gchecks_per_s": round(sweep.gchecks(), 3),
        "checks_ceiling_mfma_gchecks_per_s": round(MFMA_CHECKS_PEAK_G, 1),
        "checks_ceiling_fold_gchecks_per_s": round(FOLD_CHECKS_PEAK_G, 1),
        "frac_of_checks_ceiling": round(sweep.gchecks() / min(MFMA_CHECKS_PEAK_G, FOLD_CHECKS_PEAK_G), 5),
        "valu_screen_peak_gchecks_per_s": round(PEAK_GCHECKS, 1),
        "frac_of_valu_screen_peak": round(sweep.gchecks() / PEAK_GCHECKS, 5),
        "traffic": measured_traffic(),
        "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, copy-calibrated)",
        "launches": sweep.launches,
        "avg_launch_ms": round(sweep.ms / max(sweep.launches, 1), 4),
        "covers": "every timed launch of the workload (HIP events around each launch on its stream)",
    }
    line["executed_checks_per_step"] = sweep.executed // max(args.steps, 1)
    line["executed_over_w_ee"] = round(sweep.executed / max(sweep.w_ee, 1), 4)
    line["per_instance_kernel_ms"] = sweep.median_ms()
    line["naive_equivalent_gchecks_per_s"] = round(args.steps * w_full / wall / 1e9, 3)
    if batched:
        line["batched"] = batched
    if not args.no_served:
        line["served"] = bench_served(gc, args.served_jobs, args.served_arena_mib << 20,
                                      args.served_teams, args.served_load)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(expected, sweep.median_ms())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

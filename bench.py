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
  * batched: the 256-instance workload (seed 1507) as one persistent launch
    against a loop of plain per-instance calls on the same buffers;
  * served: a seeded Poisson stream of 10,000 jobs through the job server
    (continuous batching), with p50/p99 latency, against the same jobs one at
    a time;
  * roofline of greedy_code_kernel, the single-code kernel: every launch of it
    in this run (the sweep and the plain per-instance loop), algorithmic
    checks (W_ee) per launch over the launch's duration (HIP events on the
    launch stream, recorded by the library);
  * cpu_baseline: the oracle on a bounded sample, one host thread.

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
# MI355X: 256 CUs x 64 int32 lanes per clock x 2.4 GHz, and one distance check
# costs 2.5 VALU lane-ops (v_xor_b32 + v_bcnt_u32_b32 + half a v_min3_u32).
VALU_LANE_OPS = 256 * 64 * 2.4e9
OPS_PER_CHECK = 2.5
PEAK_GCHECKS = VALU_LANE_OPS / OPS_PER_CHECK / 1e9


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
    path = os.path.join(ROOT, "profiles", "greedy_code_kernel_screens24_28_batched_traffic.md")
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


def cpu_baseline():
    """The CPU oracle (plain sequential scan, one thread) on a bounded sample
    of the sweep: n=20, d in {3, 5}, lex and Gray."""
    import oracle
    sample = [(20, 3, "lex"), (20, 3, "gray"), (20, 5, "lex"), (20, 5, "gray")]
    t0 = time.perf_counter()
    checks = 0
    for n, d, o in sample:
        _, w_ee, _ = oracle.greedy_scan(n, d, oracle.ORDERINGS[o])
        checks += w_ee
    dt = time.perf_counter() - t0
    return {"value": round(checks / dt / 1e9, 4), "unit": "Gchecks/s", "cores": 1, "kind": "oracle",
            "sample": "plain newest-first scan, n=20 d in {3,5} lex+gray (4 instances, "
                      f"{checks:.3e} checks in {dt:.1f} s)"}


class LaunchLog:
    """Kernel time and algorithmic checks of every timed greedy_code_kernel
    launch."""

    def __init__(self):
        self.ms, self.w_ee, self.executed, self.launches = 0.0, 0, 0, 0

    def add(self, stats, w_ee):
        self.ms += stats["kernel_ms"]
        self.w_ee += w_ee
        self.executed += stats["checks_near"] + stats["checks_deep"] + stats["checks_pairs"]
        self.launches += 1

    def gchecks(self):
        return self.w_ee / (self.ms / 1e3) / 1e9 if self.ms else 0.0


def bench_sweep(gc, torch, insts, expected, steps, warmup, log):
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
                own.add(st, expected[f"{n}_{d}_{o}"][2])
                log.add(st, expected[f"{n}_{d}_{o}"][2])

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


def bench_batched(gc, torch, steps, warmup, log):
    """The 256-instance batched workload (seed 1507): one persistent launch
    over every instance (teams by job count, largest jobs first) against a
    loop of plain per-instance calls on the same preallocated buffers."""
    from paper_1507_05398_amd import workloads
    insts = workloads.batched_instances()
    expected = load_expected_batch()
    plan = gc.BatchPlan(insts)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.run(stream=stream)
    torch.cuda.synchronize()
    walls, kms = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        kms.append(plan.run(stream=stream))
        walls.append(time.perf_counter() - t0)
    for i, t in enumerate(plan.results()):
        key, m, dig, _, _ = expected[i]
        if len(t) != m or digest_of(t) != dig:
            raise SystemExit(f"BATCH MISMATCH job {i} ({key})")

    # The same batch captured once into a HIP graph and replayed.
    gwalls = []
    with plan.graph() as g:
        g.launch(stream)
        g.wait()
        for _ in range(steps):
            t0 = time.perf_counter()
            g.launch(stream)
            g.wait()
            gwalls.append(time.perf_counter() - t0)
    for i, t in enumerate(plan.results()):
        key, m, dig, _, _ = expected[i]
        if len(t) != m or digest_of(t) != dig:
            raise SystemExit(f"GRAPH MISMATCH job {i} ({key})")

    def plain(record):
        for i, ((n, d, o), (w, c)) in enumerate(zip(insts, plan.bufs)):
            st = gc.greedy_code_device_ex(n, d, o, w, c, stream=stream)
            if record:
                log.add(st, expected[i][3])
    for _ in range(warmup):
        plain(False)
    torch.cuda.synchronize()
    pwalls = []
    for _ in range(steps):
        t0 = time.perf_counter()
        plain(True)
        torch.cuda.synchronize()
        pwalls.append(time.perf_counter() - t0)
    for i, (w, c) in enumerate(plan.bufs):
        key, m, dig, _, _ = expected[i]
        if int(c.item()) != m or digest_of(w[:m]) != dig:
            raise SystemExit(f"PLAIN MISMATCH job {i} ({key})")
    tb, tp = sorted(walls)[len(walls) // 2], sorted(pwalls)[len(pwalls) // 2]
    w_ee = sum(v[3] for v in expected.values())
    return {"instances": len(insts), "seed": 1507,
            "batched_codes_per_s": round(len(insts) / tb, 2), "batched_ms": round(tb * 1e3, 3),
            "batched_kernel_ms": round(sorted(kms)[len(kms) // 2], 3),
            "plain_codes_per_s": round(len(insts) / tp, 2), "plain_ms": round(tp * 1e3, 3),
            "speedup": round(tp / tb, 3),
            "graph_codes_per_s": round(len(insts) / sorted(gwalls)[len(gwalls) // 2], 2),
            "batched_gchecks_per_s": round(w_ee / tb / 1e9, 3)}


def bench_served(gc, njobs, arena_bytes, teams, load_frac):
    """The served workload: seeded Poisson stream of `njobs` jobs (n in
    [10, 26] skewed small, d in [3, 10], random ordering).  Three passes:
    one job in flight at a time (serial: one team spanning the GPU), all
    jobs submitted at once (capacity), then the Poisson stream at
    `load_frac` of that capacity.  Latency = arrival -> words in host memory.
    Every result of the concurrent passes must equal the serial one."""
    from paper_1507_05398_amd import workloads
    unit = workloads.served_jobs(seed=1507, count=njobs, rate=1.0)
    ref = []

    def sha(words):
        return hashlib.sha256(words.astype("<u4").tobytes()).hexdigest()

    t0 = time.perf_counter()
    with gc.Server(arena_bytes=arena_bytes, teams=1) as srv:
        for _, n, d, o in unit:
            tk = srv.submit(n, d, o)
            while srv.poll(tk)[0] < gc.GC_JOB_DONE:
                pass
            ref.append(sha(srv.fetch(tk)))
            srv.release(tk)
    serial_s = time.perf_counter() - t0
    progress(f"served: serial pass {serial_s:.2f} s")

    def serve(arrivals):
        lat = [0.0] * njobs
        finish = []
        admitted_wait = 0
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
                        admitted_wait += 1
                    if st < gc.GC_JOB_DONE:
                        continue
                    i = inflight.pop(tk)
                    words = srv.fetch(tk)
                    t_fin = time.perf_counter() - t0
                    lat[i] = t_fin - arrivals[i]
                    finish.append(t_fin)
                    srv.release(tk)
                    if sha(words) != ref[i]:
                        raise SystemExit(f"SERVED MISMATCH job {i} {unit[i][1:]}")
                    done += 1
                    progressed = True
                if not progressed and nxt < njobs:
                    wait = arrivals[nxt] - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(min(wait, 1e-3))
            span = time.perf_counter() - t0
        lat.sort()
        return span, lat, admitted_wait, finish

    # Capacity: completions per second over the first 90% of a burst (the
    # last few percent are the largest codes finishing on their teams).
    burst_span, _, _, finish = serve([0.0] * njobs)
    t90 = finish[int(0.9 * njobs) - 1]
    progress(f"served: burst pass {burst_span:.2f} s (90% done at {t90:.2f} s)")
    capacity = 0.9 * njobs / t90
    rate = load_frac * capacity
    arrivals = [a / rate for a, _, _, _ in unit]
    span, lat, waits, _ = serve(arrivals)
    q = lambda f: lat[min(njobs - 1, int(f * njobs))]
    return {"jobs": njobs, "seed": 1507, "arena_bytes": arena_bytes, "teams": teams,
            "serial_jobs_per_s": round(njobs / serial_s, 2),
            "capacity_jobs_per_s": round(capacity, 2), "burst_makespan_s": round(burst_span, 3),
            "offered_rate_jobs_per_s": round(rate, 2), "load_fraction": load_frac,
            "served_jobs_per_s": round(njobs / span, 2),
            "p50_ms": round(q(0.50) * 1e3, 3), "p99_ms": round(q(0.99) * 1e3, 3),
            "max_ms": round(lat[-1] * 1e3, 3),
            "polls_waiting_for_memory": waits}


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
    ap.add_argument("--served-arena-mib", type=int, default=64)
    ap.add_argument("--served-teams", type=int, default=8)
    ap.add_argument("--served-load", type=float, default=0.7)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--host-api", action="store_true",
                    help="also time one step through the host-memory entry point")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1507_05398_amd as gc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return
    gc.load()
    expected = load_expected()
    insts = {"screens": screens_24_28, "sweep": sweep_instances, "large": large_instances}[args.workload]()
    missing = [i for i in insts if f"{i[0]}_{i[1]}_{i[2]}" not in expected]
    if missing:
        raise SystemExit(f"no oracle reference for {missing}")

    log = LaunchLog()
    wall, sweep = bench_sweep(gc, torch, insts, expected, args.steps, args.warmup, log)
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
        "dtype": "u32",
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
        batched = bench_batched(gc, torch, max(args.steps, 3), args.warmup, log)
        progress("batched done")
    line["roofline"] = {
        "bound": "alu",
        "kernel": "greedy_code_kernel",
        "achieved": round(log.gchecks(), 3),
        "peak": round(PEAK_GCHECKS, 1),
        "unit": "Gchecks/s",
        "frac": round(log.gchecks() / PEAK_GCHECKS, 5),
        "traffic": measured_traffic(),
        "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, copy-calibrated)",
        "launches": log.launches,
        "avg_launch_ms": round(log.ms / max(log.launches, 1), 4),
        "covers": "timed launches of the workload" + (" and of the plain batched loop" if batched else ""),
        "workload_only": {"achieved": round(sweep.gchecks(), 3),
                          "frac": round(sweep.gchecks() / PEAK_GCHECKS, 5),
                          "avg_launch_ms": round(sweep.ms / max(sweep.launches, 1), 4)},
    }
    line["executed_checks_per_step"] = sweep.executed // max(args.steps, 1)
    line["naive_equivalent_gchecks_per_s"] = round(args.steps * w_full / wall / 1e9, 3)
    if batched:
        line["batched"] = batched
    if not args.no_served:
        line["served"] = bench_served(gc, args.served_jobs, args.served_arena_mib << 20,
                                      args.served_teams, args.served_load)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: greedy code construction on one MI355X.

A step is one pass of the whole construction over the workload: every
instance (n, d, ordering) is built from scratch on the GPU (all 2^n candidate
positions screened, resolved and committed).  The default workload is the
sweep of four orderings x n in {20, 22, 24} x d in {3, 4, 5, 6, 8}, plus n=23
with d=7 (64 instances).  ``--workload large`` runs the n=26/28 d=3 screens
(lex and Gray) instead.

The headline value is algorithmic distance checks per second: the sum over
instances of W_ee (checks done by a sequential newest-first scan with early
exit, counted by the CPU oracle and stored in tests/golden/expected_codes.txt)
divided by the wall time of the step.  Output: one JSON line.
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


def load_expected():
    path = os.path.join(ROOT, "tests", "golden", "expected_codes.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, m, digest, w_ee, w_full = line.split()
            out[key] = (int(m), digest, int(w_ee), int(w_full))
    return out


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["sweep", "large"], default="sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1507_05398_amd as gc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    expected = load_expected()
    insts = sweep_instances() if args.workload == "sweep" else large_instances()
    missing = [i for i in insts if f"{i[0]}_{i[1]}_{i[2]}" not in expected]
    if missing:
        raise SystemExit(f"no oracle reference for {missing}")
    bufs = []
    for n, d, o in insts:
        cap = gc.greedy_code_capacity(n, d)
        bufs.append((torch.empty(cap, dtype=torch.int32, device="cuda"),
                     torch.zeros(1, dtype=torch.int64, device="cuda")))
    stream = torch.cuda.current_stream()

    def one_step():
        stats = []
        for (n, d, o), (w, c) in zip(insts, bufs):
            stats.append(gc.greedy_code_device_ex(n, d, o, w, c, stream=stream))
        return stats

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_ms = 0.0
    executed = 0
    for _ in range(args.steps):
        for st in one_step():
            kernel_ms += st["kernel_ms"]
            executed += st["checks_near"] + st["checks_deep"] + st["checks_pairs"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # Bit-exact check of the last step's output (outside the timed region).
    for (n, d, o), (w, c) in zip(insts, bufs):
        m, dig, _, _ = expected[f"{n}_{d}_{o}"]
        got = w[: int(c.item())].cpu().numpy().astype("<u4")
        if len(got) != m or hashlib.sha256(got.tobytes()).hexdigest() != dig:
            raise SystemExit(f"MISMATCH n={n} d={d} {o}: {len(got)} words vs {m}")

    w_ee = sum(expected[f"{n}_{d}_{o}"][2] for n, d, o in insts)
    w_full = sum(expected[f"{n}_{d}_{o}"][3] for n, d, o in insts)
    value = args.steps * w_ee / wall / 1e9
    launches = args.steps * len(insts)
    achieved = args.steps * w_ee / (kernel_ms / 1e3) / 1e9
    name = ("sweep: lex/gray/grlex/grevlex x n{20,22,24} x d{3,4,5,6,8} + n23 d7 (64 instances)"
            if args.workload == "sweep" else "large: lex/gray x n{26,28} x d3 (4 instances)")
    line = {
        "metric": "Gdist-checks/s (algorithmic W_ee checks per second)",
        "value": round(value, 3),
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
        "roofline": {
            "bound": "alu",
            "kernel": "greedy_persistent",
            "achieved": round(achieved, 3),
            "peak": round(PEAK_GCHECKS, 1),
            "unit": "Gchecks/s",
            "frac": round(achieved / PEAK_GCHECKS, 5),
            "traffic": None,
            "launches": launches,
            "avg_launch_ms": round(kernel_ms / launches, 4),
        },
        "executed_checks_per_step": executed // args.steps,
        "naive_equivalent_gchecks_per_s": round(args.steps * w_full / wall / 1e9, 3),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Host-side checks of bench.py (no GPU): the one-GPU rule, the roofline
constants against MI355X's published figures, the workload definitions, the
bounded CPU-baseline sample and the rule that HBM traffic is reported only for
the kernel sources the counters were taken on."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_constants():
    # 256 CUs x 4 SIMDs x 16 int32 lanes at 2.4 GHz.
    assert bench.VALU_LANE_OPS == pytest.approx(256 * 4 * 16 * 2.4e9)
    # Vector-ALU screen: 2.5 lane-ops per check.
    assert bench.PEAK_GCHECKS == pytest.approx(15728.64)
    # Dense int8 matrix peak; a 32-byte row costs 64 operations per check, and
    # the max-fold half a lane-op per check.
    assert bench.INT8_PEAK_TOPS == 5000.0
    assert bench.MFMA_CHECKS_PEAK_G == pytest.approx(78125.0)
    assert bench.FOLD_CHECKS_PEAK_G == pytest.approx(78643.2)


def test_screens_workload():
    insts = bench.screens_24_28()
    assert len(insts) == 24 and len(set(insts)) == 24
    n24 = [i for i in insts if i[0] == 24]
    assert sorted({d for _, d, _ in n24}) == [3, 4, 5, 6, 8]
    assert sorted({o for _, _, o in n24}) == sorted(bench.ORDS)
    assert sorted(i for i in insts if i[0] > 24) == [(26, 3, "gray"), (26, 3, "lex"), (28, 3, "gray"),
                                                     (28, 3, "lex")]
    expected = bench.load_expected()
    for n, d, o in insts:
        assert f"{n}_{d}_{o}" in expected


def test_sweep_workload():
    insts = bench.sweep_instances()
    assert len(insts) == 64 and len(set(insts)) == 64
    assert sum(1 for i in insts if i[:2] == (23, 7)) == 4
    expected = bench.load_expected()
    for n, d, o in insts:
        assert f"{n}_{d}_{o}" in expected


def test_cpu_sample_is_bounded():
    # The oracle's plain scan runs at 0.3-0.5 G checks/s on one host core:
    # the sample must stay in the tens of seconds.
    expected = bench.load_expected()
    w_ee = sum(expected[f"{n}_{d}_{o}"][2] for n, d, o in bench.CPU_SAMPLE)
    assert 1e9 < w_ee < 1e10
    assert set(bench.CPU_SAMPLE) <= set(bench.screens_24_28())


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    for rel in ("profiles/greedy_code_kernel_screens24_28_traffic.md",
                "paper_1507_05398_amd/csrc/greedy_code.hip", "paper_1507_05398_amd/csrc/gc_internal.h"):
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), tmp_path / rel)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    summary = (tmp_path / "profiles/greedy_code_kernel_screens24_28_traffic.md").read_text()
    stated = int(summary.split("traffic_bytes_per_launch:")[1].split()[0])
    # The sources as committed: the figure comes back only if they hash to the
    # summary's value (otherwise the counters are stale and it is withheld).
    got = bench.measured_traffic()
    assert got is None or got == stated
    # Any change to the kernel sources withholds it.
    src = tmp_path / "paper_1507_05398_amd/csrc/greedy_code.hip"
    src.write_text(src.read_text() + "\n")
    assert bench.measured_traffic() is None
    # No summary: nothing to report.
    os.remove(tmp_path / "profiles/greedy_code_kernel_screens24_28_traffic.md")
    assert bench.measured_traffic() is None

"""GPU tests of the autotuners: every tuning they pick builds the oracle's
code, and a remembered tuning is used by later builds that pass none."""
import sys

import numpy as np
import pytest

import oracle
import paper_1507_05398_amd as gc

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    gc.load()
    yield torch
    gc.greedy_code_tune_reset()


@pytest.mark.parametrize("n,d,o", [(16, 3, "lex"), (16, 4, "grlex"), (15, 5, "gray"), (14, 6, "grevlex")])
def test_tune_then_build_matches_oracle(n, d, o):
    log(f"[tune] n={n} d={d} ord={o}")
    best = gc.greedy_code_tune(n, d, o)
    assert best["ms"] > 0
    assert best["resolve_mode"] in (0, 1, 2)
    assert best["deep_tile"] in (0, 256, 512)
    ref = oracle.greedy_ball(n, d, oracle.ORDERINGS[o])[0]
    words, _ = gc.device_code(n, d, o)           # no tuning passed: the remembered one
    np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32), ref)
    np.testing.assert_array_equal(gc.greedy_code(n, d, o), ref)
    gc.greedy_code_tune_reset()
    words, _ = gc.device_code(n, d, o)
    np.testing.assert_array_equal(words.cpu().numpy().view(np.uint32), ref)


def test_tune_degenerate_is_trivial():
    assert gc.greedy_code_tune(10, 1, "lex")["ms"] == 0.0
    assert gc.greedy_code_tune(10, 11, "gray")["near_depth"] == 0


def test_batch_team_tuner():
    insts = [(12 + (i % 6), 3 + (i % 4), ["lex", "gray", "grlex", "grevlex"][i % 4]) for i in range(24)]
    log(f"[tune] batch of {len(insts)}")
    plan = gc.BatchPlan(insts)
    teams, ms = plan.tune()
    assert teams in (1, 2, 4, 8) and ms > 0
    for (n, d, o), t in zip(insts, plan.results()):
        ref = oracle.greedy_ball(n, d, oracle.ORDERINGS[o])[0]
        np.testing.assert_array_equal(t.cpu().numpy().view(np.uint32), ref)
    plan.run(teams=teams)
    for (n, d, o), t in zip(insts, plan.results()):
        ref = oracle.greedy_ball(n, d, oracle.ORDERINGS[o])[0]
        np.testing.assert_array_equal(t.cpu().numpy().view(np.uint32), ref)

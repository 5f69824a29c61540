"""CPU checks of bench.py's command line and launch arithmetic (no device).

The driver runs `python bench.py --gpus 1 --steps 20 --warmup 5`; any step
counts must be accepted, odd ones included, and the launch bookkeeping that
the roofline is computed from must count what tk_step issues."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_driver_arguments_parse():
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup, a.workload, a.precision) == (1, 20, 5, "batched", "fp64")
    for argv in (["--steps", "7", "--warmup", "3", "--graph-steps", "33"], ["--steps", "1", "--warmup", "0"]):
        bench.parse_args(argv)


@pytest.mark.parametrize("argv", [["--steps", "0"], ["--warmup", "-1"], ["--graph-steps", "-2"]])
def test_bad_arguments_rejected(argv):
    with pytest.raises(SystemExit):
        bench.parse_args(argv)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "20"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _count(steps, G, two_step):
    """Reference count by walking tk_step's loop: replays of G, then the rest;
    each block pairs steps for the two-step kernel and ends an odd count with
    one one-step launch."""
    n2 = n1 = replays = 0
    left = steps
    blocks = []
    if G > 0:
        while left >= G:
            blocks.append(G)
            left -= G
            replays += 1
    if left:
        blocks.append(left)
    for b in blocks:
        if two_step:
            n2 += b // 2
            n1 += b % 2
        else:
            n1 += b
    return replays, n2, n1, len(blocks)


@pytest.mark.parametrize("steps", [1, 2, 5, 19, 20, 21, 100, 101, 250])
@pytest.mark.parametrize("G", [0, 3, 20, 100])
@pytest.mark.parametrize("two_step", [True, False])
def test_launch_plan_matches_the_step_loop(steps, G, two_step):
    p = bench.launch_plan(steps, G, two_step)
    replays, n2, n1, bumps = _count(steps, G, two_step)
    assert (p["graph_replays"], p["two_step_launches"], p["one_step_launches"], p["bumps"]) == (replays, n2, n1,
                                                                                                 bumps)
    # every step is accounted for
    assert 2 * p["two_step_launches"] + p["one_step_launches"] == steps


def test_driver_run_times_whole_two_step_launches_in_graphs():
    # --steps 20 --warmup 5 with the default --graph-steps 100: the 20 timed
    # steps form one graph of 20 steps, i.e. ten two-step launches
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    K_main = a.steps - a.steps % 2
    G = bench.bench_graph_steps(K_main, a.graph_steps, True)
    assert G == 20
    p = bench.launch_plan(K_main, G, True)
    assert p == {"graph_replays": 1, "two_step_launches": 10, "one_step_launches": 0, "bumps": 1}
    # an odd count: the whole launches first, the odd step in a second call
    K = 21
    K_main = K - K % 2
    G = bench.bench_graph_steps(K_main, 100, True)
    assert (K_main, G) == (20, 20)
    assert bench.launch_plan(K - K_main, G, True) == {"graph_replays": 0, "two_step_launches": 0,
                                                      "one_step_launches": 1, "bumps": 1}
    # graph length never odd for the two-step kernel, never above the timed count
    for K in range(1, 60):
        for req in (0, 1, 7, 10, 100):
            G = bench.bench_graph_steps(K, req, True)
            assert G % 2 == 0 and G <= K and G <= req


def test_two_step_flops_per_update():
    # the FP64 two-step launches do not form Sigma-hat^2 (one multiply-add) and
    # 1/Sigma-hat (estimate, x/2 and two Newton steps of a multiply and two
    # multiply-adds) again at level 2's two stage points: 28 per level-2
    # update, half that per update over both levels
    per_point = 2 + 1 + 1 + 2 * (1 + 2 + 2)
    assert bench.flops_per_update("fp64", False) == 194
    assert bench.flops_per_update("fp64", True) == 194 - 2 * per_point // 2
    # FP32C: one Newton step
    per_point32 = 2 + 1 + 1 + (1 + 2 + 2)
    assert bench.flops_per_update("fp32c", False) == 312
    assert bench.flops_per_update("fp32c", True) == 312 - 2 * per_point32 // 2


def test_kernel_hash_ignores_comments_only():
    code = "int a; // one\n/* two\n three */ int b;\n\n  // four\nint c; /* five */\n"
    # a block comment stands as one blank, as the compiler reads it
    assert bench._code_only(code) == bench._code_only("int a;\n  int b;\nint c;\n")
    assert bench._code_only(code) != bench._code_only("int a;\n  int b;\nint d;\n")
    assert len(bench.kernel_hash()) == 16

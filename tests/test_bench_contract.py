"""The benchmark script's command-line contract on the host: more than one
GPU is refused with a message (the measurement covers one GPU) before any
GPU work, and the metric's static parts are well formed."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_flops_count_matches_hand_count():
    # the roofline's flop count per RHS (one trajectory) at depth 0: one ADO,
    # no neighbours: 8 d^3 (H commutator) + 8 d^2 sum d_s (V_s products)
    # + 6 d^2 (damping and stage update)
    sys.path.insert(0, ROOT)
    import bench
    import workloads as w
    import paper_2601_20550_amd as P
    params, _ = w.cfg3(depth=0)
    m = P.heom_model_build_host(params)
    d = 80
    assert bench.algorithmic_flops_per_rhs(m) == 8 * d ** 3 + 8 * d * d * (4 + 4 + 5) + 6 * d * d


def test_optional_legs_keep_to_the_wall_budget():
    # an optional leg runs only while its usual duration fits what is left of
    # the budget; otherwise the line records why it was skipped
    sys.path.insert(0, ROOT)
    import bench
    assert bench.leg_skip_reason(400.0, 55.0, 570.0) is None
    assert bench.leg_skip_reason(515.0, 55.0, 570.0) is None
    why = bench.leg_skip_reason(530.0, 55.0, 570.0)
    assert why is not None and "530 s elapsed" in why and "budget 570 s" in why

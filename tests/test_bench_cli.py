"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message, and the workload table names only known graphs."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_name_known_graphs():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1911_12877_amd import synth
    for name, wl in bench.WORKLOADS.items():
        # the census workload names the 64-graph motif batch of census_graph_params
        assert wl["graph"] in synth.CONFIGS or wl["graph"] == "census64", name
        assert wl["patterns"], name
    assert synth.census_graph_params(63)["n"] > 0


def test_cpu_baseline_sharded_oracle_agrees():
    """The benchmark's CPU leg runs the oracle once on one core and again
    sharded round-robin over worker processes; both see the same sample."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1911_12877_amd import synth
    from oracle import patterns as P
    e = synth.config_graph("er2000")
    order = P.pick_schedule(P.named("triangle"), True)[0]
    bound = list(P.reduced_bounds(P.named("triangle"), order))
    v1, dt1, vn, dtn, desc = bench.cpu_baseline(e, ["triangle"], True, [order], [bound],
                                                target_s=0.05, workers=2)
    assert v1 > 0 and vn > 0 and dt1 > 0 and dtn > 0
    assert "roots" in desc

"""bench.py on the host: it parses, refuses more than one GPU with a JSON
message, and its algorithmic counts follow their stated formulas."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_flop_and_byte_models():
    import bench
    # 3-D Euler N=4, 5 sweeps from the constant guess: one slice, 4 full sweeps, outputs
    n, m, d = 5, 5, 3
    nst, nd = n ** 4, n ** 3
    sweep = 31 * nst + 4 * 2 * n * m * nst + 2 * m * nst
    slice_rhs = 31 * nd + 3 * 2 * n * m * nd
    outputs = 31 * nst + 2 * m * d * nst + d * 2 * n * m * nd + 2 * m * nd + 2 * d * 2 * n * m * nd
    assert bench.predictor_flops(3, 4, 5, 5) == slice_rhs + 2 * m * nst + 4 * sweep + outputs
    assert bench.predictor_flops(3, 4, 5, 3, guess=2) == 2 * slice_rhs + 2 * m * nd + 5 * m * nst + 3 * sweep + outputs
    b = bench.step_bytes(3, 4, 5, 4)
    assert b["predictor"] == 2 * 8 * m * nd + 6 * 4 * m * nd
    assert b["update"] == 2 * 8 * m * nd + 6 * 4 * m * nd // n

    class P:
        N, picard, guess = 4, 0, 2
    assert bench.sweeps_of(P) == 3

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


def test_work_model_flops_per_dof():
    """The algorithmic work model reproduces the per-DOF step figures of the
    work model it states (Euler N = 2..6 with N+1 sweeps: 2.25k, 4.15k,
    7.08k, 11.3k, 17.0k flop per DOF; elasticity N = 5: about 19.5k)."""
    import bench
    want = {2: 2.25e3, 3: 4.15e3, 4: 7.08e3, 5: 11.3e3, 6: 17.0e3}
    for N, f in want.items():
        s = bench.work_model_flops(3, N, 5, N + 1)
        per_dof = (s["predictor"] + s["corrector"]) / (N + 1) ** 3
        assert abs(per_dof - f) <= 0.01 * f, (N, per_dof)
    s = bench.work_model_flops(3, 5, 9, 6, elastic=True)
    assert abs((s["predictor"] + s["corrector"]) / 216 - 19.5e3) <= 0.02 * 19.5e3


def test_split_roofline_time():
    """Mixed path: sweeps 1..P-1 at the FP32 matrix peak, sweep P and the
    outputs at the FP64 peak; the FP64 path prices everything at FP64."""
    import bench

    class P:
        dim, N, m, E, pde, picard, guess = 3, 4, 5, 262144, "euler", 0, 0
    lo, hi = bench.precision_split([P], "fp32")
    s = bench.work_model_flops(3, 4, 5, 5)
    assert lo == P.E * 4 * s["sweep"] and hi == P.E * (s["sweep"] + s["outputs"])
    t = bench.roof_time_ms(lo, hi, "fp32")
    assert abs(t - (lo / 157.3e12 + hi / 78.6e12) * 1e3) < 1e-12
    lo64, hi64 = bench.precision_split([P], "fp64")
    assert lo64 == 0 and hi64 == P.E * s["predictor"]

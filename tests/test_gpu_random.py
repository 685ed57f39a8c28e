"""Seeded random configurations against the oracle.

Each case draws a context of one to four problems (dimension, PDE, degree
within the classes that fit LDS, mesh extents 1..6 per axis, box, precision,
initial guess, averaged-trace faces, Picard count), runs three steps through
ader_step on the GPU and three oracle steps per problem.  Problems of one
context that share a kernel class are batched into the same launches.

Error measure: elastic velocities are first scaled to stress units (times
rho c_p of the element); then, per variable, the discrete L2 norm of the
difference divided by max(its own norm, 1e-3 x the largest variable norm).
The floor matters for variables that vanish by symmetry (a single element
across an axis with a centred pulse): both sides then hold rounding noise
only.  Bounds: FP64 1e-12; FP32 sweeps 1e-6 for both systems (the elastic
velocities, small three steps after rest, are compared in stress units).
"""
import sys

import numpy as np
import pytest

from paper_1808_03788_amd import inputs as I

pytestmark = pytest.mark.gpu

CASES = 24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_03788_amd import ader
    ader.lib()
    return ader


def draw_problem(rng):
    """One random problem and its initial data (supported classes only)."""
    kind = rng.choice(["euler3", "euler2", "elastic"], p=[0.5, 0.25, 0.25])
    prec = str(rng.choice(["fp64", "fp32"]))
    if kind == "elastic":
        N = int(rng.integers(0, 5))            # N = 5 runs the slow HBM variant in FP64
        nel = tuple(int(x) for x in rng.integers(1, 4, size=3))
        p = I.Problem(dim=3, N=N, nel=nel, lo=(0.0, 0.0, 0.0), hi=tuple(rng.uniform(0.5, 2.0, size=3)),
                      pde="elastic", prec=prec)
        p.material = I.homogeneous_material(p, rho=float(rng.uniform(2000, 3000)),
                                            cp=float(rng.uniform(3000, 6000)))
        init = I.stress_pulse(p, width=0.4, centre=tuple(0.5 * h for h in p.hi))
    elif kind == "euler2":
        N = int(rng.integers(0, 8))
        nel = (int(rng.integers(1, 7)), int(rng.integers(1, 7)))
        p = I.Problem(dim=2, N=N, nel=nel, lo=(0.0, 0.0), hi=(10.0, 10.0), prec=prec)
        init = I.isentropic_vortex(p)
    else:
        N = int(rng.integers(0, 6))
        nel = tuple(int(x) for x in rng.integers(1, 6, size=3))
        p = I.Problem(dim=3, N=N, nel=nel, lo=(0.0, 0.0, 0.0), hi=tuple(rng.uniform(0.5, 2.0, size=3)),
                      prec=prec)
        init = I.density_wave(p, amp=float(rng.uniform(0.05, 0.2)), noise=float(rng.uniform(0, 1e-3)),
                              seed=int(rng.integers(0, 1000)))
    p.guess = int(rng.integers(0, 4)) if p.N > 0 else 0
    p.face_avg = int(rng.integers(0, 2))
    p.picard = int(rng.integers(0, p.N + 2)) if rng.uniform() < 0.3 else 0
    return p, init


def fp64_twin(p):
    q = I.Problem(dim=p.dim, N=p.N, nel=p.nel, lo=p.lo, hi=p.hi, pde=p.pde, gamma=p.gamma, picard=p.picard,
                  cfl=p.cfl, prec="fp64", guess=p.guess, face_avg=p.face_avg)
    q.material = p.material
    return q


def scaled_error(p, a, b):
    """max over variables of ||a_v - b_v|| / max(||b_v||, 1e-3 max_w ||b_w||)
    (GL-weighted discrete L2), elastic velocities in stress units."""
    a, b = np.array(a, dtype=np.float64), np.array(b, dtype=np.float64)
    if p.pde == "elastic":
        rho, lam, mu = p.material[:, 0], p.material[:, 1], p.material[:, 2]
        z = (rho * np.sqrt((lam + 2.0 * mu) / rho))[:, None, None]
        a[:, :3, :] *= z
        b[:, :3, :] *= z
    W = I.quad_weights(p)
    dn = np.sqrt(np.einsum("evk,k->v", (a - b) ** 2, W))
    bn = np.sqrt(np.einsum("evk,k->v", b ** 2, W))
    return float(np.max(dn / np.maximum(bn, 1e-3 * bn.max())))


@pytest.mark.parametrize("case", range(CASES))
def test_random_context_vs_oracle(A, orc, case):
    import torch
    rng = np.random.default_rng(1000 + case)
    drawn = [draw_problem(rng) for _ in range(int(rng.integers(1, 5)))]
    probs = [p for p, _ in drawn]
    desc = ", ".join(f"{p.pde}{p.dim}d N={p.N} {p.nel[:p.dim]} {p.prec} g{p.guess} a{p.face_avg} P{p.picard}"
                     for p in probs)
    say(f"[random {case}] {desc}")
    ctx = A.Context(probs)
    try:
        u = ctx.upload([u0 for _, u0 in drawn])
        for _ in range(3):
            ctx.step(u, [1e9] * len(probs))
        torch.cuda.synchronize()
        outs = ctx.download(u)
    finally:
        ctx.close()
    for (p, u0), ug in zip(drawn, outs):
        uo, t, hist = u0, 0.0, None
        for _ in range(3):
            uo, t, _, hist = orc.step_hist(fp64_twin(p), uo, t, 1e9, hist)
        err = scaled_error(p, ug, uo)
        tol = 1e-12 if p.prec == "fp64" else 1e-6
        say(f"  {p.pde}{p.dim}d N={p.N} {p.prec}: error={err:.3e}")
        assert err <= tol, (case, p, err)

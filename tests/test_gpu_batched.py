"""Batched launches and captured-graph replays on the GPU.

Problems of one kernel class (dimension, degree, PDE, precision) share every
launch of a step; the arithmetic of an element does not depend on which
other problems share its launch, so a batched context must reproduce
single-problem contexts bit for bit.  ader_run replays a captured graph of
ader_step launches and must reproduce the same number of ader_step calls bit
for bit.  The FP64 results are also held to the oracle (1e-12 relative L2),
and a mixed-degree FP32 batch shaped like the 256-problem workload (smaller
meshes) to 1e-6.
"""
import sys

import numpy as np
import pytest

from paper_1808_03788_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def batch_set():
    box = dict(lo=(0, 0, 0), hi=(1, 1, 1))
    probs = [
        I.Problem(dim=3, N=3, nel=(3, 3, 3), **box),
        I.Problem(dim=3, N=2, nel=(4, 2, 3), **box),
        I.Problem(dim=3, N=3, nel=(5, 2, 3), **box),
        I.vortex_problem(nel=6, N=3),
        I.Problem(dim=3, N=2, nel=(2, 5, 2), **box),
        I.Problem(dim=3, N=3, nel=(2, 2, 7), **box),
    ]
    inits = [I.isentropic_vortex(p) if p.dim == 2 else I.density_wave(p) for p in probs]
    return probs, inits


def run_steps(A, probs, inits, steps, t_end):
    import torch
    ctx = A.Context(probs)
    u = ctx.upload(inits)
    for _ in range(steps):
        ctx.step(u, t_end)
    torch.cuda.synchronize()
    out, t = ctx.download(u), ctx.time()
    ctx.close()
    return out, t


def test_batched_classes_match_single_problem_contexts(A, orc):
    probs, inits = batch_set()
    say(f"[batched] {len(probs)} problems, 3 steps")
    together, _ = run_steps(A, probs, inits, 3, [1e9] * len(probs))
    for i, (p, u0) in enumerate(zip(probs, inits)):
        alone, _ = run_steps(A, [p], [u0], 3, [1e9])
        assert np.array_equal(together[i], alone[0]), f"problem {i} differs between batched and single"
    for i in (0, 3):
        u, t = inits[i], 0.0
        for _ in range(3):
            u, t, _ = orc.step(probs[i], u, t, 1e9)
        err = I.rel_l2(probs[i], together[i], u)
        ei = I.rel_linf(together[i], u)
        say(f"  problem {i} vs oracle rel_l2={err:.3e} rel_linf={ei:.3e}")
        assert err <= 1e-12 and ei <= 1e-11


def test_graph_replay_matches_steps(A):
    import torch
    probs, inits = batch_set()
    t_end = [0.01, 1e9, 1e9, 0.05, 1e9, 1e9]  # problem 0 reaches t_end inside the replays
    say("[graph] 2 replays of 4 steps vs 8 steps")
    ref, t_ref = run_steps(A, probs, inits, 8, t_end)
    ctx = A.Context(probs)
    u = ctx.upload(inits)
    ctx.run(u, t_end, 4)
    ctx.run(u, t_end, 4)
    torch.cuda.synchronize()
    out, t = ctx.download(u), ctx.time()
    with pytest.raises(A.AderError):
        A.ader_run(ctx.ctx, u, t_end, 0)
    ctx.close()
    assert np.array_equal(t, t_ref), (t, t_ref)
    assert t[0] == 0.01
    for i in range(len(probs)):
        assert np.array_equal(out[i], ref[i]), f"problem {i}: graph replay differs from ader_step"


def test_graph_replay_after_t_end_change(A):
    import torch
    probs, inits = batch_set()
    say("[graph] t_end change between replays")
    ref, t_ref = run_steps(A, probs, inits, 2, [1e9] * len(probs))
    ctx = A.Context(probs)
    u = ctx.upload(inits)
    ctx.run(u, [1e9] * len(probs), 1)
    ctx.run(u, [2e9] * len(probs), 1)  # same result: t_end far away
    torch.cuda.synchronize()
    out, t = ctx.download(u), ctx.time()
    ctx.close()
    assert np.array_equal(t, t_ref)
    for i in range(len(probs)):
        assert np.array_equal(out[i], ref[i])


def test_mixed_degree_fp32_batch_vs_oracle(A, orc):
    import torch
    items = I.batched_problems(count=10, seed=0, edge=(2, 4), degrees=(2, 6), prec="fp32")
    probs = [p for p, _ in items]
    inits = [I.density_wave(p, **kw) for p, kw in items]
    say(f"[fp32 batch] degrees {[p.N for p in probs]}")
    ctx = A.Context(probs)
    u = ctx.upload(inits)
    ctx.run(u, [1e9] * len(probs), 3)
    torch.cuda.synchronize()
    outs = ctx.download(u)
    ctx.close()
    for p, u0, ug in zip(probs, inits, outs):
        uo, t = u0, 0.0
        for _ in range(3):
            uo, t, _ = orc.step(p, uo, t, 1e9)
        err = I.rel_l2(p, ug, uo)
        ei = I.rel_linf(ug, uo)
        say(f"  N={p.N} E={p.E} rel_l2={err:.3e} rel_linf={ei:.3e}")
        assert err <= 1e-6 and ei <= 1e-5

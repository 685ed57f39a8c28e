"""The time step from the wave-speed maxima the update takes of the state it
writes, against the time-step kernel's pass over that state.

ader_step / ader_run take a step's dt from the maxima the previous step's
update took of the state it wrote (Sec. 3, CFL condition: the same
per-element quantity sum_A max_k |lambda_A| / h_A and the same maximum over
the mesh).  A call of ader_cfl_dt between steps discards those maxima, so
the next step reads u with the time-step kernel again.  Both sequences must
agree bit for bit in the state, the step sizes and the time, with update
tiles of several elements (3-D N = 3, ragged mesh), more elements per tile
than lanes of a wavefront (2-D N = 0), a single element per tile row chunk
(3-D N = 6), elasticity (material speeds) and a batch of mixed classes; and
graph replays must equal the same number of steps.
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


def _elastic(nel, N):
    return I.elastic_problem(nel=nel, N=N)


CASES = [
    ("euler3d_N3_ragged", lambda: [I.Problem(dim=3, N=3, nel=(9, 3, 2), lo=(0, 0, 0), hi=(1, 1, 1))],
     lambda p: I.fourier_modes(p)),
    ("euler2d_N0_70x3", lambda: [I.Problem(dim=2, N=0, nel=(70, 3), lo=(0, 0), hi=(10, 10))], I.isentropic_vortex),
    ("euler2d_N7_5x4", lambda: [I.Problem(dim=2, N=7, nel=(5, 4), lo=(0, 0), hi=(10, 10))], I.isentropic_vortex),
    ("euler3d_N6_3x2x2", lambda: [I.Problem(dim=3, N=6, nel=(3, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1))],
     lambda p: I.density_wave(p)),
    ("elastic_N2_4", lambda: [_elastic(4, 2)], lambda p: I.stress_pulse(p, width=0.2)),
    ("batch_mixed", lambda: [I.Problem(dim=3, N=2, nel=(4, 2, 3), lo=(0, 0, 0), hi=(1, 1, 1)),
                             I.vortex_problem(nel=6, N=3),
                             I.Problem(dim=3, N=3, nel=(5, 2, 3), lo=(0, 0, 0), hi=(1, 1, 1)),
                             I.Problem(dim=3, N=2, nel=(3, 3, 3), lo=(0, 0, 0), hi=(1, 1, 1))], None),
]


def _inits(probs, init):
    if init is not None:
        return [init(p) for p in probs]
    return [I.isentropic_vortex(p) if p.dim == 2 else I.density_wave(p) for p in probs]


@pytest.mark.parametrize("name,mk,init", CASES, ids=[c[0] for c in CASES])
def test_fused_maxima_bitwise(A, name, mk, init):
    import torch
    probs = mk()
    inits = _inits(probs, init)
    steps = 4
    say(f"[fused-cfl] {name}: {len(probs)} problem(s), {steps} steps")
    res = []
    for force in (False, True):
        ctx = A.Context(probs)
        u = ctx.upload(inits)
        dts = []
        for _ in range(steps):
            if force:
                ctx.cfl_dt(u)   # discards the update's maxima: the step runs the time-step kernel
            ctx.step(u, [1e9] * len(probs))
            dts.append(ctx.last_dt())
        torch.cuda.synchronize()
        res.append((u.cpu().numpy().copy(), np.array(dts), ctx.time()))
        ctx.close()
    (ua, da, ta), (ub, db, tb) = res
    assert np.array_equal(da, db), (da, db)
    assert np.array_equal(ta, tb)
    assert np.array_equal(ua.view(np.uint64), ub.view(np.uint64))


@pytest.mark.parametrize("name,mk,init", [CASES[0], CASES[4], CASES[5]], ids=["euler3d", "elastic", "batch"])
def test_fused_maxima_graph(A, name, mk, init):
    """Graph replays (the first step of the first replay from a time-step
    kernel pass before the replay, later ones from the update's maxima)
    against plain steps, with an ader_cfl_dt call between the replays."""
    import torch
    probs = mk()
    inits = _inits(probs, init)
    say(f"[fused-cfl] graph {name}")
    big = [1e9] * len(probs)
    ctx = A.Context(probs)
    u = ctx.upload(inits)
    for _ in range(6):
        ctx.step(u, big)
    torch.cuda.synchronize()
    ref = u.cpu().numpy().copy()
    ctx.close()
    ctx = A.Context(probs)
    u = ctx.upload(inits)
    ctx.run(u, big, 3)
    ctx.cfl_dt(u)
    ctx.run(u, big, 3)
    torch.cuda.synchronize()
    got = u.cpu().numpy().copy()
    ctx.close()
    assert np.array_equal(ref.view(np.uint64), got.view(np.uint64))

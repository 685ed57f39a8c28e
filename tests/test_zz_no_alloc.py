"""ader_totals_noalloc: the conservation sums without a context and without
allocation (static device scratch), against ader_totals of a context holding
the same problem.  Both use the same kernels and grid, so the sums must agree
bit for bit; two calls in a row, the second on a smaller problem, so the
scratch left by the first call cannot leak into the second."""
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


def _with_context(A, prob, u0):
    ctx = A.Context([prob])
    try:
        u = ctx.upload([u0])
        ref = ctx.totals(u)
    finally:
        ctx.close()
    return u, ref


CASES = [
    ("euler3d_then_smaller",
     [(lambda: I.Problem(dim=3, N=4, nel=(9, 7, 8), lo=(0, 0, 0), hi=(1, 1, 1)), I.density_wave),
      (lambda: I.Problem(dim=3, N=2, nel=(3, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1)), I.density_wave)]),
    ("elastic_then_euler2d",
     [(lambda: I.elastic_problem(nel=6, N=3), lambda p: I.stress_pulse(p, width=0.2)),
      (lambda: I.vortex_problem(nel=3, N=1), I.isentropic_vortex)]),
]


@pytest.mark.parametrize("name,seq", CASES, ids=[c[0] for c in CASES])
def test_totals_noalloc_matches_totals(A, name, seq):
    import torch
    stream = torch.cuda.current_stream()
    for i, (mk, init) in enumerate(seq):
        prob = mk()
        u0 = init(prob)
        u, ref = _with_context(A, prob, u0)
        sums = torch.full((prob.m,), float("nan"), dtype=torch.float64, device="cuda")
        say(f"[noalloc] {name} call {i}: {prob.pde} d={prob.dim} N={prob.N} E={prob.E}")
        A.ader_totals_noalloc(prob, u, sums, stream.cuda_stream)
        torch.cuda.synchronize()
        got = sums.cpu().numpy()
        say(f"  sums {got}")
        assert np.array_equal(got.view(np.uint64), np.asarray(ref, dtype=np.float64).view(np.uint64)), (got, ref)


def test_totals_noalloc_rejects_bad_problem(A):
    import torch
    prob = I.Problem(dim=3, N=2, nel=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1))
    u = torch.zeros(prob.E * prob.m * prob.nd, dtype=torch.float64, device="cuda")
    sums = torch.zeros(prob.m, dtype=torch.float64, device="cuda")
    prob.N = 9   # degree beyond the built range
    with pytest.raises(A.AderError) as e:
        A.ader_totals_noalloc(prob, u, sums)
    assert e.value.status == A.ADER_ERR_UNSUPPORTED
    with pytest.raises(A.AderError) as e:
        A.ader_totals_noalloc(I.Problem(dim=3, N=2, nel=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1)), None, sums)
    assert e.value.status == A.ADER_ERR_INVALID

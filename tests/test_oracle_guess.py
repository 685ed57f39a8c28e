"""Oracle pins of the initial guess extrapolated from the previous time
interval (Sec. 2.2, initial-guess paragraph; guess 3): the guess is the
previous interval's space-time polynomial continued in time and shifted to
the corrected state, it is accurate to the design order, and with it one
Picard sweep gives the scheme its design order (the paper's statement that a
guess of degree N-1 in time needs a single sweep)."""
import numpy as np
import pytest

from paper_1808_03788_amd import inputs as I


def _order(errs):
    return [np.log2(a / b) for a, b in zip(errs[:-1], errs[1:])]


@pytest.mark.parametrize("N,r", [(1, 1.0), (3, 0.8), (4, 1.3)])
def test_extrapolation_guess_is_the_previous_polynomial(orc, N, r):
    """Independent evaluation: the previous interval's nodal values at the
    Gauss-Legendre times are interpolated by numpy's polynomial fit, which
    is evaluated at the new time nodes 1 + xi_l r (in units of the previous
    step); the guess is u + p(1 + xi_l r) - p(1)."""
    prob = I.Problem(dim=2, N=N, nel=(2, 3), lo=(0, 0), hi=(10, 10), guess=3)
    rng = np.random.default_rng(7)
    n, nd = N + 1, (N + 1) ** 2
    u = I.isentropic_vortex(prob)
    qprev = u[:, :, None, :] + 1e-2 * rng.standard_normal((prob.E, prob.m, n, nd))
    dtprev = 0.01
    q0 = orc.predictor_hist(prob, u, dtprev * r, qprev, dtprev, guess_only=True)
    xi = (np.polynomial.legendre.leggauss(n)[0] + 1.0) / 2.0
    want = np.empty_like(q0)
    for e in range(prob.E):
        for v in range(prob.m):
            for k in range(nd):
                P = np.polynomial.Polynomial.fit(xi, qprev[e, v, :, k], N) if N > 0 else None
                for l in range(n):
                    want[e, v, l, k] = u[e, v, k] + (P(1.0 + xi[l] * r) - P(1.0))
    assert np.abs(q0 - want).max() <= 1e-10 * np.abs(want).max()


def test_extrapolation_guess_without_history_is_the_plain_scheme(orc):
    """The first step has no previous interval: constant guess and N+1
    sweeps, the plain scheme's step."""
    kw = dict(dim=3, N=2, nel=(3, 2, 2), lo=(0,) * 3, hi=(1,) * 3)
    u = I.density_wave(I.Problem(**kw))
    a, ta, da, _ = orc.step_hist(I.Problem(guess=3, **kw), u, 0.0, 1e9, None)
    b, tb, db = orc.step(I.Problem(guess=0, **kw), u, 0.0, 1e9)
    assert ta == tb and da == db
    assert np.array_equal(a, b)


def _guess_error(orc, N, nel):
    """max |q^0 - q*| at the third step of the density wave with CFL steps:
    q^0 the extrapolated guess, q* the converged Picard fixed point."""
    prob = I.density_wave_problem(nel=nel, N=N, guess=3)
    u, t, hist = I.density_wave(prob, noise=0), 0.0, None
    for _ in range(2):
        u, t, _, hist = orc.step_hist(prob, u, t, 1e9, hist)
    dt = orc.cfl_dt(prob, u)
    q0 = orc.predictor_hist(prob, u, dt, hist[0], hist[1], guess_only=True)
    qs, used = orc.predictor_converge(I.density_wave_problem(nel=nel, N=N), u, dt, 1e-15, 80)
    assert used < 80
    return np.abs(q0 - qs).max()


@pytest.mark.parametrize("N,meshes", [(2, (4, 8, 16)), (3, (4, 8))])
def test_extrapolation_guess_order(orc, N, meshes):
    """At a fixed CFL number the extrapolated guess differs from the
    converged predictor by O(h^(N+1)) (a degree-N polynomial continued over
    one more step, and a shift by the corrector's change of the end value
    that is O(dt h^N)), the accuracy of a guess of degree N in time."""
    errs = [_guess_error(orc, N, nel) for nel in meshes]
    assert min(_order(errs)) > N + 1 - 0.5, (errs, _order(errs))


@pytest.mark.parametrize("N,meshes", [(2, (8, 16)), (3, (4, 8))])
def test_order_with_extrapolation_guess_one_sweep(orc, N, meshes):
    """The scheme with the extrapolated guess and a single Picard sweep
    keeps the design order N+1 on the density wave, and its error against
    the exact solution is within 10% of the plain scheme's (constant guess,
    N+1 sweeps) on the same mesh."""
    errs, plain = [], []
    for nel in meshes:
        for guess, out in ((3, errs), (0, plain)):
            prob = I.density_wave_problem(nel=nel, N=N, guess=guess)
            u, t, _ = orc.run(prob, I.density_wave(prob, noise=0), 0.0, 0.05)
            out.append(I.l2_per_var(prob, u - I.density_wave(prob, t=t, noise=0))[0])
    assert _order(errs)[0] > N + 1 - 0.4, errs
    for a, b in zip(errs, plain):
        assert a <= 1.1 * b, (errs, plain)

"""Pins of the oracle's corrector, of its jump term across a material
interface, and of the predictor as the solution of an element-local linear
system.

Each test evaluates what the paper defines with code of its own (closed-form
path integrals, brute-force over-integrated quadrature of the weak forms,
exact reflection and transmission of a P wave, a dense linear solve) and
compares the oracle with it.  No GPU is needed.
"""
import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from paper_1808_03788_amd import inputs as I

# Stress component s_ij of the elastic state (u, v, w, sxx, syy, szz, sxy, syz, sxz).
SIG = [[3, 6, 8], [6, 4, 7], [8, 7, 5]]


def _lagrange(nodes, pts):
    """Lagrange basis of the nodes and its derivative at pts (Vandermonde solve)."""
    n = len(nodes)
    C = np.linalg.solve(np.vander(nodes, n, increasing=True), np.eye(n))
    L = np.stack([P.polyval(pts, C[:, k]) for k in range(n)], axis=-1)
    dL = np.stack([P.polyval(pts, P.polyder(C[:, k])) for k in range(n)], axis=-1)
    return L, dL


def _gauss01(n):
    z, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (z + 1.0), 0.5 * w


def _elastic_B(a, irho, lam, mu):
    """9x9 matrix B_a of the velocity-stress system (Sec. 3.2, volume fraction 1):
    v_t - (1/rho) div s = 0 and s_t - (lam tr(grad v) I + mu (grad v + grad v^T)) = 0,
    written as q_t + sum_a B_a dq/dx_a = 0."""
    B = np.zeros((9, 9))
    for i in range(3):
        B[i, SIG[i][a]] = -irho
    for i in range(3):
        for j in range(i, 3):
            r = SIG[i][j]
            if i == j:
                B[r, a] -= lam
            if i == a:
                B[r, j] -= mu
            if j == a:
                B[r, i] -= mu
    return B


def _cp(mat):
    rho, lam, mu = mat
    return np.sqrt((lam + 2 * mu) / rho)


def _path_mean_irho(r0, r1):
    """int_0^1 ds / (r0 + s (r1 - r0)): 1/rho along the straight path, exactly."""
    return 1.0 / r0 if r0 == r1 else np.log(r1 / r0) / (r1 - r0)


def _layered_material(nel, rng, layers_along=0):
    """Per-element (rho, lambda, mu): one material per slab along one axis."""
    E = int(np.prod(nel))
    idx = np.arange(E)
    coord = [idx % nel[0], (idx // nel[0]) % nel[1], idx // (nel[0] * nel[1])][layers_along]
    slabs = nel[layers_along]
    rho = rng.uniform(2000.0, 3000.0, slabs)
    cp = rng.uniform(3000.0, 6000.0, slabs)
    mu = rho * cp ** 2 / 3.0
    lam = rho * cp ** 2 - 2 * mu
    return np.stack([rho[coord], lam[coord], mu[coord]], axis=1)


def _neighbour(nel, e, a, d):
    idx = [e % nel[0], (e // nel[0]) % nel[1], e // (nel[0] * nel[1])]
    idx[a] = (idx[a] + d) % nel[a]
    return idx[0] + nel[0] * (idx[1] + nel[1] * idx[2])


# ------------------------------------------------- jump term at an interface

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_path_integral_closed_form(orc, axis):
    """Degree 0: one step is u_new = u - (dt/h) sum_faces D^-, so the update
    exposes the jump term of eqs. pc.scheme and rusanov directly.  With the
    material carried along the straight segment path (the material belongs to
    the state vector of the elastic system, Sec. 3.2), the path integral of
    B is B with 1/rho replaced by ln(rho+/rho-)/(rho+ - rho-) and lambda, mu by
    their means.  The oracle evaluates the path integral with the 3-point
    Gauss-Legendre rule, which is within 1e-6 of the exact value for the
    material contrasts below."""
    nel = [1, 1, 1]
    nel[axis] = 3
    prob = I.Problem(dim=3, N=0, nel=tuple(nel), lo=(0, 0, 0), hi=(0.3, 0.2, 0.25), pde="elastic")
    rng = np.random.default_rng(11 + axis)
    prob.material = _layered_material(nel, rng, layers_along=axis)
    u = rng.standard_normal((3, 9, 1))
    u[:, 3:] *= 1e7
    dt = 1e-6
    q = orc.predictor(prob, u, dt)
    np.testing.assert_array_equal(q[:, :, 0, :], u)   # degree 0: the predictor is u itself
    un = orc.corrector(prob, u, q, dt)
    h = prob.h[axis]
    exp = np.empty_like(u)
    for e in range(3):
        acc = np.zeros(9)
        me = prob.material[e]
        for d, sgn in ((+1, 1.0), (-1, -1.0)):
            nb = _neighbour(nel, e, axis, d)
            mn = prob.material[nb]
            B = _elastic_B(axis, _path_mean_irho(me[0], mn[0]), 0.5 * (me[1] + mn[1]), 0.5 * (me[2] + mn[2]))
            dq = u[nb, :, 0] - u[e, :, 0]
            smax = max(_cp(me), _cp(mn))
            acc += 0.5 * (sgn * B @ dq - smax * dq)
        exp[e, :, 0] = u[e, :, 0] - dt / h * acc
    inc_o, inc_e = un - u, exp - u
    scale = np.abs(inc_e).max(axis=(0, 2))
    assert (np.abs(inc_o - inc_e).max(axis=(0, 2)) <= 1e-5 * scale).all()
    # the same update with the material of the inside element only along the
    # path differs by far more than the tolerance (the pin is sensitive to it)
    alt = np.empty_like(u)
    for e in range(3):
        acc = np.zeros(9)
        me = prob.material[e]
        for d, sgn in ((+1, 1.0), (-1, -1.0)):
            nb = _neighbour(nel, e, axis, d)
            B = _elastic_B(axis, 1.0 / me[0], me[1], me[2])
            dq = u[nb, :, 0] - u[e, :, 0]
            acc += 0.5 * (sgn * B @ dq - max(_cp(me), _cp(prob.material[nb])) * dq)
        alt[e, :, 0] = u[e, :, 0] - dt / h * acc
    assert np.abs((alt - u) - inc_e).max() > 1e-3 * np.abs(inc_e).max()


def _pwave_run(orc, N, nx, rho2=1.5, c2=2.0, t_end=0.3):
    """Normal-incidence P wave (velocity u and stress sxx along x) crossing a
    material interface at x = 0.5 on a 1-D-in-x periodic mesh.  Medium 1
    (x < 0.5): rho = 1, c_p = 1; medium 2: rho2, c2; c_s = c_p / sqrt(3).
    A right-going Gaussian pulse u = f(x - t), sxx = -Z1 f (Z = rho c_p) starts
    at x0 = 0.3.  Continuity of velocity and traction at the interface gives
    the reflected and transmitted velocity amplitudes R = (Z1-Z2)/(Z1+Z2) and
    T = 2 Z1/(Z1+Z2); the exact solution at t_end (before any wave reaches
    the periodic seam at x = 0 = 1) is
      x < 0.5:  u = f(x - t) + R f(1 - x - t),
      x > 0.5:  u = T f(0.5 + (x - 0.5)/c2 - t).
    Returns the relative L2 error of u and the fitted amplitudes."""
    prob = I.Problem(dim=3, N=N, nel=(nx, 1, 1), lo=(0, 0, 0), hi=(1, 1, 1), pde="elastic")
    xc = (np.arange(nx) + 0.5) / nx
    mat = np.zeros((nx, 3))
    for i in range(nx):
        rho, c = (1.0, 1.0) if xc[i] < 0.5 else (rho2, c2)
        mu = rho * c * c / 3.0
        mat[i] = (rho, rho * c * c - 2 * mu, mu)
    prob.material = mat
    x = np.broadcast_to(I.grid(prob)[0], (1, 1, nx, prob.n, prob.n, prob.n))
    f = lambda z: np.exp(-(z - 0.3) ** 2 / (2 * 0.025 ** 2))
    Z1, Z2 = 1.0, rho2 * c2
    R, T = (Z1 - Z2) / (Z1 + Z2), 2 * Z1 / (Z1 + Z2)
    z = np.zeros_like(x)
    u0 = I.pack(prob, [f(x), z, z, -Z1 * f(x), z, z, z, z, z])
    u, t, _ = orc.run(prob, u0, 0.0, t_end)
    left = x < 0.5
    gR = np.where(left, f(1.0 - x - t), 0.0)
    gT = np.where(left, 0.0, f(0.5 + (x - 0.5) / c2 - t))
    ue = np.where(left, f(x - t), 0.0) + R * gR + T * gT
    un = u[:, 0, :].reshape(x.shape)
    w1 = _gauss01(prob.n)[1]
    W = np.broadcast_to(w1[None, None, None, None, None, :], x.shape)  # GL weights along x
    err = np.sqrt((W * (un - ue) ** 2).sum() / (W * ue ** 2).sum())
    Rn = (W * un * gR).sum() / (W * gR * gR).sum()
    Tn = (W * un * gT).sum() / (W * gT * gT).sum()
    return err, Rn, Tn, R, T


@pytest.mark.parametrize("N,meshes", [(2, (40, 80)), (3, (40, 80))])
def test_pwave_interface_reflection_transmission(orc, N, meshes):
    """The scheme converges at order N+1 to the exact solution of a P wave
    crossing a material interface, and the reflected and transmitted
    amplitudes tend to (Z1-Z2)/(Z1+Z2) and 2 Z1/(Z1+Z2).  (Any straight
    material path is consistent -- the path only multiplies the trace jump,
    which vanishes under refinement -- so this pins the interface physics;
    the path itself is pinned by test_path_integral_closed_form.)"""
    res = [_pwave_run(orc, N, nx) for nx in meshes]
    errs = [r[0] for r in res]
    order = np.log2(errs[0] / errs[1])
    assert order > N + 1 - 0.3, errs
    _, Rn, Tn, R, T = res[-1]
    tol = 2e-3 if N == 2 else 1e-4
    assert abs(Rn - R) < tol and abs(Tn - T) < tol, (Rn, R, Tn, T)


# ------------------------------------------------ corrector by brute force

def _corrector_bruteforce(prob, u, q, dt, nq):
    """u^{n+1} of eq. pde.nc.gw2 for the linear elastic system (F = 0,
    S = 0), every integral evaluated by nq-point Gauss quadrature per
    space-time direction with independent polynomial code:
      M (u^{n+1} - u^n) = - int int_{dOmega} Phi_k D^-.n dS dt - int int Phi_k B.grad q_h dx dt,
    M = int Phi_k Phi_l (diagonal), D^- of eq. pc.scheme with the straight
    path through state and material (1/rho integrated exactly)."""
    n, nd = prob.n, prob.nd
    nel, h = list(prob.nel), prob.h
    xi = _gauss01(n)[0]
    pts, wts = _gauss01(nq)
    L, dL = _lagrange(xi, pts)                 # (nq, n)
    L0, _ = _lagrange(xi, np.array([0.0]))
    L1, _ = _lagrange(xi, np.array([1.0]))
    Lend = [L0[0], L1[0]]
    vol = h[0] * h[1] * h[2]
    w_nodes = _gauss01(n)[1]
    Mk = vol * np.einsum("i,j,k->ijk", w_nodes, w_nodes, w_nodes)   # (k3, k2, k1)
    E = prob.E
    qr = q.reshape(E, 9, n, n, n, n)          # (e, v, l0, k3, k2, k1)
    out = np.empty_like(u)
    for e in range(E):
        me = prob.material[e]
        qe = qr[e]
        # volume: - int int Phi_k B . grad q_h
        ncp = np.zeros((9, nq, nq, nq, nq))
        for a in range(3):
            mats = [L, L, L, L]                 # (t, z, y, x)
            mats[3 - a] = dL
            g = np.einsum("vtzyx,Tt,Zz,Yy,Xx->vTZYX", qe, *mats) / h[a]
            ncp += np.einsum("rv,vTZYX->rTZYX", _elastic_B(a, 1.0 / me[0], me[1], me[2]), g)
        volk = np.einsum("rTZYX,T,Z,Y,X,Zk,Yj,Xi->rkji", ncp, wts, wts, wts, wts, L, L, L) * vol * dt
        face = np.zeros((9, n, n, n))
        for a in range(3):
            for side in (0, 1):
                sgn = 1.0 if side else -1.0
                nb = _neighbour(nel, e, a, 1 if side else -1)
                mn = prob.material[nb]
                # traces at the face quadrature points: contract axis a with the end values
                def trace(arr, end):
                    mats = [L, L, L, L]
                    mats[3 - a] = end[None, :]
                    return np.einsum("vtzyx,Tt,Zz,Yy,Xx->vTZYX", arr, *mats)
                qm = trace(qe, Lend[side])
                qp = trace(qr[nb], Lend[1 - side])
                B = _elastic_B(a, _path_mean_irho(me[0], mn[0]), 0.5 * (me[1] + mn[1]), 0.5 * (me[2] + mn[2]))
                smax = max(_cp(me), _cp(mn))
                dq = qp - qm
                D = 0.5 * (sgn * np.einsum("rv,v...->r...", B, dq) - smax * dq)
                mats = [L, L, L]                # test functions (z, y, x) on the face
                wz = [wts, wts, wts]
                mats[2 - a] = Lend[side][None, :]
                wz[2 - a] = np.ones(1)
                area = vol / h[a]
                face += np.einsum("rTZYX,T,Z,Y,X,Zk,Yj,Xi->rkji", D, wts, *wz, *mats) * area * dt
        inc = -(face + volk) / Mk[None]
        out[e] = u[e] + inc.reshape(9, nd)
    return out


@pytest.mark.parametrize("layered", [False, True])
def test_corrector_bruteforce_linear(orc, layered):
    """For the linear elastic system at N = 2 every integrand of eq.
    pde.nc.gw2 is a polynomial of degree <= 2N per direction, so the
    oracle's nodal Gauss-Legendre quadrature is exact and its update must
    equal brute-force quadrature of the weak form (any space-time polynomial
    q_h: random here).  Homogeneous medium: to round-off.  Layered medium:
    within the 3-point rule's error on the 1/rho path integral."""
    N = 2
    nel = (3, 3, 2)
    prob = I.Problem(dim=3, N=N, nel=nel, lo=(0, 0, 0), hi=(0.3, 0.45, 0.2), pde="elastic")
    rng = np.random.default_rng(21 + layered)
    if layered:
        prob.material = _layered_material(nel, rng, layers_along=2)
        prob.material = _layered_material(nel, rng, layers_along=0) * 0.5 + prob.material * 0.5
    else:
        prob.material = np.tile([2500.0, 2.1e10, 1.3e10], (prob.E, 1))
    u = rng.standard_normal((prob.E, 9, prob.nd))
    q = rng.standard_normal((prob.E, 9, prob.n, prob.nd))
    u[:, 3:] *= 1e7
    q[:, 3:] *= 1e7
    dt = 2e-6
    got = orc.corrector(prob, u, q, dt)
    ref = _corrector_bruteforce(prob, u, q, dt, nq=N + 3)
    inc_g, inc_r = got - u, ref - u
    scale = np.abs(inc_r).max(axis=(0, 2))
    err = np.abs(inc_g - inc_r).max(axis=(0, 2)) / scale
    assert (err <= (1e-5 if layered else 1e-12)).all(), err


# ------------------------------------------- predictor as a linear solve

def _predictor_system(prob, u, dt, nq):
    """Element-local linear system of eq. pde.st2 for the linear elastic
    system on one element (F = 0, S = 0), assembled column by column with
    nq-point quadrature in space-time (reference time tau = (t - t^n)/dt):
      int theta_k(1) q(1) - int int d_tau theta_k q - int theta_k(0) u
        = - dt int int theta_k B . grad q."""
    n, nd = prob.n, prob.nd
    xi = _gauss01(n)[0]
    pts, wts = _gauss01(nq)
    L, dL = _lagrange(xi, pts)
    L0, _ = _lagrange(xi, np.array([0.0]))
    L1, _ = _lagrange(xi, np.array([1.0]))
    me = prob.material[0]
    h = prob.h
    Bs = [_elastic_B(a, 1.0 / me[0], me[1], me[2]) for a in range(3)]
    ncol = 9 * n * nd

    def residual(qb, ub):            # qb (b, v, t, z, y, x), ub (v, z, y, x) or zeros
        term1 = np.einsum("bvtzyx,t,Zz,Yy,Xx,Z,Y,X,l,Zk,Yj,Xi->bvlkji", qb, L1[0], L, L, L, wts, wts, wts,
                          L1[0], L, L, L, optimize=True)
        term2 = np.einsum("bvtzyx,Tt,Zz,Yy,Xx,T,Z,Y,X,Tl,Zk,Yj,Xi->bvlkji", qb, L, L, L, L, wts, wts, wts, wts,
                          dL, L, L, L, optimize=True)
        ncp = 0.0
        for a in range(3):
            mats = [L, L, L, L]
            mats[3 - a] = dL
            g = np.einsum("bvtzyx,Tt,Zz,Yy,Xx->bvTZYX", qb, *mats, optimize=True) / h[a]
            ncp = ncp + np.einsum("rv,bvTZYX->brTZYX", Bs[a], g, optimize=True)
        termR = -np.einsum("brTZYX,T,Z,Y,X,Tl,Zk,Yj,Xi->brlkji", ncp, wts, wts, wts, wts, L, L, L, L, optimize=True)
        term3 = np.einsum("vzyx,Zz,Yy,Xx,Z,Y,X,l,Zk,Yj,Xi->vlkji", ub, L, L, L, wts, wts, wts, L0[0], L, L, L,
                          optimize=True)
        return term1 - term2 - term3[None] - dt * termR

    eye = np.eye(ncol).reshape(ncol, 9, n, n, n, n)
    zero_u = np.zeros((9, n, n, n))
    A = (residual(eye, zero_u)).reshape(ncol, ncol).T          # column c = response to unit q_c
    b = -residual(np.zeros((1, 9, n, n, n, n)), u[0].reshape(9, n, n, n)).reshape(ncol)
    return A, b


@pytest.mark.parametrize("N", [1, 2])
def test_predictor_equals_dense_solve(orc, N):
    """Linear homogeneous system: the Picard iterate after d*N sweeps from
    q0 = u_h equals the unique solution of the element-local linear system
    of eq. pde.st2, obtained here by a dense solve of the system assembled
    by over-integrated quadrature (reading c2: the iteration matrix is
    nilpotent of index dN+1 in d dimensions)."""
    prob = I.Problem(dim=3, N=N, nel=(1, 1, 1), lo=(0, 0, 0), hi=(0.01, 0.012, 0.009), pde="elastic")
    prob.material = np.array([[2500.0, 2.1e10, 1.3e10]])
    rng = np.random.default_rng(31 + N)
    u = rng.standard_normal((1, 9, prob.nd))
    u[:, 3:] *= 1e7
    dt = 3e-7
    A, b = _predictor_system(prob, u, dt, nq=N + 2)
    # scale the velocity and stress unknowns alike before solving
    s = np.ones((9, prob.n * prob.nd))
    s[3:] = 1e7
    s = s.reshape(-1)
    qd = (np.linalg.solve(A * s[None, :], b) * s).reshape(1, 9, prob.n, prob.nd)
    prob.picard = 3 * N
    qp = orc.predictor(prob, u, dt)
    for grp in (slice(0, 3), slice(3, 9)):
        ref = np.abs(qd[:, grp]).max()
        assert np.abs(qp[:, grp] - qd[:, grp]).max() <= 1e-11 * ref

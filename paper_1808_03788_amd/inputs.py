"""Seeded synthetic inputs for the ADER-DG hot path.

This module describes problems and writes initial data (and the exact
solutions of the smooth test cases) as FP64 nodal arrays.  It holds none of
the method's arithmetic: both the CPU oracle and the HIP library receive the
same arrays from here and compute everything else themselves.

Layout of a state array ``u`` (shared with the library interface):
``u[e][v][k]`` with ``e = ix + nx*(iy + ny*iz)`` and ``k = k1 + n*(k2 + n*k3)``
(k1 along x), ``n = N+1``.  Node ``k`` of element ``e`` sits at
``x_a = lo_a + (i_a + xi_{k_a}) h_a`` (Sec. 2.1, affine map to [0,1]^d), where
``xi`` are the Gauss-Legendre points of [0,1] (from numpy's ``leggauss``, used
here only to place the sample points).  Initial data are point values at the
nodes (nodal interpolation).

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

GAMMA = 1.4


@dataclasses.dataclass
class Problem:
    dim: int
    N: int
    nel: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    pde: str = "euler"            # "euler" | "elastic"
    gamma: float = GAMMA
    material: Optional[np.ndarray] = None   # elastic: [E, 3] = (rho, lambda, mu)
    picard: int = 0               # 0 -> N+1 sweeps
    cfl: float = 0.9
    prec: str = "fp64"            # predictor precision: fp64 | fp32 | bf16
    guess: int = 0                # initial guess of the Picard iteration
    face_avg: int = 0             # face integrals from time-averaged traces

    @property
    def n(self) -> int:
        return self.N + 1

    @property
    def m(self) -> int:
        return self.dim + 2 if self.pde == "euler" else 9

    @property
    def nd(self) -> int:
        return self.n ** self.dim

    @property
    def E(self) -> int:
        return int(np.prod(list(self.nel)[: self.dim]))

    @property
    def h(self):
        return [(self.hi[a] - self.lo[a]) / self.nel[a] for a in range(self.dim)]

    @property
    def dofs(self) -> int:
        """Spatial degrees of freedom E*(N+1)^d (without the factor m)."""
        return self.E * self.nd

    def zeros(self) -> np.ndarray:
        return np.zeros((self.E, self.m, self.nd))


def sample_points01(n: int) -> np.ndarray:
    z, _ = np.polynomial.legendre.leggauss(n)
    return 0.5 * (z + 1.0)


def grid(prob: Problem):
    """Broadcastable node coordinates, shape (nz,ny,nx,n,n,n) pattern (3-D) or
    (ny,nx,n,n) (2-D), in the C order of u[e][k]."""
    s = sample_points01(prob.n)
    d, n = prob.dim, prob.n
    coords = []
    for a in range(d):
        idx = np.arange(prob.nel[a])
        xa = prob.lo[a] + (idx[:, None] + s[None, :]) * prob.h[a]   # (nel_a, n)
        shape = [1] * (2 * d)
        shape[d - 1 - a] = prob.nel[a]
        shape[2 * d - 1 - a] = n
        coords.append(xa.reshape(shape))
    return coords


def pack(prob: Problem, fields) -> np.ndarray:
    """Stack m broadcast fields into u[E][m][nd]."""
    d = prob.dim
    full = [np.broadcast_to(f, tuple(list(prob.nel)[:d][::-1]) + (prob.n,) * d) for f in fields]
    u = np.stack(full, axis=d)   # (..elements.., m, ..nodes..)
    return np.ascontiguousarray(u.reshape(prob.E, prob.m, prob.nd))


def euler_state(prob: Problem, rho, vel, p):
    """Conservative Euler variables (rho, rho v, rho E) from primitives."""
    ke = 0.5 * rho * sum(np.asarray(v) ** 2 for v in vel)
    E = p / (prob.gamma - 1.0) + ke
    return [rho] + [rho * v for v in vel] + [E]


# ---------------------------------------------------------------- configs

def vortex_problem(nel: int = 16, N: int = 3, **kw) -> Problem:
    """2-D isentropic vortex on periodic [0,10]^2 (Euler, gamma = 1.4)."""
    return Problem(dim=2, N=N, nel=(nel, nel, 1), lo=(0.0, 0.0, 0.0), hi=(10.0, 10.0, 1.0), **kw)


def isentropic_vortex(prob: Problem, t: float = 0.0, eps: float = 5.0) -> np.ndarray:
    """Vortex of strength eps centred at (5,5) on the background
    (rho,u,v,p) = (1,1,1,1), translated by (t,t) with periodic minimum image:
    dv = eps/(2 pi) exp((1-r^2)/2) (-y', x'),
    T = p/rho = 1 - (gamma-1) eps^2/(8 gamma pi^2) exp(1-r^2), rho = T^{1/(gamma-1)},
    p = rho^gamma."""
    g = prob.gamma
    X, Y = grid(prob)
    L = 10.0
    xr = X - 5.0 - t
    yr = Y - 5.0 - t
    xr = xr - L * np.round(xr / L)
    yr = yr - L * np.round(yr / L)
    r2 = xr ** 2 + yr ** 2
    f = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = 1.0 - yr * f
    v = 1.0 + xr * f
    T = 1.0 - (g - 1.0) * eps ** 2 / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (g - 1.0))
    p = rho ** g
    return pack(prob, euler_state(prob, rho, [u, v], p))


def density_wave_problem(nel: int = 64, N: int = 4, **kw) -> Problem:
    """3-D Euler on the periodic unit cube."""
    return Problem(dim=3, N=N, nel=(nel, nel, nel), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), **kw)


def density_wave(prob: Problem, t: float = 0.0, amp: float = 0.2, noise: float = 1e-3,
                 seed: int = 0, kvec=(1, 1, 1), phase: float = 0.0, vel=(1.0, 1.0, 1.0)) -> np.ndarray:
    """rho = 1 + amp sin(2 pi k.(x - v t) + phase), v const, p = 1; then
    rho += noise * U(-1,1), i.i.d. per nodal DOF from default_rng(seed) drawn
    as one (E, nd) array; momentum rho v and E = p/(gamma-1) + rho |v|^2/2.
    Without noise this is an exact solution of the Euler equations."""
    X = grid(prob)
    arg = sum(kvec[a] * (X[a] - vel[a] * t) for a in range(prob.dim))
    rho = 1.0 + amp * np.sin(2.0 * math.pi * arg + phase)
    rho = np.broadcast_to(rho, tuple(list(prob.nel)[: prob.dim][::-1]) + (prob.n,) * prob.dim)
    rho = np.ascontiguousarray(rho).reshape(prob.E, prob.nd)
    if noise:
        rng = np.random.default_rng(seed)
        rho = rho + noise * rng.uniform(-1.0, 1.0, size=(prob.E, prob.nd))
    vel = [np.full_like(rho, vel[a]) for a in range(prob.dim)]
    fields = euler_state(prob, rho, vel, np.ones_like(rho))
    return np.ascontiguousarray(np.stack(fields, axis=1))


def uniform_state(prob: Problem, rho=1.0, vel=(0.3, -0.2, 0.1), p=1.0) -> np.ndarray:
    shape = (prob.E, prob.nd)
    if prob.pde == "euler":
        r = np.full(shape, rho)
        fields = euler_state(prob, r, [np.full(shape, vel[a]) for a in range(prob.dim)],
                             np.full(shape, p))
        return np.ascontiguousarray(np.stack(fields, axis=1))
    u = np.zeros((prob.E, 9, prob.nd))
    u[:, 0], u[:, 1], u[:, 2] = vel[0], vel[1], vel[2]
    u[:, 3:6] = p
    return u


def layered_material(prob: Problem, layers: int = 4, seed: int = 0) -> np.ndarray:
    """Per-element (rho, lambda, mu) of a medium of `layers` z-layers of equal
    thickness; per layer rho ~ U[2000,3000], c_p ~ U[3000,6000] (drawn in that
    order per layer from default_rng(seed)), c_s = c_p/sqrt(3),
    mu = rho c_s^2, lambda = rho c_p^2 - 2 mu."""
    rng = np.random.default_rng(seed)
    props = []
    for _ in range(layers):
        rho = rng.uniform(2000.0, 3000.0)
        cp = rng.uniform(3000.0, 6000.0)
        cs = cp / math.sqrt(3.0)
        mu = rho * cs * cs
        lam = rho * cp * cp - 2.0 * mu
        props.append((rho, lam, mu))
    nx, ny, nz = prob.nel
    iz = np.arange(prob.E) // (nx * ny)
    layer = (iz * layers) // nz
    return np.ascontiguousarray(np.array(props)[layer])


def elastic_problem(nel: int = 48, N: int = 5, layers: int = 4, seed: int = 0, **kw) -> Problem:
    prob = Problem(dim=3, N=N, nel=(nel, nel, nel), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                   pde="elastic", **kw)
    prob.material = layered_material(prob, layers, seed)
    return prob


def stress_pulse(prob: Problem, width: float = 0.05, centre=(0.5, 0.5, 0.375)) -> np.ndarray:
    """v = 0, sxx = syy = szz = exp(-|x - c|^2 / (2 width^2)), shear stress 0."""
    X = grid(prob)
    r2 = sum((X[a] - centre[a]) ** 2 for a in range(3))
    s = np.exp(-r2 / (2.0 * width ** 2))
    z = np.zeros_like(s)
    return pack(prob, [z, z, z, s, s, s, z, z, z])


def fourier_problem(nel: int = 128, N: int = 3, **kw) -> Problem:
    return density_wave_problem(nel=nel, N=N, **kw)


def fourier_modes(prob: Problem, modes: int = 8, amp: float = 0.05, seed: int = 0) -> np.ndarray:
    """rho = 1 + amp sum_i sin(2 pi k_i.x + phi_i), v_c = amp sum_i sin(2 pi k_i.x + phi_ic),
    p = 1, with k_i in {-4..4}^3 minus 0 and phases U[0, 2 pi).  Draw order per
    mode: k_i (3 integers, redrawn while zero), phi_i, phi_i1..phi_id."""
    rng = np.random.default_rng(seed)
    X = grid(prob)
    d = prob.dim
    rho = 1.0
    vel = [0.0] * d
    for _ in range(modes):
        k = np.zeros(d, dtype=int)
        while not k.any():
            k = rng.integers(-4, 5, size=d)
        ph = rng.uniform(0.0, 2.0 * math.pi, size=1 + d)
        arg = 2.0 * math.pi * sum(int(k[a]) * X[a] for a in range(d))
        rho = rho + amp * np.sin(arg + ph[0])
        for c in range(d):
            vel[c] = vel[c] + amp * np.sin(arg + ph[1 + c])
    p = 1.0
    shape = tuple(list(prob.nel)[:d][::-1]) + (prob.n,) * d
    rho = np.broadcast_to(rho, shape)
    vel = [np.broadcast_to(v, shape) for v in vel]
    return pack(prob, euler_state(prob, rho, vel, np.full(shape, p)))


def batched_problems(count: int = 256, seed: int = 0, edge=(8, 32), degrees=(2, 6), prec="fp32"):
    """`count` independent 3-D Euler density waves on the unit cube.  Per
    problem (draw order): edge k ~ U{edge}, N ~ U{degrees}, A ~ U[0.05,0.2],
    a in {1,2}^3, phi ~ U[0, 2 pi).  Returns [(Problem, params)]; the initial
    data are density_wave(prob, amp=A, noise=0, kvec=a, phase=phi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(edge[0], edge[1] + 1))
        N = int(rng.integers(degrees[0], degrees[1] + 1))
        A = float(rng.uniform(0.05, 0.2))
        a = tuple(int(x) for x in rng.integers(1, 3, size=3))
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        prob = density_wave_problem(nel=k, N=N, prec=prec)
        out.append((prob, dict(amp=A, noise=0.0, kvec=a, phase=phi)))
    return out


# ----------------------------------------------------------------- norms

def quad_weights(prob: Problem) -> np.ndarray:
    """|Omega_e| prod_a w_{k_a} for one element, shape (nd,)."""
    _, w = np.polynomial.legendre.leggauss(prob.n)
    w = 0.5 * w
    W = w
    for _ in range(prob.dim - 1):
        W = np.multiply.outer(w, W)
    return W.reshape(-1) * float(np.prod(prob.h))


def l2_per_var(prob: Problem, f: np.ndarray) -> np.ndarray:
    """Discrete L2 norm per variable: sqrt(sum_e |Omega_e| sum_k w_k f^2)."""
    W = quad_weights(prob)
    return np.sqrt(np.einsum("evk,k->v", f * f, W))


def rel_l2(prob: Problem, a: np.ndarray, ref: np.ndarray) -> float:
    """Max over variables of ||a - ref||_2 / ||ref||_2 (absolute where the
    reference variable is identically zero)."""
    num = l2_per_var(prob, a - ref)
    den = l2_per_var(prob, ref)
    r = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return float(r.max())


def linf(a: np.ndarray, ref: np.ndarray) -> float:
    return float(np.max(np.abs(a - ref)))


def rel_linf(a: np.ndarray, ref: np.ndarray) -> float:
    """Max over variables of max |a - ref| / max |ref| over the nodes of all
    elements (absolute where the reference variable is identically zero);
    a and ref are [E][m][nd]."""
    d = np.abs(np.asarray(a) - np.asarray(ref)).max(axis=(0, 2))
    s = np.abs(np.asarray(ref)).max(axis=(0, 2))
    return float(np.where(s > 0, d / np.where(s > 0, s, 1.0), d).max())


def homogeneous_material(prob: Problem, rho=2500.0, cp=4500.0) -> np.ndarray:
    cs = cp / math.sqrt(3.0)
    mu = rho * cs * cs
    lam = rho * cp * cp - 2.0 * mu
    return np.tile(np.array([rho, lam, mu]), (prob.E, 1))


def elastic_plane_waves(prob: Problem, t: float = 0.0, amp: float = 1e-3) -> np.ndarray:
    """Exact solution in a homogeneous medium (material of element 0): a P wave
    along n1 = (1,1,0)/sqrt2 (velocity along n1) plus an S wave along
    n2 = (0,1,1)/sqrt2 polarised along x, both of unit-cube periodic wave
    vector 2 pi (1,1,0) and 2 pi (0,1,1).  For a plane wave with velocity
    a f(n.x - c t) the stress is sigma = -(1/c) f (lambda (n.a) I + mu (n a^T + a n^T))."""
    rho, lam, mu = prob.material[0]
    cp = math.sqrt((lam + 2 * mu) / rho)
    cs = math.sqrt(mu / rho)
    X = grid(prob)
    waves = [((1.0, 1.0, 0.0), (1.0, 1.0, 0.0), cp), ((0.0, 1.0, 1.0), (1.0, 0.0, 0.0), cs)]
    vel = [0.0, 0.0, 0.0]
    sig = np.zeros((3, 3), dtype=object)
    sig[:, :] = 0.0
    for kvec, pol, c in waves:
        kn = math.sqrt(sum(k * k for k in kvec))
        n = [k / kn for k in kvec]
        pn = math.sqrt(sum(p * p for p in pol))
        a = [amp * p / pn for p in pol]
        kk = 2.0 * math.pi * kn
        f = np.sin(2.0 * math.pi * sum(kvec[i] * X[i] for i in range(3)) - kk * c * t)
        na = sum(n[i] * a[i] for i in range(3))
        for i in range(3):
            vel[i] = vel[i] + a[i] * f
            for j in range(3):
                s = mu * (n[i] * a[j] + a[i] * n[j]) + (lam * na if i == j else 0.0)
                sig[i, j] = sig[i, j] - s / c * f
    return pack(prob, [vel[0], vel[1], vel[2], sig[0, 0], sig[1, 1], sig[2, 2],
                       sig[0, 1], sig[1, 2], sig[0, 2]])

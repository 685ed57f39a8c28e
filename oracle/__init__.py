"""FP64 CPU oracle of the ADER-DG hot path -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library and its Python binding
never do: the two implementations share no code.  The arithmetic lives in
``ader_oracle.c`` (plain C99, FP64, OpenMP over whole elements); this module
only marshals numpy arrays through ctypes.

Problems are passed as any object with the attributes ``dim, N, nel, lo, hi,
pde ('euler' | 'elastic'), gamma, material ([E,3] or None), picard, cfl``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ader_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no intrinsics, -O2)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("N", C.c_int), ("nel", C.c_int * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("pde", C.c_int), ("gamma", C.c_double),
        ("material", C.POINTER(C.c_double)),
        ("picard", C.c_int), ("cfl", C.c_double), ("guess", C.c_int), ("face_avg", C.c_int),
    ]


_lib = None
_DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        L.orc_gauss_legendre.argtypes = [C.c_int, _DP, _DP]
        L.orc_lagrange.argtypes = [C.c_int, _DP, C.c_int, C.c_double]
        L.orc_lagrange.restype = C.c_double
        L.orc_lagrange_deriv.argtypes = [C.c_int, _DP, C.c_int, C.c_double]
        L.orc_lagrange_deriv.restype = C.c_double
        L.orc_operators.argtypes = [C.c_int] + [_DP] * 8
        L.orc_nvar.argtypes = [C.POINTER(_Problem)]
        L.orc_stability_alpha.argtypes = [C.c_int]
        L.orc_stability_alpha.restype = C.c_double
        L.orc_cfl_dt.argtypes = [C.POINTER(_Problem), _DP]
        L.orc_cfl_dt.restype = C.c_double
        L.orc_predictor.argtypes = [C.POINTER(_Problem), _DP, C.c_double, _DP]
        L.orc_predictor_converge.argtypes = [C.POINTER(_Problem), _DP, C.c_double,
                                             C.c_double, C.c_int, _DP]
        L.orc_corrector.argtypes = [C.POINTER(_Problem), _DP, _DP, C.c_double, _DP]
        L.orc_step.argtypes = [C.POINTER(_Problem), _DP, _DP, C.c_double, _DP]
        L.orc_predictor_hist.argtypes = [C.POINTER(_Problem), _DP, C.c_double, _DP, C.c_double, _DP]
        L.orc_guess_hist.argtypes = [C.POINTER(_Problem), _DP, C.c_double, _DP, C.c_double, _DP]
        L.orc_step_hist.argtypes = [C.POINTER(_Problem), _DP, _DP, C.c_double, _DP, _DP, _DP,
                                    C.POINTER(C.c_int)]
        L.orc_totals.argtypes = [C.POINTER(_Problem), _DP, _DP]
        L.orc_detect.argtypes = [C.POINTER(_Problem), _DP, _DP, C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


class _Bound:
    """A problem marshalled into the oracle's C struct (keeps material alive)."""

    def __init__(self, prob):
        s = _Problem()
        s.dim = prob.dim
        s.N = prob.N
        nel = list(prob.nel) + [1] * (3 - len(prob.nel))
        lo = list(prob.lo) + [0.0] * (3 - len(prob.lo))
        hi = list(prob.hi) + [1.0] * (3 - len(prob.hi))
        for a in range(3):
            s.nel[a] = int(nel[a])
            s.lo[a] = float(lo[a])
            s.hi[a] = float(hi[a])
        s.pde = 0 if prob.pde == "euler" else 1
        s.gamma = float(getattr(prob, "gamma", 1.4))
        self.mat = None
        if s.pde == 1:
            self.mat = np.ascontiguousarray(prob.material, dtype=np.float64)
            s.material = _ptr(self.mat)
        s.picard = int(getattr(prob, "picard", 0) or 0)
        s.cfl = float(getattr(prob, "cfl", 0.9))
        s.guess = int(getattr(prob, "guess", 0) or 0)
        s.face_avg = int(getattr(prob, "face_avg", 0) or 0)
        self.s = s
        self.n = prob.N + 1
        self.nd = self.n ** prob.dim
        self.E = int(np.prod(nel[: prob.dim]))
        self.m = lib().orc_nvar(C.byref(s))

    @property
    def ref(self):
        return C.byref(self.s)


def operators(N: int) -> dict:
    """Gauss-Legendre rule and the 1-D operator tables of degree N."""
    n = N + 1
    out = {k: np.zeros(n * n) for k in ("Dhat", "K", "K1", "T")}
    out.update({k: np.zeros(n) for k in ("xi", "w", "F0", "F1")})
    rc = lib().orc_operators(N, *(_ptr(out[k]) for k in
                                  ("xi", "w", "Dhat", "F0", "F1", "K", "K1", "T")))
    assert rc == 0
    for k in ("Dhat", "K", "K1", "T"):
        out[k] = out[k].reshape(n, n)
    return out


def gauss_legendre(n: int):
    xi, w = np.zeros(n), np.zeros(n)
    assert lib().orc_gauss_legendre(n, _ptr(xi), _ptr(w)) == 0
    return xi, w


def lagrange(xi: np.ndarray, k: int, x: float, deriv: bool = False) -> float:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    f = lib().orc_lagrange_deriv if deriv else lib().orc_lagrange
    return f(len(xi), _ptr(xi), k, float(x))


def stability_alpha(N: int) -> float:
    return lib().orc_stability_alpha(N)


def cfl_dt(prob, u: np.ndarray) -> float:
    b = _Bound(prob)
    return lib().orc_cfl_dt(b.ref, _ptr(np.ascontiguousarray(u, dtype=np.float64)))


def predictor(prob, u: np.ndarray, dt: float) -> np.ndarray:
    """Space-time DOFs q[E][m][n][n^d] of the Picard predictor."""
    b = _Bound(prob)
    u = np.ascontiguousarray(u, dtype=np.float64)
    q = np.zeros((b.E, b.m, b.n, b.nd))
    assert lib().orc_predictor(b.ref, _ptr(u), float(dt), _ptr(q)) == 0
    return q


def detect(prob, u_old: np.ndarray, u_new: np.ndarray) -> np.ndarray:
    """Troubled-element flags [E] (bit 1 NaN/Inf, 2 positivity, 4 relaxed DMP)."""
    b = _Bound(prob)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    u_new = np.ascontiguousarray(u_new, dtype=np.float64)
    flags = np.zeros(b.E, dtype=np.int32)
    assert lib().orc_detect(b.ref, _ptr(u_old), _ptr(u_new), flags.ctypes.data_as(C.c_void_p)) == 0
    return flags


def initial_guess(prob, u: np.ndarray, dt: float) -> np.ndarray:
    """The Picard iteration's initial guess q^0[E][m][n][n^d] selected by
    prob.guess (no sweep)."""
    q, used = predictor_converge(prob, u, dt, 0.0, 0)
    assert used == 0
    return q


def predictor_converge(prob, u: np.ndarray, dt: float, tol: float, max_sweeps: int):
    b = _Bound(prob)
    u = np.ascontiguousarray(u, dtype=np.float64)
    q = np.zeros((b.E, b.m, b.n, b.nd))
    used = lib().orc_predictor_converge(b.ref, _ptr(u), float(dt), float(tol),
                                        int(max_sweeps), _ptr(q))
    assert used >= 0
    return q, used


def corrector(prob, u: np.ndarray, q: np.ndarray, dt: float) -> np.ndarray:
    b = _Bound(prob)
    u = np.ascontiguousarray(u, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    un = np.zeros_like(u)
    assert lib().orc_corrector(b.ref, _ptr(u), _ptr(q), float(dt), _ptr(un)) == 0
    return un


def step(prob, u: np.ndarray, t: float, t_end: float):
    """One step in place on a copy; returns (u_new, t_new, dt)."""
    b = _Bound(prob)
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    tt = C.c_double(t)
    dt = C.c_double(0.0)
    rc = lib().orc_step(b.ref, _ptr(u), C.byref(tt), float(t_end), C.byref(dt))
    if rc != 0:
        raise FloatingPointError("oracle: non-physical or non-finite state")
    return u, tt.value, dt.value


def predictor_hist(prob, u: np.ndarray, dt: float, qprev=None, dtprev: float = 0.0,
                   guess_only: bool = False) -> np.ndarray:
    """Predictor (or, with guess_only, its initial guess alone) with the
    previous interval's predictor qprev[E][m][n][n^d] of step dtprev (guess 3)."""
    b = _Bound(prob)
    u = np.ascontiguousarray(u, dtype=np.float64)
    q = np.zeros((b.E, b.m, b.n, b.nd))
    qp = None if qprev is None else np.ascontiguousarray(qprev, dtype=np.float64)
    f = lib().orc_guess_hist if guess_only else lib().orc_predictor_hist
    assert f(b.ref, _ptr(u), float(dt), None if qp is None else _ptr(qp), float(dtprev), _ptr(q)) == 0
    return q


def step_hist(prob, u: np.ndarray, t: float, t_end: float, hist=None):
    """One step that carries the previous interval (guess 3): hist is None
    or (qprev, dtprev) from the step before; returns (u_new, t_new, dt, hist)."""
    b = _Bound(prob)
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    if hist is None:
        qprev, dtp, has = np.zeros((b.E, b.m, b.n, b.nd)), C.c_double(0.0), C.c_int(0)
    else:
        qprev, dtp, has = np.array(hist[0], dtype=np.float64, order="C", copy=True), C.c_double(hist[1]), C.c_int(1)
    tt = C.c_double(t)
    dt = C.c_double(0.0)
    rc = lib().orc_step_hist(b.ref, _ptr(u), C.byref(tt), float(t_end), C.byref(dt), _ptr(qprev), C.byref(dtp),
                             C.byref(has))
    if rc != 0:
        raise FloatingPointError("oracle: non-physical or non-finite state")
    return u, tt.value, dt.value, (qprev, dtp.value)


def run(prob, u: np.ndarray, t0: float, t_end: float, max_steps: int = 1 << 30):
    """Steps until t_end or max_steps; returns (u, t, steps)."""
    t, steps, hist = t0, 0, None
    while t < t_end and steps < max_steps:
        if int(getattr(prob, "guess", 0) or 0) == 3:
            u, t, _, hist = step_hist(prob, u, t, t_end, hist)
        else:
            u, t, _ = step(prob, u, t, t_end)
        steps += 1
    return u, t, steps


def totals(prob, u: np.ndarray) -> np.ndarray:
    b = _Bound(prob)
    out = np.zeros(b.m)
    assert lib().orc_totals(b.ref, _ptr(np.ascontiguousarray(u, dtype=np.float64)),
                            _ptr(out)) == 0
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops (for timing)."""
    lib().orc_set_threads(int(n))

"""Thin ctypes binding of ``libader.so`` (declared in ``include/ader.h``).

Every function below marshals its arguments and calls the C entry point of
the same name; all arithmetic runs in the library's HIP kernels.  Device
buffers are torch tensors (torch is used for device memory and streams
only).  If the library is missing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libader.so")

ADER_OK, ADER_ERR_INVALID, ADER_ERR_UNSUPPORTED, ADER_ERR_OOM, ADER_ERR_DEVICE, ADER_ERR_NONFINITE = range(6)
ADER_EULER, ADER_ELASTIC = 0, 1
ADER_FP64, ADER_FP32, ADER_BF16 = 0, 1, 2
PREC = {"fp64": ADER_FP64, "fp32": ADER_FP32, "bf16": ADER_BF16}
PDE = {"euler": ADER_EULER, "elastic": ADER_ELASTIC}

EXPORTS = [
    "ader_create", "ader_destroy", "ader_layout", "ader_state_size", "ader_cfl_dt",
    "ader_predictor", "ader_qhat_layout", "ader_corrector", "ader_step", "ader_time",
    "ader_set_time", "ader_last_dt", "ader_totals", "ader_last_error",
    "ader_stability_alpha", "ader_basis", "ader_version", "ader_profile", "ader_stage_times",
    "ader_describe", "ader_run", "ader_set_detection", "ader_detect_flags",
    "ader_totals_noalloc",
]


class ader_problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("degree", C.c_int32), ("nelem", C.c_int32 * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("pde", C.c_int32), ("gamma", C.c_double), ("material", C.POINTER(C.c_double)),
        ("prec", C.c_int32), ("picard_iters", C.c_int32), ("cfl", C.c_double),
        ("guess", C.c_int32), ("face_avg", C.c_int32),
    ]


class AderError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ader status {status}: {msg}")
        self.status = status


_lib = None
_DP = C.POINTER(C.c_double)
_VP = C.c_void_p


def lib():
    """Load libader.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1808_03788_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.ader_create.argtypes = [C.POINTER(ader_problem), C.c_int32, _VP, C.POINTER(_VP)]
        L.ader_destroy.argtypes = [_VP]
        L.ader_layout.argtypes = [_VP, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.ader_qhat_layout.argtypes = [_VP, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.ader_state_size.argtypes = [_VP, C.POINTER(C.c_int64)]
        L.ader_cfl_dt.argtypes = [_VP, _VP, _DP]
        L.ader_predictor.argtypes = [_VP, _VP, _VP, _VP]
        L.ader_corrector.argtypes = [_VP, _VP, _VP]
        L.ader_step.argtypes = [_VP, _VP, _DP]
        L.ader_run.argtypes = [_VP, _VP, _DP, C.c_int32]
        L.ader_set_detection.argtypes = [_VP, C.c_int32]
        L.ader_detect_flags.argtypes = [_VP, _VP]
        L.ader_time.argtypes = [_VP, _DP]
        L.ader_set_time.argtypes = [_VP, _DP]
        L.ader_last_dt.argtypes = [_VP, _DP]
        L.ader_totals.argtypes = [_VP, _VP, _DP]
        L.ader_totals_noalloc.argtypes = [C.POINTER(ader_problem), _VP, _VP, _VP]
        L.ader_last_error.argtypes = [_VP]
        L.ader_last_error.restype = C.c_char_p
        L.ader_stability_alpha.argtypes = [C.c_int32, _DP]
        L.ader_basis.argtypes = [C.c_int32, _DP, _DP, _DP, _DP]
        L.ader_version.restype = C.c_char_p
        L.ader_profile.argtypes = [_VP, C.c_int32]
        L.ader_stage_times.argtypes = [_VP, _DP, C.POINTER(C.c_int64)]
        L.ader_describe.argtypes = [_VP, C.c_int32, C.c_char_p, C.c_int32]
        for name in EXPORTS:
            if name not in ("ader_last_error", "ader_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int, ctx=None):
    if status != ADER_OK:
        msg = lib().ader_last_error(ctx).decode(errors="replace")
        raise AderError(status, msg)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


# ------------------------------------------------------------ host queries

def ader_version() -> str:
    return lib().ader_version().decode()


def ader_stability_alpha(degree: int) -> float:
    a = C.c_double()
    _check(lib().ader_stability_alpha(degree, C.byref(a)))
    return a.value


def ader_basis(degree: int):
    n = degree + 1
    xi, w, d, t = np.zeros(n), np.zeros(n), np.zeros(n * n), np.zeros(n * n)
    p = lambda a: a.ctypes.data_as(_DP)
    _check(lib().ader_basis(degree, p(xi), p(w), p(d), p(t)))
    return xi, w, d.reshape(n, n), t.reshape(n, n)


# ------------------------------------------------------------ context calls

def make_problem(prob, keep: list) -> ader_problem:
    """Marshal a problem description (attributes dim, N, nel, lo, hi, pde,
    gamma, material, prec, picard, cfl) into the C struct."""
    s = ader_problem()
    s.dim = prob.dim
    s.degree = prob.N
    nel = list(prob.nel) + [1] * (3 - len(prob.nel))
    lo = list(prob.lo) + [0.0] * (3 - len(prob.lo))
    hi = list(prob.hi) + [1.0] * (3 - len(prob.hi))
    for a in range(3):
        s.nelem[a] = int(nel[a])
        s.lo[a] = float(lo[a])
        s.hi[a] = float(hi[a])
    s.pde = PDE[prob.pde]
    s.gamma = float(getattr(prob, "gamma", 1.4))
    if prob.pde == "elastic":
        mat = np.ascontiguousarray(prob.material, dtype=np.float64)
        keep.append(mat)
        s.material = mat.ctypes.data_as(_DP)
    s.prec = PREC[getattr(prob, "prec", "fp64")]
    s.picard_iters = int(getattr(prob, "picard", 0) or 0)
    s.guess = int(getattr(prob, "guess", 0) or 0)
    s.face_avg = int(getattr(prob, "face_avg", 0) or 0)
    s.cfl = float(getattr(prob, "cfl", 0.9))
    return s


def ader_create(problems: Sequence, stream: int = 0) -> int:
    keep: list = []
    arr = (ader_problem * len(problems))(*[make_problem(p, keep) for p in problems])
    ctx = _VP()
    _check(lib().ader_create(arr, len(problems), _VP(stream), C.byref(ctx)))
    return ctx.value


def ader_destroy(ctx: int):
    _check(lib().ader_destroy(_VP(ctx)))


def ader_layout(ctx: int, prob: int):
    off, cnt = C.c_int64(), C.c_int64()
    _check(lib().ader_layout(_VP(ctx), prob, C.byref(off), C.byref(cnt)), ctx)
    return off.value, cnt.value


def ader_qhat_layout(ctx: int, prob: int):
    off, cnt = C.c_int64(), C.c_int64()
    _check(lib().ader_qhat_layout(_VP(ctx), prob, C.byref(off), C.byref(cnt)), ctx)
    return off.value, cnt.value


def ader_state_size(ctx: int) -> int:
    cnt = C.c_int64()
    _check(lib().ader_state_size(_VP(ctx), C.byref(cnt)), ctx)
    return cnt.value


def ader_cfl_dt(ctx: int, u, nprob: Optional[int] = None):
    """Launch the time-step reduction; with nprob, synchronise and return dt."""
    if nprob is None:
        _check(lib().ader_cfl_dt(_VP(ctx), _VP(_ptr(u)), None), ctx)
        return None
    out = np.zeros(nprob)
    _check(lib().ader_cfl_dt(_VP(ctx), _VP(_ptr(u)), out.ctypes.data_as(_DP)), ctx)
    return out


def ader_predictor(ctx: int, u, dt_dev=None, qhat_out=None):
    _check(lib().ader_predictor(_VP(ctx), _VP(_ptr(u)), _VP(_ptr(dt_dev)), _VP(_ptr(qhat_out))), ctx)


def ader_corrector(ctx: int, u, dt_dev=None):
    _check(lib().ader_corrector(_VP(ctx), _VP(_ptr(u)), _VP(_ptr(dt_dev))), ctx)


def ader_step(ctx: int, u, t_end: Sequence[float]):
    te = np.ascontiguousarray(t_end, dtype=np.float64)
    _check(lib().ader_step(_VP(ctx), _VP(_ptr(u)), te.ctypes.data_as(_DP)), ctx)


def ader_run(ctx: int, u, t_end: Sequence[float], nsteps: int):
    te = np.ascontiguousarray(t_end, dtype=np.float64)
    _check(lib().ader_run(_VP(ctx), _VP(_ptr(u)), te.ctypes.data_as(_DP), int(nsteps)), ctx)


def ader_set_detection(ctx: int, enable: bool):
    _check(lib().ader_set_detection(_VP(ctx), 1 if enable else 0), ctx)


def ader_detect_flags(ctx: int, total_elements: int) -> np.ndarray:
    out = np.zeros(total_elements, dtype=np.int32)
    _check(lib().ader_detect_flags(_VP(ctx), out.ctypes.data_as(_VP)), ctx)
    return out


def ader_time(ctx: int, nprob: int) -> np.ndarray:
    out = np.zeros(nprob)
    _check(lib().ader_time(_VP(ctx), out.ctypes.data_as(_DP)), ctx)
    return out


def ader_set_time(ctx: int, t: Sequence[float]):
    tt = np.ascontiguousarray(t, dtype=np.float64)
    _check(lib().ader_set_time(_VP(ctx), tt.ctypes.data_as(_DP)), ctx)


def ader_last_dt(ctx: int, nprob: int) -> np.ndarray:
    out = np.zeros(nprob)
    _check(lib().ader_last_dt(_VP(ctx), out.ctypes.data_as(_DP)), ctx)
    return out


def ader_totals(ctx: int, u, nvars: int) -> np.ndarray:
    out = np.zeros(nvars)
    _check(lib().ader_totals(_VP(ctx), _VP(_ptr(u)), out.ctypes.data_as(_DP)), ctx)
    return out


def ader_totals_noalloc(prob, u, sums_dev, stream: int = 0):
    """Domain integrals of one problem's state u into the device buffer
    sums_dev (m doubles), without a context and without allocation; does not
    synchronise."""
    keep: list = []
    desc = make_problem(prob, keep)
    _check(lib().ader_totals_noalloc(C.byref(desc), _VP(_ptr(u)), _VP(_ptr(sums_dev)), _VP(stream)))


def ader_profile(ctx: int, enable: bool):
    _check(lib().ader_profile(_VP(ctx), int(bool(enable))), ctx)


STAGES = ("cfl", "predictor", "face", "update")


def ader_stage_times(ctx: int):
    """Summed device milliseconds and step counts per stage of ader_step."""
    ms = np.zeros(4)
    cnt = (C.c_int64 * 4)()
    _check(lib().ader_stage_times(_VP(ctx), ms.ctypes.data_as(_DP), cnt), ctx)
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(4)}


def ader_describe(ctx: int, prob: int = 0) -> str:
    buf = C.create_string_buffer(512)
    _check(lib().ader_describe(_VP(ctx), prob, buf, 512), ctx)
    return buf.value.decode()


def ader_last_error(ctx: Optional[int]) -> str:
    return lib().ader_last_error(_VP(ctx)).decode(errors="replace")


# ------------------------------------------------------------ convenience

class Context:
    """Owns one ader_ctx on the current torch device and stream.

    ``u`` buffers are flat float64 CUDA tensors of ``state_size`` doubles;
    ``upload``/``download`` convert per-problem numpy arrays u[E][m][nd].
    """

    def __init__(self, problems: Sequence, stream=None):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("the ADER library needs a HIP device")
        self.problems = list(problems)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = ader_create(self.problems, self.stream.cuda_stream)
        self.nprob = len(self.problems)
        self.size = ader_state_size(self.ctx)
        self.layouts = [ader_layout(self.ctx, p) for p in range(self.nprob)]
        self.nvars = sum(p.m for p in self.problems)

    def _state(self, u):
        """The state buffer the kernels will index: a contiguous float64
        tensor on the GPU with at least state_size values (checked here
        because the library trusts its pointer arguments)."""
        t = self.torch
        if not isinstance(u, t.Tensor) or u.dtype != t.float64 or not u.is_cuda or not u.is_contiguous():
            raise ValueError("u must be a contiguous float64 GPU tensor")
        if u.numel() < self.size:
            raise ValueError(f"u holds {u.numel()} values, the context needs {self.size}")
        return u

    def _per_problem(self, x, what):
        """One float64 value per problem (a scalar is broadcast)."""
        a = np.full(self.nprob, float(x)) if np.isscalar(x) else np.ascontiguousarray(x, dtype=np.float64)
        if a.shape != (self.nprob,):
            raise ValueError(f"{what} needs {self.nprob} values, got shape {a.shape}")
        return a

    def close(self):
        if self.ctx:
            ader_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        return self.torch.empty(self.size, dtype=self.torch.float64, device="cuda")

    def upload(self, arrays):
        if len(arrays) != self.nprob:
            raise ValueError(f"{len(arrays)} arrays for {self.nprob} problems")
        u = self.empty()
        for (off, cnt), a in zip(self.layouts, arrays):
            a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            assert a.size == cnt, (a.size, cnt)
            u[off:off + cnt].copy_(self.torch.from_numpy(a))
        return u

    def download(self, u):
        host = self._state(u).detach().cpu().numpy()
        return [host[off:off + cnt].reshape(p.E, p.m, p.nd).copy()
                for (off, cnt), p in zip(self.layouts, self.problems)]

    def cfl_dt(self, u):
        return ader_cfl_dt(self.ctx, self._state(u), self.nprob)

    def predictor(self, u, dt=None, qhat=False):
        """dt: None (context step) or a sequence of per-problem steps."""
        dt_dev = None
        if dt is not None:
            dt_dev = self.torch.tensor(self._per_problem(dt, "dt"), device="cuda")
        q = None
        if qhat:
            total = sum(ader_qhat_layout(self.ctx, p)[1] for p in range(self.nprob))
            q = self.torch.zeros(total, dtype=self.torch.float64, device="cuda")
        ader_predictor(self.ctx, self._state(u), dt_dev, q)
        self._dt_keep = dt_dev
        return q

    def qhat_views(self, q):
        host = q.detach().cpu().numpy()
        out = []
        for p, prob in enumerate(self.problems):
            off, cnt = ader_qhat_layout(self.ctx, p)
            out.append(host[off:off + cnt].reshape(prob.E, prob.m, prob.n, prob.nd).copy())
        return out

    def corrector(self, u, dt=None):
        dt_dev = None
        if dt is not None:
            dt_dev = self.torch.tensor(self._per_problem(dt, "dt"), device="cuda")
        ader_corrector(self.ctx, self._state(u), dt_dev)
        self._dt_keep = dt_dev

    def step(self, u, t_end):
        ader_step(self.ctx, self._state(u), self._per_problem(t_end, "t_end"))

    def run(self, u, t_end, nsteps):
        """nsteps steps replayed as one captured HIP graph."""
        ader_run(self.ctx, self._state(u), self._per_problem(t_end, "t_end"), nsteps)

    def set_detection(self, enable=True):
        ader_set_detection(self.ctx, enable)

    def detect_flags(self):
        """Troubled-element flags of the last step, one int32 array [E] per problem."""
        flat = ader_detect_flags(self.ctx, sum(p.E for p in self.problems))
        out, off = [], 0
        for p in self.problems:
            out.append(flat[off:off + p.E].copy())
            off += p.E
        return out

    def time(self):
        return ader_time(self.ctx, self.nprob)

    def set_time(self, t):
        ader_set_time(self.ctx, self._per_problem(t, "t"))

    def last_dt(self):
        return ader_last_dt(self.ctx, self.nprob)

    def totals(self, u):
        return ader_totals(self.ctx, self._state(u), self.nvars)

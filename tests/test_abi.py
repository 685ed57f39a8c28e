"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol that include/ader.h declares, rejects bad arguments before
touching a device, and its host tables obey the paper's identities."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1808_03788_amd import ader as A
from paper_1808_03788_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ader.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ader_status|const char \*)\s*(ader_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(A.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(A.EXPORTS)


def test_version():
    assert "gfx950" in A.ader_version()


@pytest.mark.parametrize("N", range(8))
def test_host_basis_identities(N):
    xi, w, D, T = A.ader_basis(N)
    n = N + 1
    z, wz = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(xi, 0.5 * (z + 1), atol=3e-15)
    np.testing.assert_allclose(w, 0.5 * wz, atol=3e-15)
    for p in range(n):
        np.testing.assert_allclose(D @ xi ** p, p * xi ** max(p - 1, 0) * (p > 0), atol=2e-11 * n * n)
    for p in range(N):
        np.testing.assert_allclose(T @ xi ** p, xi ** (p + 1) / (p + 1), atol=1e-13 * n * n)


def test_host_basis_matches_oracle(orc):
    for N in range(8):
        xi, w, D, T = A.ader_basis(N)
        o = orc.operators(N)
        np.testing.assert_allclose(xi, o["xi"], atol=3e-15)
        np.testing.assert_allclose(w, o["w"], atol=3e-15)
        np.testing.assert_allclose(D, o["Dhat"], atol=1e-12 * (N + 1) ** 3)
        np.testing.assert_allclose(T, o["T"], atol=1e-14 * (N + 1) ** 2)


def test_stability_alpha_matches_oracle_and_bound(orc):
    for N in range(8):
        a = A.ader_stability_alpha(N)
        assert a == orc.stability_alpha(N)
        assert a <= 1.0 / (2 * N + 1) + 1e-15
    with pytest.raises(A.AderError) as e:
        A.ader_stability_alpha(8)
    assert e.value.status == A.ADER_ERR_UNSUPPORTED


def _bad(**kw):
    p = I.density_wave_problem(nel=2, N=2)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,status", [
    (dict(dim=4), A.ADER_ERR_INVALID),
    (dict(N=-1), A.ADER_ERR_INVALID),
    (dict(N=8), A.ADER_ERR_UNSUPPORTED),
    (dict(nel=(0, 2, 2)), A.ADER_ERR_INVALID),
    (dict(hi=(1.0, -1.0, 1.0)), A.ADER_ERR_INVALID),
    (dict(gamma=1.0), A.ADER_ERR_INVALID),
    (dict(cfl=0.0), A.ADER_ERR_INVALID),
    (dict(cfl=1.5), A.ADER_ERR_INVALID),
    (dict(picard=-2), A.ADER_ERR_INVALID),
    (dict(guess=4), A.ADER_ERR_INVALID),
    (dict(guess=-1), A.ADER_ERR_INVALID),
])
def test_create_rejects_bad_arguments(kw, status):
    with pytest.raises(A.AderError) as e:
        A.ader_create([_bad(**kw)])
    assert e.value.status == status
    assert A.ader_last_error(None)


def test_create_rejects_bad_material():
    p = I.elastic_problem(nel=2, N=1)
    p.material = p.material.copy()
    p.material[3, 0] = -1.0
    with pytest.raises(A.AderError) as e:
        A.ader_create([p])
    assert e.value.status == A.ADER_ERR_INVALID
    assert "material" in A.ader_last_error(None)
    p2 = I.Problem(dim=2, N=1, nel=(2, 2, 1), lo=(0, 0, 0), hi=(1, 1, 1), pde="elastic")
    p2.material = np.ones((4, 3))
    with pytest.raises(A.AderError) as e:
        A.ader_create([p2])
    assert e.value.status == A.ADER_ERR_UNSUPPORTED


def test_null_arguments():
    L = A.lib()
    assert L.ader_destroy(None) == A.ADER_OK
    assert L.ader_create(None, 1, None, None) == A.ADER_ERR_INVALID
    out = ctypes.c_void_p()
    assert L.ader_create(None, 1, None, ctypes.byref(out)) == A.ADER_ERR_INVALID
    assert L.ader_cfl_dt(None, None, None) == A.ADER_ERR_INVALID
    assert L.ader_step(None, None, None) == A.ADER_ERR_INVALID
    assert L.ader_basis(-1, None, None, None, None) == A.ADER_ERR_INVALID


def test_product_path_does_not_use_oracle():
    """The binding and the library never reach the oracle."""
    src = open(os.path.join(ROOT, "paper_1808_03788_amd", "ader.py")).read()
    assert "oracle" not in src.replace("the oracle", "")
    csrc = os.path.join(ROOT, "paper_1808_03788_amd", "csrc")
    for f in os.listdir(csrc):
        assert "orc_" not in open(os.path.join(csrc, f)).read(), f


def test_binding_rejects_buffers_the_kernels_would_overrun():
    """The Python Context checks what the library trusts: the state tensor
    (float64, on the GPU, contiguous, at least state_size values) and one
    value per problem for t_end, dt and t (checked on the host, no GPU)."""
    import torch
    ctx = object.__new__(A.Context)  # the checks only, without a device context
    ctx.torch, ctx.nprob, ctx.size, ctx.ctx = torch, 2, 10, 0
    for bad in (torch.zeros(10, dtype=torch.float64),    # host memory
                torch.zeros(10, dtype=torch.float32),    # wrong type
                np.zeros(10)):                           # not a tensor
        with pytest.raises(ValueError):
            ctx._state(bad)
    for bad in ([1.0], [1.0, 2.0, 3.0], [[1.0, 2.0]]):
        with pytest.raises(ValueError):
            ctx._per_problem(bad, "t_end")
    assert list(ctx._per_problem(5.0, "t_end")) == [5.0, 5.0]
    assert list(ctx._per_problem([1, 2], "dt")) == [1.0, 2.0]
    with pytest.raises(ValueError):
        ctx.upload([np.zeros(1)])

"""The library's Q1 stencil rows (the header its diffusion and elliptic kernels
use), built as host C++, against the oracle's element-by-element assembly
(paper section 3.1: Q1 elements, lumped mass): every row applied to a random
field, the diagonal and the lumped mass, on 1D, 2D and 3D grids, degenerate
extents and anisotropic diagonal conductivities; a constant field gives
exactly zero (the difference form).  Bar: 1e-14 of the row scale."""
import ctypes
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

from oracle.diffusion import assemble

HERE = Path(__file__).resolve().parent
CSRC = HERE.parent / "paper_2510_27447_amd" / "csrc"


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    so = tmp_path_factory.mktemp("stencil") / "stencil_host.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", str(HERE / "host_stub"),
                    "-I", str(CSRC), "-o", str(so), str(HERE / "host_stub" / "stencil_host.cpp")],
                   check=True)
    return ctypes.CDLL(str(so))


def rows(lib, x, shape, sigma):
    n = x.size
    out, dg, ms = np.zeros(n), np.zeros(n), np.zeros(n)
    s = np.asarray(sigma, dtype=np.float64)
    P = ctypes.POINTER(ctypes.c_double)
    rc = lib.q1_rows(x.ctypes.data_as(P), *[ctypes.c_longlong(k) for k in shape],
                     s.ctypes.data_as(P), out.ctypes.data_as(P), dg.ctypes.data_as(P),
                     ms.ctypes.data_as(P))
    assert rc == 0
    return out, dg, ms


@pytest.mark.parametrize("shape", [(9, 8, 5), (13, 11, 1), (40, 1, 1), (1, 7, 1), (1, 1, 6),
                                   (3, 1, 4), (2, 2, 2), (1, 1, 1), (70, 3, 2)])
@pytest.mark.parametrize("sigma", [(1.0, 1.0, 1.0), (1.5e-3, 0.5e-3, 1.0e-3)])
def test_rows_match_assembly(lib, shape, sigma):
    h = 0.02
    d = sum(1 for k in shape if k > 1)
    n = int(np.prod(shape))
    x = np.random.default_rng(3).uniform(-85.0, 30.0, n)
    out, dg, ms = rows(lib, x, shape, sigma)
    A, _, ml = assemble(shape, h, sigma)
    want = (A @ x) / h ** (d - 2) if d else np.zeros(n)
    scale = np.abs(A).sum(axis=1).max() / h ** (d - 2) * np.abs(x).max() if d else 1.0
    assert np.max(np.abs(out - want)) <= 1e-14 * scale
    assert np.allclose(dg, A.diagonal() / h ** (d - 2) if d else 0.0, rtol=1e-15, atol=0.0)
    assert np.allclose(ms, ml / h ** d, rtol=1e-15, atol=0.0)
    const, _, _ = rows(lib, np.full(n, -85.123), shape, sigma)
    assert np.all(const == 0.0)

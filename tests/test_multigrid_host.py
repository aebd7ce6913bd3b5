"""The multigrid preconditioner's host planning (multigrid_plan.cpp), built as
host C++: the level extents; the fine level's 1D stiffness and mass rows
against the oracle's Q1 assembly of a 1D grid (paper section 3.1); the
prolongation reproducing constant and linear fields exactly; every coarser
level's rows equal to the Galerkin products P^T K P and P^T M P formed here
densely; the coarsest level's inverse against A_c + alpha 1 1^T assembled here
from its rows (alpha = trace / n^2).  The solve itself is checked on the GPU
against the oracle's direct solve (test_gpu_bidomain.py)."""
import ctypes
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

from oracle.diffusion import assemble

HERE = Path(__file__).resolve().parent
CSRC = HERE.parent / "paper_2510_27447_amd" / "csrc"
INCLUDE = HERE.parent / "include"


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    so = tmp_path_factory.mktemp("mg") / "mg_host.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC",
                    "-I", str(HERE / "host_stub"), "-I", str(CSRC), "-I", str(INCLUDE),
                    "-o", str(so), str(HERE / "host_stub" / "multigrid_host.cpp"),
                    str(CSRC / "multigrid_plan.cpp")], check=True)
    return ctypes.CDLL(str(so))


def plan(lib, shape):
    dims = np.zeros(48, dtype=np.int64)
    usable = ctypes.c_int()
    td = ctypes.c_longlong()
    L = lib.mg_host_plan(*[ctypes.c_longlong(n) for n in shape],
                         dims.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                         ctypes.byref(usable), ctypes.byref(td))
    return [tuple(int(v) for v in dims[3 * l:3 * l + 3]) for l in range(L)], bool(usable.value), td.value


def tables(lib, shape, s):
    levels, usable, td = plan(lib, shape)
    out = np.zeros(td)
    offs = np.zeros(9 * len(levels) + 1, dtype=np.int64)
    sv = np.asarray(s, dtype=np.float64)
    L = lib.mg_host_tables(*[ctypes.c_longlong(n) for n in shape],
                           sv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_longlong(td),
                           offs.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    assert L == len(levels)
    return levels, usable, out, offs


def tri(rows):
    n = rows.shape[0]
    T = np.diag(rows[:, 1])
    T += np.diag(rows[1:, 0], -1) + np.diag(rows[:-1, 2], 1)
    return T


def factors(levels, out, offs, l, a):
    n = levels[l][a]
    oK, oM, oP = offs[9 * l + 3 * a: 9 * l + 3 * a + 3]
    K = out[oK:oK + 3 * n].reshape(n, 3)
    M = out[oM:oM + 3 * n].reshape(n, 3)
    P = None
    if oP >= 0:
        nc = levels[l + 1][a]
        I0 = out[oP:oP + n].astype(int)
        w0, w1 = out[oP + n:oP + 2 * n], out[oP + 2 * n:oP + 3 * n]
        P = np.zeros((n, nc))
        for i in range(n):
            P[i, I0[i]] += w0[i]
            if w1[i] != 0.0:
                P[i, I0[i] + 1] += w1[i]
    return K, M, P


SHAPES = [(100, 100, 100), (30, 24, 10), (5000, 1, 1), (60, 50, 1), (2, 300, 1), (9, 8, 5)]


@pytest.mark.parametrize("shape", SHAPES)
def test_level_extents(lib, shape):
    levels, usable, _ = plan(lib, shape)
    assert levels[0] == shape
    for f, c in zip(levels, levels[1:]):
        for nf, nc in zip(f, c):
            assert nc == (nf if nf <= 2 else ((nf + 1) // 2 if nf % 2 else nf // 2 + 1))
        assert np.prod(f) > 512
    assert usable == (len(levels) >= 2 and np.prod(levels[-1]) <= 512)


@pytest.mark.parametrize("shape", SHAPES[:5])
def test_tables(lib, shape):
    s = (2.5e-3, 2.5e-3, 1.7e-3)
    levels, usable, out, offs = tables(lib, shape, s)
    assert usable
    for a in range(3):
        n = shape[a]
        K, M, _ = factors(levels, out, offs, 0, a)
        if n > 1:   # the oracle's 1D Q1 assembly with h = 1: stiffness and consistent mass
            A1, M1, _ = assemble((n, 1, 1), 1.0)
            assert np.allclose(tri(K), A1.toarray(), rtol=0, atol=1e-15)
            assert np.allclose(tri(M), M1.toarray(), rtol=0, atol=1e-15)
        else:
            assert np.all(K == 0) and np.array_equal(M, [[0.0, 1.0, 0.0]])
    for l in range(len(levels) - 1):
        for a in range(3):
            K, M, P = factors(levels, out, offs, l, a)
            Kc, Mc, _ = factors(levels, out, offs, l + 1, a)
            nf, nc = P.shape
            # exact for constants and for linear fields in the index
            pos = np.array([i if nc == nf else min(2 * i, nf - 1) for i in range(nc)], float)
            assert np.allclose(P @ np.ones(nc), 1.0, rtol=0, atol=1e-15)
            assert np.allclose(P @ pos, np.arange(nf), rtol=0, atol=1e-12)
            assert np.allclose(tri(Kc), P.T @ tri(K) @ P, rtol=0, atol=1e-12)
            assert np.allclose(tri(Mc), P.T @ tri(M) @ P, rtol=0, atol=1e-12)
    # the coarsest level's inverse
    Lc = len(levels) - 1
    F = [factors(levels, out, offs, Lc, a)[:2] for a in range(3)]
    kx, mx = tri(F[0][0]), tri(F[0][1])
    ky, my = tri(F[1][0]), tri(F[1][1])
    kz, mz = tri(F[2][0]), tri(F[2][1])
    Ac = (s[0] * np.kron(mz, np.kron(my, kx)) + s[1] * np.kron(mz, np.kron(ky, mx))
          + s[2] * np.kron(kz, np.kron(my, mx)))
    nc = Ac.shape[0]
    assert np.allclose(Ac @ np.ones(nc), 0.0, atol=1e-15)   # constants: the null space
    B = Ac + np.trace(Ac) / nc ** 2
    inv = out[offs[-1]:offs[-1] + nc * nc].reshape(nc, nc)
    assert np.allclose(inv @ B, np.eye(nc), rtol=0, atol=1e-10)
    assert np.allclose(inv, inv.T, rtol=0, atol=1e-12 * np.abs(inv).max())

"""The projection's multigrid hierarchy, built by the library's host code
(amg_build), checked on the CPU: conjugate gradients preconditioned by one of
its V-cycles solve the stiffness system of a graded channel with walls and of
the periodic square (singular: constants are its null space) to the exact
solution of a sparse direct solve, in a few tens of iterations where Jacobi
needs hundreds; the hierarchy coarsens.  The driver is compiled from
tests/amg_host_check.cpp and csrc/k_amg.hip with hipcc (host code only runs)."""
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import projection as PR
from synth import configs as CF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# the host code is built with AddressSanitizer and UndefinedBehaviorSanitizer
# (host pass only: the flags follow -Xarch_host); any report fails the run
HOST_SANITIZERS = "-g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all".split()


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("amg") / "amg_host_check"
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wno-unused-command-line-argument", *HOST_SANITIZERS, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "amg_host_check.cpp"),
           os.path.join(ROOT, "paper_1006_0720_amd", "csrc", "k_amg.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return str(out)


def _system(mesh, seed):
    K = PR.stiffness(mesh).tocsr()
    masters = np.nonzero(mesh.node_master == np.arange(mesh.n_nodes))[0]
    A = K[masters][:, masters].tocsr()
    A.sort_indices()
    b = np.random.default_rng(seed).standard_normal(A.shape[0])
    b -= b.mean()  # consistent with the null space
    return A, b


def _run(driver, tmp_path, A, b, tol2):
    fin, fout = tmp_path / "a.bin", tmp_path / "x.bin"
    with open(fin, "wb") as f:
        np.array([A.shape[0], A.nnz], np.int32).tofile(f)
        A.indptr.astype(np.int32).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
        b.astype(np.float64).tofile(f)
    r = subprocess.run([driver, str(fin), str(fout), repr(tol2)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    it = int(r.stdout.split("iterations")[1].split()[0])
    levels = [int(v) for v in r.stdout.split("levels")[1].split()]
    return it, levels, np.fromfile(fout, np.float64)


def _exact(A, b):
    n = A.shape[0]
    x = np.zeros(n)
    x[1:] = spla.spsolve(A[1:, 1:].tocsc(), b[1:])  # pin one unknown, then the zero-mean representative
    return x - x.mean()


def _jacobi_iterations(A, b, tol2):
    d = A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = r / d
    p = z.copy()
    rz = r @ z
    bb = rz
    for it in range(20000):
        if not rz > tol2 * bb:
            return it
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        z = r / d
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    return 20000


@pytest.mark.parametrize("make", [lambda: CF.channel(nx=60, n_half=25, ppe=1).mesh,
                                  lambda: CF.periodic_square(n=48, ppe=1).mesh],
                         ids=["graded_channel_walls", "periodic_square"])
def test_multigrid_pcg_solves_the_stiffness_system(driver, tmp_path, make):
    mesh = make()
    A, b = _system(mesh, seed=5)
    tol2 = 1e-24
    it, levels, x = _run(driver, tmp_path, A, b, tol2)
    assert len(levels) >= 2 and all(levels[i] > levels[i + 1] for i in range(len(levels) - 1)), levels
    assert levels[-1] <= 400
    xe = _exact(A, b)
    x = x - x.mean()
    assert np.abs(x - xe).max() <= 1e-9 * np.abs(xe).max()
    jit = _jacobi_iterations(A, b, tol2)
    print(f"[multigrid] n={A.shape[0]} levels={levels}: {it} iterations, Jacobi {jit}")
    assert it <= 60
    assert it * 4 <= jit

"""The elliptic relaxation's aggregation chain, built by the library's host
code (agg_chain), checked on the CPU by tests/agg_chain_check.cpp: the coarse
values that every solve forms as sums over the gather lists equal the
Galerkin product with the tentative prolongator, the coarse patterns hold all
its entries in sorted rows, and the member lists invert the aggregate map."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# the host code is built with AddressSanitizer and UndefinedBehaviorSanitizer
# (host pass only: the flags follow -Xarch_host); any report fails the run
HOST_SANITIZERS = "-g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all".split()


@pytest.mark.parametrize("n", [12, 40])
def test_aggregation_chain_gathers_the_galerkin_product(tmp_path, n):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path / "agg_chain_check"
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wno-unused-command-line-argument", *HOST_SANITIZERS, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "agg_chain_check.cpp"),
           os.path.join(ROOT, "paper_1006_0720_amd", "csrc", "k_amg.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(out), str(n)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr

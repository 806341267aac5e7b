"""Host eigensolver of the basis construction (Householder tridiagonalisation
+ implicit QL), built with g++ from the library's own source and checked on
Hermitian matrices of known spectrum: graded spectra and rank-deficient Gram
matrices whose null space forms a cluster at round-off level."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_2110_13115_amd", "csrc")


@pytest.fixture(scope="module")
def eig_check(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("eig") / "eig_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", SRC, os.path.join(HERE, "host", "eig_check.cpp"),
                    os.path.join(SRC, "linalg.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("n,lo,rank", [(120, -12, 120), (200, -30, 200), (300, -3, 40), (400, -8, 150),
                                       (256, -1, 1)])
def test_herm_eig_spectrum(eig_check, n, lo, rank):
    r = subprocess.run([eig_check, str(n), str(lo), str(rank)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout

"""The compile-time tables of the GPU path have the symmetry the predictor's
row projection relies on: the Gauss nodes on [-1/2, 1/2] are symmetric
(x[N-1-h] = -x[h], w[N-1-h] = w[h]) and the monic Legendre basis has the
parity of its degree, so the L2 projection weights satisfy
proj[a][N-1-h] = (-1)^a proj[a][h] exactly; the FP64 projection sums node
pairs (x_h + x_{N-1-h} for even a, x_h - x_{N-1-h} for odd a) on that basis.
Checked bitwise on the host: the table header is plain constexpr C++ and
compiles with g++ (CPU only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_13295_amd", "csrc")

SRC = r"""
#include <cstdio>
#include "hog_tables.h"
template <int P>
int check()
{
    constexpr hog::Rules<P> R{};
    constexpr int N = P + 1;
    int bad = 0;
    for (int h = 0; h < N; ++h) {
        bad += R.x[N - 1 - h] != -R.x[h];
        bad += R.w[N - 1 - h] != R.w[h];
        for (int a = 0; a <= P; ++a) {
            const double s = (a % 2) ? -1.0 : 1.0;
            bad += R.proj[a][N - 1 - h] != s * R.proj[a][h];
        }
    }
    if (N % 2 == 1)
        for (int a = 1; a <= P; a += 2) bad += R.proj[a][N / 2] != 0.0;
    std::printf("P=%d mismatches=%d\n", P, bad);
    return bad;
}
int main() { return check<1>() + check<2>() + check<3>(); }
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_projection_weights_have_the_parity_of_the_degree(tmp_path):
    src = tmp_path / "tables.cpp"
    src.write_text(SRC)
    exe = tmp_path / "tables"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("mismatches=0") == 3

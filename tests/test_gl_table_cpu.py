"""The Gauss-Legendre rules the device's storage bound reads (built at compile
time in csrc/sweeps.h) against numpy's rule: every size the bound uses, nodes
on [0, 1] and their weights.  A host program including the kernel header is
compiled with hipcc and prints the table; no GPU is used."""
import os
import shutil
import subprocess

import numpy as np
import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(REPO, "paper_1407_7370_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include "sweeps.h"
int main()
{
    for (int n = dl::kBoundMinNodes; n <= dl::kBoundNodes; ++n)
        for (int q = 0; q < n; ++q)
            std::printf("%d %d %.17g %.17g\n", n, q, dl::kGLRules.t[dl::gl_base(n) + q],
                        dl::kGLRules.w[dl::gl_base(n) + q]);
    return 0;
}
"""


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("gl")
    src, exe = d / "gl.hip", d / "gl"
    src.write_text(PROGRAM)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(REPO, "include"),
                    "-I", CSRC, str(src), "-o", str(exe)], check=True, capture_output=True, timeout=600)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout
    return np.array([[float(v) for v in line.split()] for line in out.splitlines()])


def test_every_rule_matches_numpy(table):
    sizes = sorted(set(int(n) for n in table[:, 0]))
    assert sizes == list(range(8, 49))
    for n in sizes:
        rows = table[table[:, 0] == n]
        x, w = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(rows[:, 2] - 0.5 * (x + 1.0))) <= 4e-16, n
        assert np.max(np.abs(rows[:, 3] - 0.5 * w) / (0.5 * w)) <= 1e-11, n
        # the rule integrates polynomials of degree 2n - 1 on [0, 1] exactly
        for deg in (0, n, 2 * n - 1):
            assert abs(np.dot(rows[:, 3], rows[:, 2] ** deg) - 1.0 / (deg + 1)) <= 1e-13, (n, deg)

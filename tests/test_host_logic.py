"""Host-side logic of the library checked on the CPU: the FGMRES stagnation rule (compiled
from the library's own header with g++; no HIP involved)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_08266_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "stall.hpp"
int main(int argc, char **argv)
{
    // argv: residual norms of consecutive restart cycles; prints the cycle index that stops
    int stalls = 0;
    double prev = -1.0;
    for (int i = 1; i < argc; ++i) {
        const double b = std::atof(argv[i]);
        if (fsi::krylov_stagnated(prev, b, stalls)) {
            std::printf("%d\n", i - 1);
            return 0;
        }
        prev = b;
    }
    std::printf("-1\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def stall_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("stall")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)], check=True)
    return str(exe)


def _stop(exe, seq):
    out = subprocess.run([exe, *[repr(float(v)) for v in seq]], capture_output=True, text=True, check=True)
    return int(out.stdout.strip())


def test_three_consecutive_stalls_stop(stall_exe):
    assert _stop(stall_exe, [1.0, 0.9995, 0.9991, 0.9989]) == 3


def test_progress_resets_the_stall_count(stall_exe):
    # slow cycles scattered through a long, converging solve never stop it
    seq = [1.0]
    for _ in range(20):
        seq += [seq[-1] * 0.9995, seq[-1] * 0.9995 * 0.5]
    assert _stop(stall_exe, seq) == -1
    # two stalls, progress, two stalls: still running; a third consecutive one stops it
    assert _stop(stall_exe, [1.0, 0.9999, 0.9998, 0.5, 0.49999, 0.49998]) == -1
    assert _stop(stall_exe, [1.0, 0.9999, 0.9998, 0.5, 0.49999, 0.49998, 0.49997]) == 6


def test_growth_counts_as_a_stall(stall_exe):
    assert _stop(stall_exe, [1.0, 2.0, 3.0, 4.0]) == 3

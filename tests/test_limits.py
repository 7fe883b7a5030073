"""Host-side size guards of the C-ABI library (csrc/limits.h), compiled on
their own with the host compiler: the upstream chain's pair total and its
neighbour-pair total are refused above 2^31 - 1, including totals that a
32-bit sum would wrap to a small value."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1005_5312_amd", "csrc")

PROGRAM = r"""
#include <stdio.h>
#include "limits.h"
int main(void)
{
    using start::upstream_pairs_fit;
    const unsigned long long cases[][2] = {
        {0ull, 1}, {1ull, 1}, {2147483647ull, 1}, {2147483648ull, 0}, {4294967295ull, 0},
        {4294967296ull + 5ull, 0},            /* wraps to 5 in 32 bits */
        {(1ull << 40), 0}, {~0ull, 0}};
    int bad = 0;
    for (unsigned k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k)
        if ((int)upstream_pairs_fit(cases[k][0]) != (int)cases[k][1]) {
            printf("wrong for %llu\n", cases[k][0]);
            bad = 1;
        }
    /* the list lengths are summed in 64 bits: 2^16 particles with 2^16 + 1
       entries each is refused */
    unsigned long long total = 0;
    for (int i = 0; i < 65536; ++i) total += 65537ull;
    if (upstream_pairs_fit(total) || (unsigned)total == total) { printf("sum\n"); bad = 1; }
    /* the neighbour pairs: the same limit */
    for (unsigned k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k)
        if ((int)start::neighbour_pairs_fit(cases[k][0]) != (int)cases[k][1]) {
            printf("neighbours: wrong for %llu\n", cases[k][0]);
            bad = 1;
        }
    return bad;
}
"""


def test_upstream_pair_guard(tmp_path):
    src = tmp_path / "limits_test.cpp"
    exe = tmp_path / "limits_test"
    src.write_text(PROGRAM)
    try:
        subprocess.run(["g++", "-std=c++17", "-Wall", "-I", CSRC, str(src), "-o", str(exe)], check=True,
                       capture_output=True, text=True)
    except FileNotFoundError:
        pytest.skip("no host C++ compiler")
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr

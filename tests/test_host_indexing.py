"""Host-side checks of the index arithmetic the 2D bandwidth kernels and the
on-chip FFT products rely on (no GPU): the division-free layout helpers of
mgwr_internal.h against the original ones, the block renumberings, and the
twelve-point form of the restriction of the implicit residual (Section 6:
full weighting; the residual after a red-black half-sweep lives at the
first colour only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1608_05400_amd", "csrc")

CHECK = r"""
#include "mgwr_internal.h"
#include <cstdio>
using namespace mgwr;
int main() {
    long bad = 0;
    for (int n : {1, 3, 7, 15, 31, 63, 127, 255, 511, 1023}) {
        const int P = n * n;
        for (int split = 0; split <= 1; ++split)
            for (int p = 0; p < P; ++p) {
                const int y = p / n, x = p % n;
                if (lay_pos_xy(n, split, x, y) != lay_pos(2, n, split, p)) ++bad;
                int xx, yy;
                lay_xy(n, split, lay_pos(2, n, split, p), xx, yy);
                if (xx != x || yy != y) ++bad;
            }
        for (int c = 0; c < 2; ++c)
            for (int j = 0; j < colour_count(2, n, c); ++j) {
                int x, y;
                colour_xy(n, c, j, x, y);
                if (y * n + x != colour_point(2, n, c, j)) ++bad;
            }
    }
    printf("%ld\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_layout_helpers_match_the_originals(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECK)
    exe = tmp_path / "check"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "0", out.stdout


@pytest.mark.parametrize("nb", [8, 16, 65536, 130568])
def test_block_renumberings_are_bijections(nb):
    lb = np.arange(nb)
    # k_fft_chip's pair of block lb, and k_group's per-XCD runs (nb a multiple of 8)
    q = (lb & 7) * (nb >> 3) + (lb >> 3)
    assert np.array_equal(np.sort(q), lb)
    # the blocks of one XCD (lb mod 8 equal) take one contiguous range
    for x in range(8):
        r = np.sort(q[lb % 8 == x])
        assert r[-1] - r[0] == len(r) - 1


def _implicit_restriction_five(B, n):
    """Full weighting of R, where R at first-colour points is the sum of the
    four second-colour neighbours of B (zero outside) and R is zero at the
    second colour: the centre and the four corners of every coarse point."""
    nc = (n - 1) // 2
    Bp = np.pad(B, 1)

    def R(y, x):
        return Bp[y, x + 1] + Bp[y + 2, x + 1] + Bp[y + 1, x] + Bp[y + 1, x + 2]

    out = np.zeros((nc, nc))
    for J in range(nc):
        for I in range(nc):
            x, y = 2 * I + 1, 2 * J + 1
            out[J, I] = (R(y - 1, x - 1) + R(y - 1, x + 1) + 4 * R(y, x) + R(y + 1, x - 1) + R(y + 1, x + 1)) / 16
    return out


def _implicit_restriction_twelve(B, n):
    nc = (n - 1) // 2
    Bp = np.pad(B, 2)
    at = lambda y, x: Bp[y + 2, x + 2]
    out = np.zeros((nc, nc))
    for J in range(nc):
        for I in range(nc):
            x, y = 2 * I + 1, 2 * J + 1
            inner = at(y - 1, x) + at(y + 1, x) + at(y, x - 1) + at(y, x + 1)
            outer = (at(y - 2, x - 1) + at(y - 2, x + 1) + at(y + 2, x - 1) + at(y + 2, x + 1)
                     + at(y - 1, x - 2) + at(y + 1, x - 2) + at(y - 1, x + 2) + at(y + 1, x + 2))
            out[J, I] = (6 * inner + outer) / 16
    return out


@pytest.mark.parametrize("n", [3, 7, 15, 31])
def test_implicit_restriction_twelve_point_form(n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    # only the second colour (x + y odd) carries values
    yy, xx = np.mgrid[0:n, 0:n]
    B[(xx + yy) % 2 == 0] = 0.0
    five = _implicit_restriction_five(B, n)
    twelve = _implicit_restriction_twelve(B, n)
    assert np.allclose(five, twelve, rtol=0, atol=1e-14 * np.abs(B).max())

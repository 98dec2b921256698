"""The propagator's sin(pi x), cos(pi x) (a reduced-argument Taylor evaluation, written
from the series of sin and cos) against long-double libm, on the host: the function is
compiled for the CPU from the kernels' header, so the device code's arithmetic is what
is checked.  The bound is a few units in the last place over random arguments in
[-4, 4], large ones up to 1e13, and the quarter points where the results are exact."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include <cmath>
#include <cstdio>
#include <random>
#include "kernels.h"
int main() {
    std::mt19937_64 g(2210);
    double worst = 0;
    auto check = [&](double x) {
        double s, c;
        eifp::sincospi_series(x, &s, &c);
        const long double pi = 3.14159265358979323846264338327950288L;
        const long double red = (long double)x - 2.0L * roundl((long double)x / 2.0L);  // exact
        const double es = (double)fabsl((long double)s - sinl(pi * red));
        const double ec = (double)fabsl((long double)c - cosl(pi * red));
        worst = fmax(worst, fmax(es, ec));
    };
    std::uniform_real_distribution<double> u(-4, 4), v(0, 1);
    for (int i = 0; i < 400000; ++i) check(u(g));
    for (int i = 0; i < 40000; ++i) check(v(g) * 1e7);
    for (int i = 0; i < 40000; ++i) check(-v(g) * 1e13);
    double s, c, s2, c2, s3, c3;
    eifp::sincospi_series(0.5, &s, &c);
    eifp::sincospi_series(-1.0, &s2, &c2);
    eifp::sincospi_series(0.25, &s3, &c3);
    printf("%.6e %.17g %.17g %.17g %.17g %.17g %.17g\n", worst, s, c, s2, c2, s3 - c3, s3);
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_series_sincospi_matches_long_double(tmp_path):
    src = tmp_path / "h.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "h"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2210_06232_amd", "csrc")]
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-host-only", *inc, str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120).stdout.split()
    worst, s, c, s2, c2, d3, s3 = map(float, out)
    assert worst <= 4 * 2.0 ** -53 * 2, worst       # a few units in the last place of values <= 1
    assert (s, c) == (1.0, 0.0) and (s2, c2) == (0.0, -1.0)   # quarter turns are exact
    assert abs(d3) <= 2.0 ** -53 and abs(s3 - 0.7071067811865476) <= 2.0 ** -53

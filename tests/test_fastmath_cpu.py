"""Host build of the float64 reciprocal / quotient / logarithm / square root used for the
objective terms (csrc/nmf_math.h), checked against the C library on random
arguments spanning the float64 range that quotients of float32 values reach.
On the GPU the same code starts from the hardware float32 reciprocal instead of
an exact float32 division; the objective parity tests cover that build."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2106_15214_amd", "csrc")

HARNESS = r"""
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>
#include "nmf_math.h"

static double ulps(double got, double ref) {
  if (got == ref) return 0.0;
  const double u = std::nextafter(std::fabs(ref), INFINITY) - std::fabs(ref);
  return std::fabs(got - ref) / u;
}

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> ex(-160.0, 160.0), unit(-1.0, 1.0);
  double worst_log = 0, worst_div = 0, worst_rcp = 0, worst_sqrt = 0, worst_rsq = 0;
  for (int i = 0; i < 2000000; ++i) {
    double x;
    if (i % 4 == 0) x = 1.0 + unit(rng) * std::ldexp(1.0, -(int)(i % 53));  // near 1
    else x = std::exp2(ex(rng)) * (1.0 + 0.5 * unit(rng));
    const double a = std::exp2(ex(rng) / 2) * (1.0 + 0.5 * unit(rng));
    worst_log = std::fmax(worst_log, ulps(nmf::log64(x), std::log(x)));
    if (std::fabs(std::log2(x)) < 120) {
      worst_rcp = std::fmax(worst_rcp, ulps(nmf::rcp64(x), 1.0 / x));
      worst_div = std::fmax(worst_div, ulps(nmf::div64(a, x), a / x));
      const double r = nmf::rsqrt64(x);
      worst_rsq = std::fmax(worst_rsq, ulps(r, 1.0 / std::sqrt(x)));
      worst_sqrt = std::fmax(worst_sqrt, ulps(nmf::sqrt64(x, r), std::sqrt(x)));
    }
  }
  std::printf("%.3f %.3f %.3f %.3f %.3f\n", worst_log, worst_div, worst_rcp, worst_sqrt, worst_rsq);
  return 0;
}
"""


def test_fast_log_div_rcp_match_libm(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "h.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "h"
    subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I" + CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    worst_log, worst_div, worst_rcp, worst_sqrt, worst_rsq = map(float, out)
    # a few units in the last place: far below what the 1e-6 objective gate needs
    assert worst_log <= 4.0, worst_log
    assert worst_div <= 1.0, worst_div
    assert worst_rcp <= 1.0, worst_rcp
    assert worst_sqrt <= 1.0, worst_sqrt
    assert worst_rsq <= 4.0, worst_rsq

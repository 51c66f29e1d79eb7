"""The device functions that replace library transcendentals in the FP64
normal and the Polya-Gamma sampler, compiled for the host and checked
against the x87 long-double library:

* log_open_unit (logarithm of an open uniform): within 2 ulp of the
  correctly rounded value over random open uniforms (the library's
  (m + 1/2) 2^-52 grid), every binade down to 2^-53, and the neighbourhoods
  of 1 and of the reduction's switch point sqrt(1/2);
* cos_2pi_unit (cos(2 pi u) for u in [0, 1]): within 4e-16 absolute over
  random uniforms and around the fold points k / 8;
* sin_2pi_unit (the sine branch of the paired normals): the same bound.

The FP64 draws' agreement with the oracle's library functions rests on
these bounds."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include "rng.hpp"
static double ulps(double v, long double ref)
{
    const double r = (double)ref;
    const double ulp = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    const long double d = (long double)v - ref;
    return (double)((d < 0 ? -d : d) / ulp);
}
int main()
{
    std::mt19937_64 g(7);
    double worst = 0.0;
    long n = 0;
    auto check = [&](double u) {
        const double e = ulps(gmrf::log_open_unit(u), logl((long double)u));
        worst = e > worst ? e : worst;
        ++n;
    };
    for (long i = 0; i < 2000000; ++i)
        check(((double)(g() >> 12) + 0.5) * 0x1p-52);
    for (int e = 1; e <= 53; ++e)
        for (int j = 0; j < 4000; ++j) {
            const double u = std::ldexp(1.0 + j / 4000.0, -e);
            if (u < 1.0 && u >= 0x1p-53)
                check(u);
        }
    for (long j = 0; j < 100000; ++j)
        check(1.0 - (j + 0.5) * 0x1p-52);
    for (long j = 0; j < 100000; ++j)
        check(0.70710678118654752440 + (j - 50000) * 0x1p-52);
    std::printf("%ld %.6f\n", n, worst);
    return 0;
}
"""


def test_log_open_unit_within_two_ulp(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "log_check.hip"
    exe = tmp_path / "log_check"
    src.write_text(PROGRAM)
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-host-only",
                    "-I", os.path.join(ROOT, "paper_1702_05518_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), "-x", "hip", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    n, worst = int(out[0]), float(out[1])
    assert n > 2_000_000
    assert worst <= 2.0, worst


COS_PROGRAM = r"""
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include "rng.hpp"
int main()
{
    std::mt19937_64 g(11);
    const long double pi = 3.141592653589793238462643383279502884L;
    double worst = 0.0;
    long n = 0;
    auto check = [&](double u) {
        const long double d = (long double)gmrf::cos_2pi_unit(u) - cosl(2.0L * pi * (long double)u);
        const double e = (double)(d < 0 ? -d : d);
        worst = e > worst ? e : worst;
        ++n;
    };
    for (long i = 0; i < 2000000; ++i)
        check(((double)(g() >> 12) + 0.5) * 0x1p-52);
    for (int k = 0; k <= 8; ++k)
        for (long j = -2000; j <= 2000; ++j) {
            const double u = k / 8.0 + j * 0x1p-52;
            if (u >= 0.0 && u <= 1.0)
                check(u);
        }
    std::printf("%ld %.6g\n", n, worst);
    return 0;
}
"""


def test_cos_2pi_unit_within_4e16(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "cos_check.hip"
    exe = tmp_path / "cos_check"
    src.write_text(COS_PROGRAM)
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-host-only",
                    "-I", os.path.join(ROOT, "paper_1702_05518_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), "-x", "hip", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    n, worst = int(out[0]), float(out[1])
    assert n > 2_000_000
    assert worst <= 4e-16, worst


SIN_PROGRAM = COS_PROGRAM.replace("gmrf::cos_2pi_unit(u)", "gmrf::sin_2pi_unit(u)").replace(
    "cosl(2.0L", "sinl(2.0L")


def test_sin_2pi_unit_within_4e16(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    assert "sin_2pi_unit" in SIN_PROGRAM and "sinl(" in SIN_PROGRAM
    src = tmp_path / "sin_check.hip"
    exe = tmp_path / "sin_check"
    src.write_text(SIN_PROGRAM)
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-host-only",
                    "-I", os.path.join(ROOT, "paper_1702_05518_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), "-x", "hip", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    n, worst = int(out[0]), float(out[1])
    assert n > 2_000_000
    assert worst <= 4e-16, worst

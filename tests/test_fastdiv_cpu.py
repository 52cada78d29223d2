"""The post-processing kernels' 32-bit division by invariant integers
(csrc/fastdiv.h) against exact division: every 32-bit numerator for a few
divisors, and for divisors 1..20000 and the extreme ones the numerators next
to multiples of d, the ends of the range and random draws."""
import shutil
import subprocess

import pytest

from paper_2503_18356_amd import build

CHECK = r"""
#include <cstdio>
#include <random>
#include "fastdiv.h"
int main() {
    using namespace rac;
    std::mt19937_64 rng(7);
    unsigned long long bad = 0;
    auto check = [&](uint32_t x, uint32_t d, const FastDiv& f) {
        if (fastdiv(x, f) != x / d && bad++ < 5) std::printf("x=%u d=%u\n", x, d);
    };
    for (uint32_t d = 1; d <= 20000; ++d) {
        const FastDiv f = make_fastdiv(d);
        for (uint32_t x : {0u, 1u, d - 1, d, d + 1, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu})
            check(x, d, f);
        for (int k = 0; k < 50; ++k) {
            const uint32_t x = (uint32_t)rng(), y = x - x % d;
            check(x, d, f);
            check(y, d, f);
            if (y) check(y - 1, d, f);
        }
    }
    for (uint32_t d : {0x80000000u, 0x80000001u, 0xfffffffeu, 0xffffffffu, 641u, 6700417u, 65537u}) {
        const FastDiv f = make_fastdiv(d);
        for (int k = 0; k < 200000; ++k) check((uint32_t)rng(), d, f);
    }
    for (uint32_t d : {10u, 100u}) {  // exhaustive
        const FastDiv f = make_fastdiv(d);
        for (uint64_t x = 0; x <= 0xffffffffull; ++x) check((uint32_t)x, d, f);
    }
    std::printf("bad %llu\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fastdiv_matches_exact_division(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECK)
    exe = tmp_path / "check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__host__=", "-D__device__=", "-I", build.CSRC,
                    str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr

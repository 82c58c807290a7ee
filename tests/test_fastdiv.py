"""The launch-time division constants of the kernels (fastdiv.h), on the CPU:
divu(make_divu32(d), n) == n / d for divisors 1..70000, every power of two and
its neighbours up to 2^32 - 1, and numerators at every edge (0, multiples of d
and their neighbours, 2^31 and 2^32 neighbours) plus seeded random ones."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2302_04741_amd",
                    "csrc")

PROGRAM = r"""
#include <stdio.h>
#include <stdint.h>
#include "fastdiv.h"

static uint64_t rng = 88172645463325252ull;
static uint32_t next32(void) { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return (uint32_t)rng; }

static int check(uint32_t d, uint32_t n)
{
    const lbm::DivU32 q = lbm::make_divu32(d);
    if (lbm::divu(q, n) != n / d) {
        printf("mismatch d=%u n=%u: %u vs %u\n", d, n, lbm::divu(q, n), n / d);
        return 1;
    }
    return 0;
}

static int sweep(uint32_t d)
{
    const uint32_t edge[] = {0u, 1u, 2u, d - 1u, d, d + 1u, 2u * d - 1u, 2u * d, 0x7fffffffu,
                             0x80000000u, 0x80000001u, 0xfffffffeu, 0xffffffffu};
    int bad = 0;
    for (uint32_t e : edge) bad |= check(d, e);
    const uint32_t top = 0xffffffffu / d;  // largest quotient
    bad |= check(d, top * d) | check(d, top * d - 1u) | check(d, top * d + (d - 1u));
    for (int k = 0; k < 24; ++k) bad |= check(d, next32());
    return bad;
}

int main(void)
{
    int bad = 0;
    for (uint32_t d = 1; d <= 70000u; ++d) bad |= sweep(d);
    for (int k = 1; k < 32; ++k) {
        const uint32_t p = 1u << k;
        bad |= sweep(p - 1u) | sweep(p) | sweep(p + 1u);
    }
    bad |= sweep(0xffffffffu) | sweep(0xfffffffeu) | sweep(0x80000001u);
    for (int k = 0; k < 20000; ++k) bad |= sweep(next32() | 1u);
    puts(bad ? "fastdiv: mismatches" : "fastdiv: all exact");
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_division_constants_exact(tmp_path):
    src = tmp_path / "fastdiv_check.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "fastdiv_check"
    # the header's functions carry HIP qualifiers; on the host they are plain
    cmd = ["g++", "-std=c++17", "-O2", "-D__host__=", "-D__device__=", "-I" + CSRC, str(src),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout[-2000:]
    assert "all exact" in run.stdout

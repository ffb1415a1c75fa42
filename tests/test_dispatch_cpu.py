"""CPU check of the fused kernels' workgroup placement: the XCD remap of
dispatch.h must be a bijection on [0, total) for every grid size and group
size, or a block would be computed twice and another not at all.  The header
is compiled for the host (its device qualifiers defined away) and checked
exhaustively on small grids and on the grid sizes of the throughput
configurations."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1510_04895_amd", "csrc")

DRIVER = r"""
#define __device__
#define __forceinline__ inline
#include "dispatch.h"
#include <cstdio>
#include <vector>
using chebfd::xcd_remap;
static int check(uint32_t total, int lg) {
    std::vector<char> seen(total, 0);
    for (uint32_t b = 0; b < total; ++b) {
        const uint32_t l = xcd_remap(b, total, lg);
        if (l >= total || seen[l]) return 1;
        seen[l] = 1;
        // 2^lg consecutive logical blocks of a full span share one XCD
        const uint32_t span = 8u << lg, full = total / span * span;
        if (lg > 0 && l < full && ((l >> lg) & 7u) != (b & 7u)) return 2;
    }
    return 0;
}
int main() {
    for (int lg = 0; lg <= 6; ++lg)
        for (uint32_t total = 1; total <= 3000; ++total)
            if (int e = check(total, lg)) { std::printf("fail total=%u lg=%d e=%d\n", total, lg, e); return 1; }
    // 64x64x32 SELL c128: 65536 row blocks x 8 slabs; matrix-free: 65536 x 8;
    // 128x128x64 z-march: 16 x-blocks x 128 y x 64 z x 8 slabs
    const uint32_t big[] = {524288u, 524288u + 77u, 1048576u};
    for (uint32_t t : big)
        for (int lg = 0; lg <= 6; ++lg)
            if (int e = check(t, lg)) { std::printf("fail total=%u lg=%d e=%d\n", t, lg, e); return 1; }
    std::printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_xcd_remap_is_a_bijection(tmp_path):
    inc = tmp_path / "inc" / "hip"
    inc.mkdir(parents=True)
    (inc / "hip_runtime.h").write_text("#pragma once\n")
    src = tmp_path / "remap.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "remap"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", str(tmp_path / "inc"), "-I", CSRC,
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip() == "ok"


def test_oracle_and_library_share_no_code():
    """The oracle and the HIP path are independent: no library source
    includes or names the oracle, no oracle source includes the library's
    headers or imports its package, and the product package never imports
    the oracle (only tests, the smoke check and the benchmark's CPU
    baseline do)."""
    pkg = os.path.join(ROOT, "paper_1510_04895_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if not f.endswith((".py", ".cpp", ".hip", ".h", ".c")):
                continue
            text = open(os.path.join(dp, f), encoding="utf-8").read()
            assert "import oracle" not in text and "from oracle" not in text, f
            assert "chebfd_oracle" not in text and "liboracle" not in text, f
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if not f.endswith((".py", ".c", ".h")):
            continue
        text = open(os.path.join(odir, f), encoding="utf-8").read()
        assert "import paper_1510_04895_amd" not in text, f
        assert "from paper_1510_04895_amd" not in text, f
        assert not re.search(r'#\s*include\s*[<"][^>"]*(chebfd|internal|pack|dispatch)\.h', text), f
        assert "libchebfd" not in text, f

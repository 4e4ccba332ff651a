"""The K ranges of the split moment contraction cover every angular cell
(host logic, CPU): the library's own chunk rule (csrc/ksplit.h) is compiled
with g++ and checked over every K split the plans can hold."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1903_08475_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <initializer_list>
#include "ksplit.h"
// kang: n_patches * n_ang padded to 128 (GEMM1's K); steps: 16 (FP64 K slab)
// and 32 (split-BF16 K slab); every split count up to kang / 64 (the most a
// plan's work space holds)
int main() {
    long long checked = 0;
    for (int kang = 128; kang <= 16 * 98304; kang += 128) {
        for (int step : {16, 32}) {
            for (int s = 1; s <= kang / 64; ++s) {
                const int c = mpg::ksplit_chunk(kang, s, step);
                if (c % step || c <= 0 || (long long)c * s < kang || c >= (kang + s - 1) / s + step) {
                    std::printf("FAIL kang %d step %d splits %d chunk %d\n", kang, step, s, c);
                    return 1;
                }
                ++checked;
            }
        }
        if (kang > 4 * 49152) kang += 128 * 7;  // sparser above the grids in use
    }
    std::printf("ok %lld\n", checked);
    return 0;
}
"""


def test_ksplit_chunks_cover_k():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "drv.cpp")
        exe = os.path.join(d, "drv")
        with open(src, "w") as f:
            f.write(DRIVER)
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True)
        r = subprocess.run([exe], stdout=subprocess.PIPE, text=True)
        assert r.returncode == 0, r.stdout
        assert r.stdout.startswith("ok")


def test_ksplit_known_case():
    """Yin-Yang at pi/256 (49152 cells per patch, padded to 128), FP64 K
    slab 16, 37 splits: the old rule gave 1328 cells per split and left the
    last 16 cells out; every split count now covers all of them."""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "one.cpp")
        exe = os.path.join(d, "one")
        with open(src, "w") as f:
            f.write('#include <cstdio>\n#include "ksplit.h"\nint main(){std::printf("%d", mpg::ksplit_chunk(49152, 37, 16));}\n')
        subprocess.run(["g++", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True)
        c = int(subprocess.run([exe], stdout=subprocess.PIPE, text=True).stdout)
        assert c * 37 >= 49152 and c % 16 == 0
        assert (49152 // 37 + 15) // 16 * 16 * 37 < 49152  # the old rule's shortfall

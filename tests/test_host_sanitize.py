"""The host-side tensor builder under AddressSanitizer and UndefinedBehaviorSanitizer:
tensor_build.cpp is compiled with g++ into a small driver that builds the tensors of
every kernel / fragment-law / order combination the library accepts (threads
included) and checks that each raw-flux row is finite.  Host code only; nothing here
touches a GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2607_13740_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include "tensor_build.h"
using namespace gd;
int main() {
    struct Case { int kernel, frag, bins, order, cons, levels; double xmin, xmax; };
    const Case cases[] = {
        {GD_KERNEL_CONST, GD_FRAG_NONE, 6, 2, 0, 1, 1e-3, 1e5},
        {GD_KERNEL_ADDITIVE, GD_FRAG_POWERLAW, 5, 3, 1, 1, 1e-4, 1e8},
        {GD_KERNEL_MULTIPLICATIVE, GD_FRAG_UNIFORM_BINARY, 4, 1, 0, 1, 1e-6, 1e3},
        {GD_KERNEL_BALLISTIC, GD_FRAG_REMNANT_ONLY, 5, 0, 1, 1, 1e-4, 1e8},
        {GD_KERNEL_BALLISTIC, GD_FRAG_POWERLAW, 5, 2, 1, 3, 1e-4, 1e8},
        {GD_KERNEL_MAXWELL, GD_FRAG_GENERAL, 6, 2, 1, 2, 1e-6, 1e3},
        {GD_KERNEL_BALLISTIC, GD_FRAG_GENERAL, 4, 4, 0, 1, 1e-4, 1e8},
    };
    int bad = 0;
    for (const Case& c : cases) {
        TensorSpec sp;
        sp.kernel = c.kernel; sp.frag = c.frag; sp.bins = c.bins; sp.order = c.order;
        sp.conservative = c.cons; sp.x_min = c.xmin; sp.x_max = c.xmax;
        sp.v0 = c.kernel == GD_KERNEL_MAXWELL ? 0.5 : 1.0; sp.v_bounce = 0.1; sp.alpha = -1.83;
        if (c.frag != GD_FRAG_NONE) { sp.levels.clear(); for (int l = 0; l < c.levels; ++l) sp.levels.push_back(0.4 + 0.3 * l); }
        HostTensor T;
        build_tensor(sp, T);
        for (double v : T.T) if (!std::isfinite(v)) { ++bad; break; }
        std::printf("kernel %d frag %d N %d k %d: %zu entries\n", c.kernel, c.frag, c.bins, c.order, T.T.size());
    }
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tensor_builder_under_sanitizers(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread", "-I", CSRC, str(src), os.path.join(CSRC, "tensor_build.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.count("entries") == 7

"""The checked build (libgracedg_checks.so: device-side bounds checks of work items,
iteration descriptors, fragment ranges and slot -> cell indices, and a flag for
non-finite stage outputs) against the regular build on the GPU.  The checks only
read indices and sizes, so on valid inputs every result must be bit for bit the
regular build's, with an empty check word; a state with a non-finite coefficient,
passed from the host, must raise the non-finite bit, and reading the word clears
it.  The checked build runs in a child process (GRACEDG_LIBRARY=checks), both runs
through tests/checked_build_run.py."""
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2607_13740_amd import gracedg as G  # noqa: E402

import checked_build_run as R  # noqa: E402

GD_CHECK_NONFINITE = 8


def test_checked_build_matches_regular_build(tmp_path):
    lib = os.path.join(os.path.dirname(G.LIB_PATH), "libgracedg_checks.so")
    assert os.path.exists(lib), "build it with `python -m paper_2607_13740_amd.build checks`"
    out_c = str(tmp_path / "checked.npz")
    env = dict(os.environ, GRACEDG_LIBRARY="checks")
    print("child: checked build", flush=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "checked_build_run.py"), out_c], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    out_r = str(tmp_path / "regular.npz")
    R.main(out_r)
    c, g = np.load(out_c), np.load(out_r)
    for prec in ("fp64", "mixed"):
        for name in ("raw", "L", "step", "advance", "clock"):
            a, b = c[f"{prec}_{name}"], g[f"{prec}_{name}"]
            assert np.all(np.isfinite(b)), (prec, name)
            assert np.array_equal(a, b), (prec, name, float(np.max(np.abs(a - b))))
        assert int(c[f"{prec}_checks"]) == 0, (prec, int(c[f"{prec}_checks"]))
        assert int(c[f"{prec}_checks_nonfinite"]) & GD_CHECK_NONFINITE, prec
        assert int(c[f"{prec}_checks_after_read"]) == 0, prec
        # the regular build has no device checks
        assert int(g[f"{prec}_checks_error"]) == G.GD_EUNSUPPORTED

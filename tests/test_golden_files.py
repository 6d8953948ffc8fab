"""The stored oracle results of the full-size workloads still belong to the
inputs the seeded generator makes, and are consistent in themselves (CPU).  The
512^3 file's sources are checked against the generator by the GPU test that
builds those inputs anyway (test_workload5_full_size_against_oracle)."""
import json
import os

import numpy as np

from paper_1711_06277_amd import inputs as I

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_workload4_fd_file_matches_inputs():
    """The central differences were taken on today's 128^3 adjoint workload
    (input sums equal to the stored ones), at relative steps 1e-3 of n_H and of
    min(x_n, 1 - x_n), and they agree with the oracle adjoint stored beside them
    (the generating script's own check, re-read here)."""
    with open(os.path.join(HERE, "workload4_fd.json")) as f:
        fd = json.load(f)
    wl = I.config(4)
    chk = fd["inputs_check"]
    assert float(wl.n_H.astype(np.float64).sum()) == chk["sum_n_H"]
    assert float(wl.x_n.astype(np.float64).sum()) == chk["sum_x_n"]
    assert float(wl.w.astype(np.float64).sum()) == chk["sum_w"]
    assert float(wl.v.astype(np.float64).sum()) == chk["sum_v"]
    cells = np.asarray(fd["cells"])
    assert cells.size == 64 and np.unique(cells).size == 64
    nH = wl.n_H.astype(np.float64)[cells]
    xn = wl.x_n.astype(np.float64)[cells]
    np.testing.assert_allclose(fd["step_n_H"], fd["h"] * nH, rtol=1e-15)
    np.testing.assert_allclose(fd["step_x_n"], fd["h"] * np.minimum(xn, 1.0 - xn), rtol=1e-15)
    for name in ("g_nH", "g_xn"):
        a = np.asarray(fd["fd_" + name])
        b = np.asarray(fd["oracle_" + name])
        assert np.all(np.abs(a - b) <= 1e-6 * np.abs(b)), name

"""Write ``workload4_fd.json``: central finite differences of the adjoint
workload's loss at 64 random cells, from the FP64 oracle's forward sweep.

The workload is the 128^3 lognormal field with a sigmoid neutral fraction,
8 sources and two bins; the loss is L = sum_c w_c rate_c + sum_c v_c . F_c with
the seeded weights.  For each chosen cell c the forward is run at
n_H(c) (1 +- h) and at x_n(c) +- h min(x_n(c), 1 - x_n(c)) with h = 1e-3 (the
second form keeps x_n inside [0, 1]), every other cell unchanged, and the
derivative is (L+ - L-) / (2 step).  The loss difference is summed cell by
cell from the two runs' outputs, so cells the perturbation does not reach add
exactly zero.  The oracle's own adjoint at the same cells is stored beside the
differences, and the script checks that the two agree.

Calls only the oracle (``oracle/``) and the seeded input generator; nothing
from the HIP path.  Run from the repository root (about ten minutes on 8 cores):

    python tests/golden/make_workload4_fd.py
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1711_06277_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload4_fd.json")
H = 1e-3
N_CELLS = 64
CELL_SEED = 4004

_WL = None  # the workload, inherited by the forked workers


def loss_difference(task):
    """(L+ - L-) for one cell and one field, and the step taken."""
    c, field = task
    wl = _WL
    kw = wl.params()
    nH = wl.n_H.astype(np.float64)
    xn = wl.x_n.astype(np.float64)
    if field == "n_H":
        step = H * nH[c]
    else:
        step = H * min(xn[c], 1.0 - xn[c])
    outs = []
    for sgn in (1.0, -1.0):
        a, b = nH.copy(), xn.copy()
        if field == "n_H":
            a[c] += sgn * step
        else:
            b[c] += sgn * step
        r = O.trace(wl.nx, wl.ny, wl.nz, a, b, wl.src_pos, wl.src_lum, **kw)
        outs.append((r.rate, r.force))
    (rp, fp), (rm, fm) = outs
    w = wl.w.astype(np.float64)
    v = wl.v.astype(np.float64).reshape(3, -1)
    dL = float(np.dot(w, rp - rm) + np.sum(v * (fp - fm)))
    return c, field, step, dL


def main():
    global _WL
    O.build(force=False)
    t0 = time.time()
    wl = I.config(4)
    _WL = wl
    N = wl.n_cells
    cells = np.sort(np.random.default_rng(CELL_SEED).choice(N, N_CELLS, replace=False))
    print(f"{wl.name}: {N_CELLS} cells, h = {H}", flush=True)
    tasks = [(int(c), f) for c in cells for f in ("n_H", "x_n")]
    workers = min(len(tasks), os.cpu_count() or 1, 16)
    with mp.get_context("fork").Pool(workers) as pool:
        res = {}
        for i, (c, f, step, dL) in enumerate(pool.imap_unordered(loss_difference, tasks)):
            res[(c, f)] = (step, dL)
            if (i + 1) % 16 == 0:
                print(f"  {i + 1}/{len(tasks)} differences, {time.time() - t0:.0f} s", flush=True)
    g_nH, g_xn = O.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum, wl.w, wl.v,
                           **wl.params())
    fd_nH = [res[(int(c), "n_H")][1] / (2 * res[(int(c), "n_H")][0]) for c in cells]
    fd_xn = [res[(int(c), "x_n")][1] / (2 * res[(int(c), "x_n")][0]) for c in cells]
    for name, fd, adj in (("dL/dn_H", fd_nH, g_nH[cells]), ("dL/dx_n", fd_xn, g_xn[cells])):
        fd = np.asarray(fd)
        err = np.abs(fd - adj) / np.maximum(np.abs(adj), 1e-300)
        print(f"{name}: FD vs oracle adjoint, max rel diff {err.max():.2e}, median {np.median(err):.2e}",
              flush=True)
        assert err.max() < 1e-4, (name, err.max())
    out = {"_source": "oracle/ (FP64) on the seeded 128^3 workload of paper_1711_06277_amd.inputs.config(4); "
                      "written by tests/golden/make_workload4_fd.py",
           "workload": wl.name, "h": H, "cell_seed": CELL_SEED,
           "inputs_check": {"sum_n_H": float(wl.n_H.astype(np.float64).sum()),
                            "sum_x_n": float(wl.x_n.astype(np.float64).sum()),
                            "sum_w": float(wl.w.astype(np.float64).sum()),
                            "sum_v": float(wl.v.astype(np.float64).sum())},
           "cells": [int(c) for c in cells],
           "step_n_H": [res[(int(c), "n_H")][0] for c in cells],
           "step_x_n": [res[(int(c), "x_n")][0] for c in cells],
           "fd_g_nH": fd_nH, "fd_g_xn": fd_xn,
           "oracle_g_nH": [float(x) for x in g_nH[cells]],
           "oracle_g_xn": [float(x) for x in g_xn[cells]],
           "max_abs_oracle_g_nH": float(np.abs(g_nH).max()),
           "max_abs_oracle_g_xn": float(np.abs(g_xn).max())}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

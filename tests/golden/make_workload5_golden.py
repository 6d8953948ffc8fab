"""Write ``workload5_sources.json``: the FP64 oracle's ray tree (rays created,
split, exited and terminated per level), escaped and residual luminosity per bin
and segment count of two sources of the 512^3 workload (1024 sources,
dN/dL ~ L^-2 on [1, 1e4], std-2 lognormal field, two bins): source 0 and the
brightest source.

Calls only the oracle (``oracle/``) and the seeded input generator; nothing from
the HIP path.  Run from the repository root:

    python tests/golden/make_workload5_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1711_06277_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload5_sources.json")


def main():
    O.build(force=False)
    t0 = time.time()
    wl = I.config(5)
    print(f"{wl.name}: inputs in {time.time() - t0:.0f} s", flush=True)
    picks = [0, int(np.argmax(wl.src_lum[:, 0]))]
    out = {"_source": "oracle/ (FP64) on the seeded 512^3 workload of paper_1711_06277_amd.inputs.config(5); "
                      "written by tests/golden/make_workload5_golden.py",
           "workload": wl.name, "sources": []}
    for s in picks:
        t1 = time.time()
        ref = O.trace_workload(wl.subset([s]))
        rec = {"index": s, "pos": wl.src_pos[s].tolist(), "lum": wl.src_lum[s].astype(float).tolist(),
               "segments": int(ref.segments[0]), "destroy": int(ref.destroy),
               "escaped": ref.escaped[0].tolist(), "residual": ref.residual[0].tolist(),
               "absorbed": ref.absorbed[0].tolist()}
        for key in ("created", "split", "exited", "terminated"):
            rec[key] = [int(x) for x in ref.__dict__[key][0]]
        out["sources"].append(rec)
        print(f"source {s}: {rec['segments']} segments in {time.time() - t1:.0f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()

"""The autotuner's result cache: JSON helpers on the CPU, a cache hit on the GPU."""
import json

import numpy as np
import pytest


def test_cache_helpers_round_trip(tmp_path):
    from paper_1711_06277_amd import api
    p = tmp_path / "sub" / "tune.json"
    assert api.autotune_cache_path(None) is None and api.autotune_cache_path(False) is None
    assert api.autotune_cache_path(str(p)) == str(p)
    assert api.load_autotune_cache(str(p)) == {}
    api.store_autotune_cache(str(p), "gpu|8x8x8|src1", (128, 6, 1.5))
    api.store_autotune_cache(str(p), "gpu|8x8x8|src2", (64, 16, 2.5))
    data = json.loads(p.read_text())
    assert data == {"gpu|8x8x8|src1": [128, 6, 1.5], "gpu|8x8x8|src2": [64, 16, 2.5]}
    p.write_text("not json")
    assert api.load_autotune_cache(str(p)) == {}


@pytest.mark.gpu
def test_cached_shape_is_applied(tmp_path):
    """A second autotune with the same key returns the stored shape without timing and
    the traces it then runs match those of the timed shape bit for bit."""
    import torch
    from paper_1711_06277_amd import inputs as I
    from paper_1711_06277_amd.api import ArtTracer
    wl = I.config(4, n_src=3, n=32)
    cache = tmp_path / "tune.json"
    args = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (wl.n_H, wl.x_n, wl.src_pos, wl.src_lum)]
    outs = []
    for k in range(2):
        tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins, max_sources=wl.n_src,
                       deterministic=True)
        try:
            res = tr.autotune(*args, cache=str(cache))
            outs.append((res, tr.trace(*args)[0].clone()))
        finally:
            tr.close()
    (b0, p0, ms0), r0 = outs[0]
    (b1, p1, ms1), r1 = outs[1]
    assert (b0, p0, ms0) == (b1, p1, ms1)
    assert list(json.loads(cache.read_text()).values()) == [[b0, p0, ms0]]
    assert torch.equal(r0, r1)

"""Source waves planned on the device: when the pool cannot hold every source's
tree at the geometric bound all sources share, each source's own bound (from its
position) packs the waves.  The bound must hold for every source (else the pool
would overflow), the plan must need fewer waves than the shared bound, and the
results must not depend on it (bitwise, fixed point)."""
import numpy as np
import pytest
import torch

from paper_1711_06277_amd import inputs as I
from tests.gpu_common import compare_cells

pytestmark = pytest.mark.gpu


def _problem(n=48, n_src=16, seed=3):
    wl = I.config(4, n_src=n_src, n=n)
    rng = np.random.default_rng(seed)
    pos = wl.src_pos.copy()
    # a few sources near corners, edges and faces, where the bound is tightest
    pos[0] = [0.3, 0.4, 0.2]
    pos[1] = [n - 0.3, n - 0.2, n - 0.4]
    pos[2] = [n / 2 + 0.1, 0.2, n / 2 - 0.3]
    pos[3] = [n / 2 + 0.13, n / 2 - 0.21, n / 2 + 0.07]
    pos[4:] += rng.uniform(-0.2, 0.2, pos[4:].shape)
    wl.src_pos = np.ascontiguousarray(np.clip(pos, 0.01, n - 0.01))
    return wl


def _run(wl, rot=None, **kw):
    from paper_1711_06277_amd.api import ArtTracer
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins, max_sources=wl.n_src,
                   deterministic=True, rot=rot, **kw)
    try:
        args = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (wl.n_H, wl.x_n, wl.src_pos, wl.src_lum)]
        out = [t.cpu().numpy() for t in tr.trace(*args, want_J=True)]
        st = tr.stats(wl.n_src)
    finally:
        tr.close()
    return out, st


@pytest.mark.parametrize("rotated", [False, True])
def test_device_planned_waves(rotated):
    wl = _problem()
    rot = None
    if rotated:
        from oracle import rotation as R
        rot = R.uniform_rotation([0.31, 0.72, 0.45])
    ref, st1 = _run(wl, rot=rot)
    assert st1.status == 0 and st1.n_waves == 1
    per_src = st1.src_created.sum(axis=1)
    # a pool that the shared geometric bound fills with one or two sources
    pool = int(per_src.max() * 2.5)
    got, st = _run(wl, rot=rot, pool_rays=pool)
    assert st.status == 0, f"device status {st.status}"
    assert np.all(st.src_rays_bound >= per_src), (st.src_rays_bound, per_src)
    assert np.all(st.src_rays_bound > 0)
    assert 1 < st.n_waves < wl.n_src
    print(f"\n{st.n_waves} waves; bound / rays per source: "
          f"{np.round(st.src_rays_bound / per_src, 2).tolist()}")
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    assert np.array_equal(st.src_created, st1.src_created)

"""The ionization subcycle on the GPU (paper Sec. 2.3) against the FP64 oracle
(oracle/ion.py): one substep from the same float32 state (substep size, Method B
update, momentum kick), the whole subcycle of the R-type front, graph capture,
and the degenerate cases."""
import math

import numpy as np
import pytest
import torch

from paper_1711_06277_amd import inputs as I

pytestmark = pytest.mark.gpu


def tracer(wl, **kw):
    from paper_1711_06277_amd.api import ArtTracer
    return ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                     level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                     tau_term=wl.tau_term, max_sources=max(1, wl.n_src), **kw)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return t if dtype is None else t.to(dtype)


def front_state(p, t):
    """The oracle's subcycle of the R-type problem up to time t, as float32."""
    from oracle import ion as X
    wl = p.wl
    res = X.subcycle(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum, alpha_B=p.alpha_B,
                     gamma_scale=p.gamma_scale, C=0.1, t_end=t,
                     trace_kw=dict(s_H=wl.s_H, s_d=wl.s_d, n_bins=1))
    return res.x_n.astype(np.float32)


def r_if(x):
    """Radius of the sphere with the volume of the cells with x_n < 0.5."""
    return (3.0 * float((x < 0.5).sum()) / (4.0 * math.pi)) ** (1.0 / 3.0)


@pytest.mark.parametrize("deterministic", [False, True])
def test_substep_matches_oracle(deterministic):
    """From the same state (a front inside the box): dt of Eq. e:dtss to 1e-5, x_n after
    Method B to 1e-5 absolute, the clock, and impulse = force dt."""
    from oracle import ion as X
    from oracle import oracle as O
    p = I.rtype_problem(32)
    wl = p.wl
    t0, t_end, C = 0.5, 4.0, 0.1
    x0 = front_state(p, t0)
    assert 0.05 < float((x0 < 0.5).mean()) < 0.5  # the front is inside the box
    ref = O.trace(wl.nx, wl.ny, wl.nz, wl.n_H, x0, wl.src_pos, wl.src_lum, s_H=wl.s_H, s_d=0.0, n_bins=1)
    G = X.gamma_from_J(ref.J[0], p.gamma_scale)
    dt_ref = min(X.substep_dt(wl.n_H, x0, G, p.alpha_B, C), t_end - t0)
    x_ref = X.method_b(x0, wl.n_H, G, p.alpha_B, dt_ref)

    tr = tracer(wl, deterministic=deterministic)
    try:
        x = dev(x0)
        t_now = torch.tensor([t0], dtype=torch.float64, device="cuda")
        imp = torch.zeros((3, wl.n_cells), dtype=torch.float32, device="cuda")
        rate, force, J = tr.ion_substep(dev(wl.n_H), x, dev(wl.src_pos), dev(wl.src_lum), alpha_B=p.alpha_B,
                                        gamma_scale=p.gamma_scale, C=C, t_end=t_end, t_now=t_now,
                                        impulse=imp)
        dt = float(t_now.item()) - t0
    finally:
        tr.close()
    assert dt == pytest.approx(dt_ref, rel=1e-5)
    xg = x.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(xg - x_ref)) < 1e-5
    assert np.max(np.abs(xg - x0)) <= C + 1e-6  # the substep rule bounds the change
    Fr = ref.force * dt_ref
    d = np.linalg.norm(imp.cpu().numpy().astype(np.float64) - Fr, axis=0)
    assert np.all(d <= 1e-4 * np.linalg.norm(Fr, axis=0) + 1e-6 * np.abs(Fr).max())
    np.testing.assert_allclose(J[0].cpu().numpy(), ref.J[0], rtol=1e-4, atol=1e-8 * ref.J[0].max())


def test_subcycle_matches_oracle_trajectory():
    """The whole subcycle of the R-type problem at 32^3 to t = 1 t_rec: the same number
    of substeps as the oracle, the same ionized volume, x_n close cell by cell."""
    from oracle import ion as X
    p = I.rtype_problem(32)
    wl = p.wl
    ref = X.subcycle(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum, alpha_B=p.alpha_B,
                     gamma_scale=p.gamma_scale, C=0.1, t_end=1.0,
                     trace_kw=dict(s_H=wl.s_H, s_d=0.0, n_bins=1))
    tr = tracer(wl, deterministic=True)
    try:
        x = dev(wl.x_n)
        k, t = tr.ion_subcycle(dev(wl.n_H), x, dev(wl.src_pos), dev(wl.src_lum), alpha_B=p.alpha_B,
                               gamma_scale=p.gamma_scale, C=0.1, t_end=1.0)
    finally:
        tr.close()
    assert t == 1.0
    assert abs(k - len(ref.dts)) <= 1
    xg = x.cpu().numpy().astype(np.float64)
    assert abs(r_if(xg) / r_if(ref.x_n) - 1) < 0.01
    assert np.mean(np.abs(xg - ref.x_n)) < 1e-3
    assert np.max(np.abs(xg - ref.x_n)) < 0.05


def test_rtype_front_128():
    """Sec. 3.3.1 at the paper's resolution (128^3, C = 0.1, Method B): the front
    follows R_S (1 - e^{-t/t_rec})^{1/3} within 5% and within 1% at 4 t_rec."""
    p = I.rtype_problem(128)
    wl = p.wl
    tr = tracer(wl, deterministic=True)
    nH, pos, lum = dev(wl.n_H), dev(wl.src_pos), dev(wl.src_lum)
    x = dev(wl.x_n)
    t_prev, total = 0.0, 0
    try:
        for m in (0.25, 0.5, 1.0, 2.0, 4.0):
            k, t = tr.ion_subcycle(nH, x, pos, lum, alpha_B=p.alpha_B, gamma_scale=p.gamma_scale, C=0.1,
                                   t_end=m - t_prev)
            assert t == pytest.approx(m - t_prev, rel=1e-12)
            total += k
            t_prev = m
            r = r_if(x.cpu().numpy())
            ref = p.R_S * (1.0 - math.exp(-m)) ** (1.0 / 3.0)
            print(f"t = {m}: {total} substeps, r_IF {r:.2f} analytic {ref:.2f} ({r / ref - 1:+.3f})", flush=True)
            assert abs(r / ref - 1) < 0.05
        assert abs(r / ref - 1) < 0.01
    finally:
        tr.close()


def test_substep_graph_replay_matches_eager():
    """Three substeps captured in one HIP graph and replayed equal three eager substeps
    bit for bit (fixed-point deposits), clock included."""
    p = I.rtype_problem(32)
    wl = p.wl
    x0 = front_state(p, 0.25)
    tr = tracer(wl, deterministic=True)
    try:
        nH, pos, lum = dev(wl.n_H), dev(wl.src_pos), dev(wl.src_lum)
        N = wl.n_cells
        out = (torch.empty(N, device="cuda"), torch.empty((3, N), device="cuda"), torch.empty((1, N), device="cuda"))
        x = dev(x0)
        t_now = torch.zeros(1, dtype=torch.float64, device="cuda")
        imp = torch.zeros((3, N), device="cuda")

        def steps():
            for _ in range(3):
                tr.ion_substep(nH, x, pos, lum, alpha_B=p.alpha_B, gamma_scale=p.gamma_scale, C=0.1,
                               t_end=4.0, t_now=t_now, out=out, impulse=imp, check=False)

        steps()
        torch.cuda.synchronize()
        assert tr.sync() == 0
        ref = (x.clone(), t_now.clone(), imp.clone())
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            x.copy_(dev(x0)); t_now.zero_(); imp.zero_()
            steps()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            steps()
        for rep in range(3):
            x.copy_(dev(x0))
            t_now.zero_()
            imp.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert tr.sync() == 0
            assert torch.equal(x, ref[0]) and torch.equal(t_now, ref[1]) and torch.equal(imp, ref[2]), rep
            (torch.randn(1 << 16, device="cuda") * 2).sum().item()  # eager work between replays
        del g
    finally:
        tr.close()


def test_substep_degenerate_cases():
    """t_now >= t_end: dt = 0 and nothing changes.  No source: pure recombination,
    Method B with Gamma = 0 (oracle).  Bad parameters are rejected."""
    from oracle import ion as X
    from paper_1711_06277_amd._abi import ArtError
    p = I.rtype_problem(16)
    wl = p.wl
    rng = np.random.default_rng(3)
    x0 = rng.uniform(0.0, 1.0, wl.n_cells).astype(np.float32)
    tr = tracer(wl)
    try:
        nH = dev(wl.n_H)
        x = dev(x0)
        t_now = torch.tensor([2.0], dtype=torch.float64, device="cuda")
        imp = torch.zeros((3, wl.n_cells), device="cuda")
        tr.ion_substep(nH, x, dev(wl.src_pos), dev(wl.src_lum), alpha_B=1.0, gamma_scale=p.gamma_scale,
                       C=0.1, t_end=2.0, t_now=t_now, impulse=imp)
        assert float(t_now.item()) == 2.0
        assert torch.equal(x, dev(x0)) and not imp.any()
        # no sources
        t_now.zero_()
        tr.ion_substep(nH, x, np.zeros((0, 3)), np.zeros((0, 1), dtype=np.float32), alpha_B=1.0,
                       gamma_scale=p.gamma_scale, C=0.1, t_end=10.0, t_now=t_now)
        dt_ref = X.substep_dt(wl.n_H, x0, np.zeros(wl.n_cells), 1.0, 0.1)
        assert float(t_now.item()) == pytest.approx(dt_ref, rel=1e-12)
        x_ref = X.method_b(x0, wl.n_H, 0.0, 1.0, dt_ref)
        assert np.max(np.abs(x.cpu().numpy() - x_ref)) < 1e-6
        with pytest.raises(ArtError):
            tr.ion_substep(nH, x, dev(wl.src_pos), dev(wl.src_lum), alpha_B=1.0, gamma_scale=1.0, C=0.0,
                           t_end=1.0, t_now=t_now)
        with pytest.raises(ArtError):
            tr.ion_substep(nH, x, dev(wl.src_pos), dev(wl.src_lum), alpha_B=-1.0, gamma_scale=1.0, C=0.1,
                           t_end=1.0, t_now=t_now)
    finally:
        tr.close()

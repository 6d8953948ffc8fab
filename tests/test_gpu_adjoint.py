"""GPU adjoint parity: dL/dn_H and dL/dx_n from the HIP reverse sweep against the
FP64 oracle adjoint (which is itself pinned by finite differences and the
tangent dot-product test on the CPU)."""
import numpy as np
import pytest

from paper_1711_06277_amd import inputs as I

pytestmark = pytest.mark.gpu


def adjoint_problem(n=32, n_src=3, seed=4, tau_term=I.TAU_TERM_1E10):
    wl = I.config(4, n_src=n_src, n=n)
    wl.tau_term = tau_term
    return wl


def gpu_adjoint(wl, deterministic=False, with_forward=True, expect_waves=False, **opts):
    import torch
    from paper_1711_06277_amd.api import ArtTracer
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                   tau_term=wl.tau_term, deterministic=deterministic,
                   max_sources=wl.n_src, enable_adjoint=True, **opts)
    try:
        d = "cuda"
        nH = torch.from_numpy(wl.n_H).to(d)
        xn = torch.from_numpy(wl.x_n).to(d)
        pos = torch.from_numpy(wl.src_pos).to(d)
        lum = torch.from_numpy(wl.src_lum).to(d)
        w = torch.from_numpy(wl.w).to(d)
        v = torch.from_numpy(wl.v).to(d)
        tape = None
        if with_forward:
            tr.trace(nH, xn, pos, lum)
            tape = tr.last_tape or None
        g_nH, g_xn = tr.adjoint(nH, xn, pos, lum, w, v, tape=tape)
        if expect_waves:
            assert tr.stats(wl.n_src).n_waves > 1
        return g_nH.cpu().numpy(), g_xn.cpu().numpy()
    finally:
        tr.close()


def compare_grad(name, gpu, ref, rel=1e-4, floor=1e-6):
    """Relative error on cells whose |gradient| exceeds floor * max |gradient|."""
    m = np.abs(ref) > floor * np.abs(ref).max()
    err = np.abs(gpu[m] - ref[m]) / np.abs(ref[m])
    assert err.max() <= rel, f"{name}: max rel err {err.max():.3e} over {m.sum()} cells"
    return float(err.max())


@pytest.mark.parametrize("with_forward", [True, False])
def test_adjoint_vs_oracle(oracle, with_forward):
    wl = adjoint_problem()
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    g_nH, g_xn = gpu_adjoint(wl, with_forward=with_forward)
    e1 = compare_grad("g_nH", g_nH, ref_nH)
    e2 = compare_grad("g_xn", g_xn, ref_xn)
    print(f"\nadjoint max rel err: g_nH {e1:.2e}, g_xn {e2:.2e}")


@pytest.mark.parametrize("level0", [0, 4])
@pytest.mark.parametrize("deterministic", [False, True], ids=["fp64_accumulator", "fixed_point"])
def test_adjoint_other_start_levels(oracle, level0, deterministic):
    """Start levels 0 (12 rays per source) and 4 (the paper's fiducial 768), both
    accumulator modes."""
    wl = adjoint_problem(n=28, n_src=2, seed=6)
    wl.level0 = level0
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    g_nH, g_xn = gpu_adjoint(wl, deterministic=deterministic)
    e1 = compare_grad("g_nH", g_nH, ref_nH)
    e2 = compare_grad("g_xn", g_xn, ref_xn)
    print(f"\nlevel0 {level0}: adjoint max rel err g_nH {e1:.2e}, g_xn {e2:.2e}")


@pytest.mark.parametrize("deterministic", [False, True], ids=["fp64_accumulator", "fixed_point"])
def test_adjoint_sources_on_corners_and_boundary(oracle, deterministic):
    """Sources on a cell corner (exact ties between faces) and on the domain's
    lower corner (half the rays start outside): the backward walk reproduces the
    forward's segments, ties and empty rays included."""
    wl = adjoint_problem(n=28, n_src=2)
    wl.src_pos = np.array([[14.0, 14.0, 14.0], [0.0, 0.0, 0.0]])
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    g_nH, g_xn = gpu_adjoint(wl, deterministic=deterministic)
    e1 = compare_grad("g_nH", g_nH, ref_nH)
    e2 = compare_grad("g_xn", g_xn, ref_xn)
    print(f"\ncorner sources: adjoint max rel err g_nH {e1:.2e}, g_xn {e2:.2e}")


def test_adjoint_with_terminations(oracle):
    wl = adjoint_problem(n=28, n_src=2, seed=7, tau_term=3.0)
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    g_nH, g_xn = gpu_adjoint(wl)
    compare_grad("g_nH", g_nH, ref_nH)
    compare_grad("g_xn", g_xn, ref_xn)


def test_adjoint_deterministic_bitwise(oracle):
    wl = adjoint_problem(n=24, n_src=2)
    a = gpu_adjoint(wl, deterministic=True)
    b = gpu_adjoint(wl, deterministic=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    compare_grad("g_nH", a[0], ref_nH)
    compare_grad("g_xn", a[1], ref_xn)


def test_adjoint_multiwave(oracle):
    """A pool that holds about one source's tree: the adjoint retraces and walks
    back one wave at a time (each wave's tree is gone once the next is seeded)."""
    wl = adjoint_problem(n=24, n_src=3)
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    g_nH, g_xn = gpu_adjoint(wl, pool_rays=32000, expect_waves=True)
    compare_grad("g_nH", g_nH, ref_nH)
    compare_grad("g_xn", g_xn, ref_xn)


def test_autograd_function(oracle):
    """torch.autograd through ArtTrace gives the adjoint of the weighted loss."""
    import torch
    from paper_1711_06277_amd.api import ArtTracer, art_trace
    wl = adjoint_problem(n=24, n_src=2)
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   max_sources=wl.n_src, enable_adjoint=True)
    try:
        nH = torch.from_numpy(wl.n_H).cuda().requires_grad_(True)
        xn = torch.from_numpy(wl.x_n).cuda().requires_grad_(True)
        rate, force = art_trace(nH, xn, tr, torch.from_numpy(wl.src_pos).cuda(),
                                torch.from_numpy(wl.src_lum).cuda())
        loss = (torch.from_numpy(wl.w).cuda() * rate).sum() + (torch.from_numpy(wl.v).cuda() * force).sum()
        loss.backward()
        ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos,
                                        wl.src_lum, wl.w, wl.v, **wl.params())
        compare_grad("g_nH", nH.grad.cpu().numpy(), ref_nH)
        compare_grad("g_xn", xn.grad.cpu().numpy(), ref_xn)
    finally:
        tr.close()


@pytest.mark.parametrize("deterministic,n_dense,n_thick", [(False, 3.0e38, 1.0e4), (True, 1.0e4, 1.0e4)])
def test_adjoint_through_opaque_cells(oracle, deterministic, n_dense, n_thick):
    """Cells of enormous opacity (n_H = 3e38: optical depths ~1e36 in one
    segment) next to thick ones (1e4): the transmission through them is 0 in
    FP64 on both sides, the walk back recovers the depth in front of them, and
    the gradients stay finite and match the oracle.  The fixed-point dL/dx_n is
    scaled by a bound that grows with the largest n_H, so that case stays at a
    density contrast of ~1e4 (blocks of n_H = 1e4 in a field of mean 1)."""
    wl = adjoint_problem(n=24, n_src=2, seed=11)
    nH = wl.n_H.reshape(24, 24, 24).copy()
    nH[10:13, 4:7, 4:7] = n_dense
    nH[4:6, 15:18, 12:14] = n_thick
    wl.n_H = np.ascontiguousarray(nH.reshape(-1))
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    assert np.isfinite(ref_nH).all() and np.isfinite(ref_xn).all()
    g_nH, g_xn = gpu_adjoint(wl, deterministic=deterministic)
    assert np.isfinite(g_nH).all() and np.isfinite(g_xn).all()
    compare_grad("g_nH", g_nH, ref_nH)
    compare_grad("g_xn", g_xn, ref_xn)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_repeated_adjoints_over_one_tape(oracle):
    """Several adjoints over the tree of one trace: the second with the same
    weights is bitwise equal to the first (fixed point), and one with other
    weights equals a fresh context's adjoint, which traces the tree again."""
    import torch
    from paper_1711_06277_amd.api import ArtTracer
    wl = adjoint_problem(n=28, n_src=3, seed=9)
    rng = np.random.default_rng(12)
    w2 = rng.uniform(-1, 1, wl.n_cells).astype(np.float32)
    v2 = rng.uniform(-1, 1, (3, wl.n_cells)).astype(np.float32)
    kw = dict(s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins, tau_term=wl.tau_term, deterministic=True,
              max_sources=wl.n_src, enable_adjoint=True)
    args = (_dev(wl.n_H), _dev(wl.x_n), _dev(wl.src_pos), _dev(wl.src_lum))
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, **kw)
    try:
        tr.trace(*args)
        tape = tr.last_tape
        assert tape != 0
        a1 = [t.clone() for t in tr.adjoint(*args, _dev(wl.w), _dev(wl.v), tape=tape)]
        a2 = [t.clone() for t in tr.adjoint(*args, _dev(wl.w), _dev(wl.v), tape=tape)]
        b1 = [t.clone() for t in tr.adjoint(*args, _dev(w2), _dev(v2), tape=tape)]
        assert torch.any(a1[0] != 0)
        for x, y in zip(a1, a2):
            assert torch.equal(x, y)
    finally:
        tr.close()
    fresh = ArtTracer(wl.nx, wl.ny, wl.nz, **kw)
    try:
        b2 = fresh.adjoint(*args, _dev(w2), _dev(v2))
        for x, y in zip(b1, b2):
            assert torch.equal(x, y)
    finally:
        fresh.close()
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    w2, v2, **wl.params())
    compare_grad("g_nH", b1[0].cpu().numpy(), ref_nH)
    compare_grad("g_xn", b1[1].cpu().numpy(), ref_xn)


def test_tape_is_refused_when_stale():
    """A tape token is refused (ART_ERR_NO_FORWARD) after any call that replaced
    the stored tree or changed what it depends on, for other input pointers, and
    is 0 for a trace split into several source waves."""
    from paper_1711_06277_amd import _abi as A
    from paper_1711_06277_amd.api import ArtTracer
    wl = adjoint_problem(n=24, n_src=2)
    args = (_dev(wl.n_H), _dev(wl.x_n), _dev(wl.src_pos), _dev(wl.src_lum))
    w, v = _dev(wl.w), _dev(wl.v)
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   max_sources=wl.n_src, enable_adjoint=True)
    try:
        tr.trace(*args)
        t1 = tr.last_tape
        tr.trace(*args)
        t2 = tr.last_tape
        assert t1 and t2 and t1 != t2
        with pytest.raises(A.ArtError) as e:  # an older trace's token
            A.art_trace_adjoint_tape(tr._ctx, t1, *(A.C.c_void_p(t.data_ptr()) for t in args), wl.n_src,
                                     A.C.c_void_p(w.data_ptr()), A.C.c_void_p(v.data_ptr()),
                                     A.C.c_void_p(w.data_ptr()), A.C.c_void_p(v.data_ptr()))
        assert e.value.code == A.ART_ERR_NO_FORWARD
        other = args[0].clone()  # same contents, another buffer
        with pytest.raises(A.ArtError) as e:
            out = (torch_empty(wl.n_cells), torch_empty(wl.n_cells))
            A.art_trace_adjoint_tape(tr._ctx, t2, A.C.c_void_p(other.data_ptr()),
                                     *(A.C.c_void_p(t.data_ptr()) for t in args[1:]), wl.n_src,
                                     A.C.c_void_p(w.data_ptr()), A.C.c_void_p(v.data_ptr()),
                                     A.C.c_void_p(out[0].data_ptr()), A.C.c_void_p(out[1].data_ptr()))
        assert e.value.code == A.ART_ERR_NO_FORWARD
        tr.adjoint(*args, w, v, tape=t2)  # still valid
        for invalidate in (lambda: tr.set_rotation(np.eye(3)), lambda: tr.set_transparent(None),
                           lambda: tr.adjoint(*args, w, v)):
            tr.trace(*args)
            t = tr.last_tape
            invalidate()
            assert A.art_get_tape(tr._ctx) == 0
            with pytest.raises(A.ArtError) as e:
                tr.adjoint(*args, w, v, tape=t)
            assert e.value.code == A.ART_ERR_NO_FORWARD
    finally:
        tr.close()
    tm = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   max_sources=wl.n_src, enable_adjoint=True, pool_rays=30000)
    try:
        tm.trace(*args)
        assert tm.stats(wl.n_src).n_waves > 1 and tm.last_tape == 0
    finally:
        tm.close()
    tn = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins, max_sources=wl.n_src)
    try:
        tn.trace(*args)
        assert tn.last_tape == 0
        with pytest.raises(A.ArtError) as e:
            tn.adjoint(*args, w, v)
        assert e.value.code == A.ART_ERR_NO_ADJOINT
    finally:
        tn.close()


def torch_empty(n):
    import torch
    return torch.empty(n, dtype=torch.float32, device="cuda")


def test_adjoint_after_ionization_substep(oracle):
    """An ionization substep traces x_n and then updates it in place: the tree it
    left belongs to the old x_n.  An adjoint afterwards on the same buffers traces
    the updated x_n (the substep leaves no tape), and equals a fresh context's
    adjoint (bitwise, fixed point) and the oracle adjoint of the updated x_n.
    The R-type setup at 32^3 with the density lowered 200-fold (4.4 -> 2.2 optical
    depths per cell length once ionized), so that the rays cross many cells and
    the gradients are not the rounding noise of cells that absorb everything."""
    import torch
    from paper_1711_06277_amd.api import ArtTracer
    p = I.rtype_problem(32)
    wl = p.wl
    wl.n_H = np.full(wl.n_cells, 0.005, dtype=np.float32)
    w, v = I.random_adjoint_weights(wl.n_cells, seed=31)
    nH, pos, lum = _dev(wl.n_H), _dev(wl.src_pos), _dev(wl.src_lum)
    x = _dev(wl.x_n)
    kw = dict(s_H=wl.s_H, s_d=wl.s_d, n_bins=1, max_sources=1, enable_adjoint=True, deterministic=True)
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, **kw)
    try:
        t_now = torch.zeros(1, dtype=torch.float64, device="cuda")
        tr.ion_substep(nH, x, pos, lum, alpha_B=p.alpha_B, gamma_scale=p.gamma_scale, C=0.1, t_end=10.0,
                       t_now=t_now)
        from paper_1711_06277_amd import _abi as A
        assert A.art_get_tape(tr._ctx) == 0
        x_new = x.cpu().numpy()
        assert not np.array_equal(x_new, wl.x_n)
        g = [t.cpu().numpy() for t in tr.adjoint(nH, x, pos, lum, _dev(w), _dev(v))]
    finally:
        tr.close()
    fresh = ArtTracer(wl.nx, wl.ny, wl.nz, **kw)
    try:
        gf = [t.cpu().numpy() for t in fresh.adjoint(nH, _dev(x_new), pos, lum, _dev(w), _dev(v))]
    finally:
        fresh.close()
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, x_new, wl.src_pos, wl.src_lum, w, v,
                                    s_H=wl.s_H, s_d=wl.s_d, n_bins=1)
    assert np.array_equal(g[0], gf[0]) and np.array_equal(g[1], gf[1])
    compare_grad("g_nH", g[0], ref_nH)
    compare_grad("g_xn", g[1], ref_xn)


def test_adjoint_of_host_arrays_traces_their_contents(oracle):
    """Host arrays are copied to temporary device buffers per call, which can land
    on the addresses of an earlier call's temporaries: an adjoint of host arrays
    whose contents differ from the preceding trace's is the adjoint of those
    contents (the tree is traced again, never taken from the pool by address)."""
    from paper_1711_06277_amd.api import ArtTracer
    wl = adjoint_problem(n=24, n_src=2, seed=5)
    x2 = np.clip(wl.x_n * np.float32(0.5), 0, 1).astype(np.float32)
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   max_sources=wl.n_src, enable_adjoint=True)
    try:
        tr.trace(wl.n_H, wl.x_n, wl.src_pos, wl.src_lum)
        g_nH, g_xn = tr.adjoint(wl.n_H, x2, wl.src_pos, wl.src_lum, wl.w, wl.v)
        g_nH, g_xn = g_nH.cpu().numpy(), g_xn.cpu().numpy()
    finally:
        tr.close()
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, x2, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    compare_grad("g_nH", g_nH, ref_nH)
    compare_grad("g_xn", g_xn, ref_xn)


def test_autograd_backward_twice(oracle):
    """backward(retain_graph=True) twice over one forward gives the same gradient
    twice (the stored tree is walked again with cleared claim counters)."""
    import torch
    from paper_1711_06277_amd.api import ArtTracer, art_trace
    wl = adjoint_problem(n=24, n_src=2, seed=6)
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   max_sources=wl.n_src, enable_adjoint=True, deterministic=True)
    try:
        nH = _dev(wl.n_H).requires_grad_(True)
        xn = _dev(wl.x_n).requires_grad_(True)
        rate, force = art_trace(nH, xn, tr, _dev(wl.src_pos), _dev(wl.src_lum))
        loss = (_dev(wl.w) * rate).sum() + (_dev(wl.v) * force).sum()
        loss.backward(retain_graph=True)
        g1 = (nH.grad.clone(), xn.grad.clone())
        nH.grad = None
        xn.grad = None
        loss.backward()
        assert torch.equal(nH.grad, g1[0]) and torch.equal(xn.grad, g1[1])
        assert torch.any(g1[0] != 0)
    finally:
        tr.close()
    ref_nH, ref_xn = oracle.adjoint(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                                    wl.w, wl.v, **wl.params())
    compare_grad("g_nH", g1[0].cpu().numpy(), ref_nH)
    compare_grad("g_xn", g1[1].cpu().numpy(), ref_xn)

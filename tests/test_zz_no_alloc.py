"""art_trace_noalloc (the forward sweep on the library's static workspace, for
callers that cannot allocate) against art_trace on the same inputs: bitwise in
fixed point, to the parity bar with FP32 atomics, on two calls in a row, the
second on a smaller grid with fewer sources (the workspace keeps the first
call's contents, so whatever must start at zero has to be cleared)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1711_06277_amd import _abi as A
from paper_1711_06277_amd import inputs as I
from tests.gpu_common import compare_cells

pytestmark = pytest.mark.gpu


def _problem(n, n_src, seed):
    wl = I.config(4, n_src=n_src, n=n)
    rng = np.random.default_rng(seed)
    wl.src_pos = np.ascontiguousarray(wl.src_pos + rng.uniform(-0.1, 0.1, wl.src_pos.shape))
    return wl


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _noalloc(wl, deterministic, want_J):
    from paper_1711_06277_amd.api import ArtTracer
    # the parameters exactly as ArtTracer builds them
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins, deterministic=deterministic,
                   max_sources=wl.n_src)
    try:
        args = (_dev(wl.n_H), _dev(wl.x_n), _dev(wl.src_pos), _dev(wl.src_lum))
        ref = [t.clone() for t in tr.trace(*args, want_J=want_J)]
        params = tr.params
    finally:
        tr.close()
    N = wl.n_cells
    rate = torch.full((N,), -1.0, device="cuda")
    force = torch.full((3, N), -1.0, device="cuda")
    J = torch.full((wl.n_bins, N), -1.0, device="cuda") if want_J else None
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    p = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    A.art_trace_noalloc(wl.nx, wl.ny, wl.nz, params, *(p(t) for t in args), wl.n_src, p(rate), p(force), p(J),
                        p(status), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(status.item()) == A.ART_OK
    got = [rate, force] + ([J] if want_J else [])
    return ref, got


@pytest.mark.parametrize("deterministic", [True, False], ids=["fixed_point", "fp32_atomic"])
def test_noalloc_matches_art_trace(deterministic):
    for k, (n, n_src, want_J) in enumerate(((36, 4, True), (20, 2, False))):
        wl = _problem(n, n_src, seed=k)
        ref, got = _noalloc(wl, deterministic, want_J)
        if deterministic:
            for a, b in zip(ref, got):
                assert torch.equal(a, b), f"call {k}"
        else:
            # FP32 atomics add in a different order on every run
            L = float(wl.src_lum.astype(np.float64).sum())
            compare_cells(f"call {k} rate", got[0].cpu().numpy(), ref[0].cpu().numpy().astype(np.float64), L)
            d = (got[1] - ref[1]).norm(dim=0)
            f = ref[1].norm(dim=0)
            assert bool((d <= 1e-4 * f + 1e-6 * float(f.max())).all()), f"call {k} force"
            if want_J:
                for b in range(wl.n_bins):
                    compare_cells(f"call {k} J{b}", got[2][b].cpu().numpy(),
                                  ref[2][b].cpu().numpy().astype(np.float64), L)


def test_noalloc_reports_device_errors():
    """A source outside the domain is reported through the status int."""
    wl = _problem(20, 2, seed=3)
    wl.src_pos = wl.src_pos.copy()
    wl.src_pos[1, 0] = wl.nx + 2.0
    from paper_1711_06277_amd.api import ArtTracer
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins, max_sources=wl.n_src)
    params = tr.params
    tr.close()
    N = wl.n_cells
    bufs = [_dev(wl.n_H), _dev(wl.x_n), _dev(wl.src_pos), _dev(wl.src_lum)]
    rate = torch.empty(N, device="cuda")
    force = torch.empty((3, N), device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    A.art_trace_noalloc(wl.nx, wl.ny, wl.nz, params, *(p(t) for t in bufs), wl.n_src, p(rate), p(force), None,
                        p(status), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(status.item()) == A.ART_ERR_SOURCE_OUTSIDE

"""Helpers shared by the GPU parity tests (HIP path through the C ABI vs the
FP64 oracle on the same seeded inputs)."""
from __future__ import annotations

import numpy as np

# Acceptance bar for FP32 cell outputs: relative error 1e-4 on cells whose
# oracle value exceeds 1e-8 of the batch luminosity; photon conservation 1e-6.
REL_TOL = 1e-4
CELL_FLOOR = 1e-8
CONS_TOL = 1e-6


def run_gpu(wl, want_J=True, deterministic=None, **opts):
    """Trace a Workload on cuda:0 through the C ABI; numpy outputs + stats."""
    import torch
    from paper_1711_06277_amd.api import ArtTracer

    det = wl.deterministic if deterministic is None else deterministic
    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                   tau_term=wl.tau_term, deterministic=det,
                   max_sources=max(1, wl.n_src), **opts)
    try:
        out = tr.trace(torch.from_numpy(wl.n_H), torch.from_numpy(wl.x_n),
                       torch.from_numpy(wl.src_pos), torch.from_numpy(wl.src_lum), want_J=want_J)
        torch.cuda.synchronize()
        st = tr.stats(wl.n_src)
        res = [o.cpu().numpy() for o in out]
    finally:
        tr.close()
    return res, st


def kappas(wl):
    nH = wl.n_H.astype(np.float64)
    xn = wl.x_n.astype(np.float64)
    return [nH * (xn * wl.s_H + wl.s_d), nH * wl.s_d][: wl.n_bins]


def compare_cells(name, gpu, ref, L_tot, rel=REL_TOL, floor=CELL_FLOOR):
    """Relative error on cells where |ref| > floor * L_tot (scalar fields)."""
    ref = np.asarray(ref, dtype=np.float64)
    gpu = np.asarray(gpu, dtype=np.float64)
    m = np.abs(ref) > floor * L_tot
    assert m.any(), f"{name}: no cell above threshold"
    err = np.abs(gpu[m] - ref[m]) / np.abs(ref[m])
    worst = int(np.argmax(err))
    assert err.max() <= rel, (f"{name}: max rel err {err.max():.3e} at cell "
                              f"{np.flatnonzero(m)[worst]} ({m.sum()} cells compared)")
    # cells below the floor must still be tiny on the GPU side
    assert np.abs(gpu[~m]).max(initial=0.0) <= 10 * floor * L_tot + 1e-30, f"{name}: spurious deposit"
    return float(err.max())


# Cells whose net force is below this fraction of the summed magnitudes
# sum_b kappa_b J_b >= sum |Delta L n| (rays from opposite sides cancel, e.g.
# around a source): the FP32 rounding of each deposit, ~1e-7 relative, then sums
# to ~1e-7 kappa J, which is 1e-4 of |F| only where |F| >= 1e-3 kappa J.
CANCEL = 1e-3


def compare_force(gpu_F, ref_F, L_tot, kj_ref, rel=REL_TOL, floor=CELL_FLOOR, name="force"):
    """|dF| / |F| <= rel on every cell with |F| above the floor, except the
    counted cancellation cells (|F| < CANCEL kappa J), which are held to
    |dF| <= rel kappa J instead.  Returns (max |dF|/|F| over the other cells,
    number of cancellation cells, max |dF| / (kappa J) over them)."""
    ref = np.asarray(ref_F, dtype=np.float64)
    gpu = np.asarray(gpu_F, dtype=np.float64)
    kj = np.asarray(kj_ref, dtype=np.float64)
    fmag = np.linalg.norm(ref, axis=0)
    d = np.linalg.norm(gpu - ref, axis=0)
    m = fmag > floor * L_tot
    assert m.any(), f"{name}: no cell above threshold"
    cancel = m & (fmag < CANCEL * kj)
    plain = m & ~cancel
    err_rel = d[plain] / fmag[plain]
    err_c = d[cancel] / kj[cancel]
    worst = float(err_rel.max(initial=0.0))
    worst_c = float(err_c.max(initial=0.0))
    print(f"\n{name}: {plain.sum()} cells at |dF|/|F| <= {worst:.2e}; {cancel.sum()} cancellation "
          f"cells (|F| < {CANCEL:g} kappa J) at |dF|/(kappa J) <= {worst_c:.2e}")
    assert worst <= rel, f"{name}: max |dF|/|F| {worst:.3e} over {plain.sum()} cells"
    assert worst_c <= rel, f"{name}: max |dF|/(kappa J) {worst_c:.3e} over {cancel.sum()} cancellation cells"
    # gpu cells below the floor stay tiny
    assert d[~m].max(initial=0.0) <= 10 * floor * L_tot + 1e-30, f"{name}: spurious deposit"
    return worst, int(cancel.sum()), worst_c


def conservation(wl, J_gpu, st):
    """Per-bin relative imbalance |sum_c kappa_b J_b + escaped + residual - emitted| / emitted."""
    ks = kappas(wl)
    out = []
    for b in range(wl.n_bins):
        absorbed = float((ks[b] * J_gpu[b].astype(np.float64)).sum())
        emitted = float(wl.src_lum[:, b].astype(np.float64).sum())
        esc = float(st.src_escaped[:, b].sum())
        resid = float(st.src_residual[:, b].sum())
        out.append(abs(absorbed + esc + resid - emitted) / emitted)
    return out


def tree_equal(st, ref, n_src=None):
    """Bit-exact ray tree per source and level (created / split / exited / terminated)."""
    n = ref.created.shape[0] if n_src is None else n_src
    for key, mine in (("created", st.src_created), ("split", st.src_split),
                      ("exited", st.src_exited), ("terminated", st.src_terminated)):
        theirs = ref.__dict__[key][:n]
        assert np.array_equal(mine[:n], theirs), f"tree mismatch in {key}:\n{mine[:n]}\n{theirs}"

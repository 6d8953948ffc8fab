"""Benchmark of the ART sweep on one MI355X.

A step is one full batched forward trace (seed, every level's sweep, finalize)
of the 256^3 lognormal workload with 64 sources of log-uniform luminosity and
two frequency bins, inputs resident in HBM.  Prints ONE JSON line with
segments/s (whole job), ms per full trace per source, the plain (one source
per call) comparison, the roofline of the sweep kernel and the FP64 oracle's
rate on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload 3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# algorithmic bytes per ray-cell segment: the (n_H, x_n) gather (8 B) and a
# read-modify-write of the cell's four FP32 outputs (J_i, F_x, F_y, F_z).  The
# fixed-point mode's 8-byte accumulators would count 72 B; the roofline uses the
# method's 40 B in both modes.
BYTES_PER_SEGMENT = 40
BYTES_PER_SEGMENT_FIXED_POINT = 72
# the adjoint walks every segment once (backwards): it gathers (n_H, x_n, w, v)
# (24 B) and adds dL/dn_H and dL/dx_n to two FP64 cells (2 x 16 B RMW)
ADJOINT_BYTES_PER_SEGMENT = 56


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha() -> str:
    """Hash of the kernel sources' code: comments and blank space are dropped, so
    a comment edit keeps the committed counter summaries valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("paper_1711_06277_amd/csrc/art.hip", "paper_1711_06277_amd/csrc/art_device.h"):
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _summary_value(name: str, key: str):
    """A value of a committed rocprofv3 summary, or None if the summary is missing
    or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in (key, "kernel_sources_sha"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha") != kernel_sources_sha() or key not in vals:
        return None
    return float(vals[key])


def measured_traffic(workload: int, deterministic: bool):
    """HBM bytes per trace of the forward sweep from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None if the kernel has
    changed since."""
    if workload != 3:
        return None
    name = "k_sweep_c3_traffic.md" if deterministic else "k_sweep_c3_atomic_traffic.md"
    return _summary_value(name, "traffic_bytes_per_trace")


def measured_adjoint_traffic(workload: int, deterministic: bool):
    """HBM bytes per adjoint sweep, likewise (profiled in the fixed-point mode)."""
    if workload != 3 or not deterministic:
        return None
    return _summary_value("k_adjoint_c3_traffic.md", "traffic_bytes_per_adjoint")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true", help="skip the one-source-per-call timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint sweep timing")
    ap.add_argument("--no-ion", action="store_true", help="skip the ionization-subcycle timing")
    ap.add_argument("--graph", action="store_true",
                    help="also time forward + adjoint captured in one HIP graph (adjoint leg)")
    ap.add_argument("--atomic", action="store_true",
                    help="FP32 atomic deposits instead of the (faster) 64-bit fixed-point ones")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the sweep's launch shape with art_autotune before timing")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the sweep is not "
              "sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1711_06277_amd import inputs as I
    from paper_1711_06277_amd.api import ArtTracer

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.device("cuda:0")

    t0 = time.time()
    wl = I.config(args.workload)
    # 64-bit fixed-point deposits: integer LDS and global atomics are faster than
    # FP32 ones on this GPU, and the sums are bitwise reproducible
    wl.deterministic = not args.atomic
    log(f"[bench] workload {wl.name}: generated in {time.time() - t0:.1f}s")

    tr = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                   level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                   tau_term=wl.tau_term, deterministic=wl.deterministic,
                   max_sources=wl.n_src, block_size=args.block_size,
                   blocks_per_cu=args.blocks_per_cu, device=dev)
    nH = torch.from_numpy(wl.n_H).to(dev)
    xn = torch.from_numpy(wl.x_n).to(dev)
    pos = torch.from_numpy(wl.src_pos).to(dev)
    lum = torch.from_numpy(wl.src_lum).to(dev)
    N = wl.n_cells
    rate = torch.empty(N, dtype=torch.float32, device=dev)
    force = torch.empty((3, N), dtype=torch.float32, device=dev)
    out = (rate, force, None)

    if args.autotune:
        bb, bp, ms = tr.autotune(nH, xn, pos, lum)
        log(f"[bench] autotune: {bb} threads x {bp} workgroups per CU ({ms:.1f} ms)")

    # ---- batched: all sources in one call ----
    for _ in range(args.warmup):
        tr.trace(nH, xn, pos, lum, out=out, check=False)
    rc = tr.sync()
    if rc != 0:
        log(f"[bench] device status {rc} after warm-up")
        sys.exit(1)
    st = tr.stats(wl.n_src)
    segments = st.segments
    log(f"[bench] {segments} segments per trace, {st.n_waves} wave(s), "
        f"rays in the largest wave {st.rays_max_wave}")

    torch.cuda.synchronize()
    tr.set_timing(True)
    sweep_ms = 0.0
    sweep_launches = 0
    t_start = time.perf_counter()
    for _ in range(args.steps):
        tr.trace(nH, xn, pos, lum, out=out, check=False)
        s_ms, n_l, _ = tr.timing()  # synchronises; sums this call's sweep-kernel events
        sweep_ms += s_ms
        sweep_launches += n_l
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    tr.set_timing(False)
    rc = tr.sync()
    if rc != 0:
        log(f"[bench] device status {rc}")
        sys.exit(1)
    ms_per_step = 1e3 * t_total / args.steps
    seg_per_s = segments * args.steps / t_total
    ms_per_source = ms_per_step / wl.n_src
    log(f"[bench] batched: {ms_per_step:.2f} ms/trace, {seg_per_s:.3e} segments/s, "
        f"{ms_per_source:.3f} ms per trace per source")

    # roofline of the sweep kernel: algorithmic bytes / summed kernel time
    sweep_s = sweep_ms / 1e3
    bps = BYTES_PER_SEGMENT
    achieved_gbs = segments * args.steps * bps / sweep_s / 1e9
    avg_launch_ms = sweep_ms / max(1, sweep_launches)

    # ---- plain: one source per call, same kernel and parameters ----
    plain = None
    if not args.no_plain:
        tp = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                       level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                       tau_term=wl.tau_term, deterministic=wl.deterministic, max_sources=1,
                       block_size=args.block_size, blocks_per_cu=args.blocks_per_cu, device=dev)
        r1 = torch.empty_like(rate)
        f1 = torch.empty_like(force)
        acc_r = torch.zeros_like(rate)
        acc_f = torch.zeros_like(force)
        tp.trace(nH, xn, pos[:1], lum[:1], out=(r1, f1, None), check=False)  # warm-up
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for s in range(wl.n_src):
            tp.trace(nH, xn, pos[s:s + 1], lum[s:s + 1], out=(r1, f1, None), check=False)
            acc_r += r1
            acc_f += f1
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - tp0
        rc = tp.sync()
        tp.close()
        # same accuracy: the sum of plain traces equals the batched trace
        m = rate.abs() > 1e-8 * float(wl.src_lum.sum())
        rel = ((acc_r - rate).abs()[m] / rate.abs()[m]).max().item() if m.any() else 0.0
        plain = {"ms_per_trace": 1e3 * t_plain, "segments_per_s": segments / t_plain,
                 "ms_per_trace_per_source": 1e3 * t_plain / wl.n_src,
                 "speedup_batched_over_plain": t_plain / (t_total / args.steps),
                 "max_rel_diff_rate_vs_batched": rel, "status": rc}
        log(f"[bench] plain: {1e3 * t_plain:.2f} ms for {wl.n_src} sources, speedup "
            f"{plain['speedup_batched_over_plain']:.2f}x, max rel diff {rel:.2e}")

    # ---- adjoint: the forward trace records the tree, then the adjoint sweep
    #      computes dL/dn_H and dL/dx_n for L = <w, rate> + <v, force> ----
    adjoint = None
    if not args.no_adjoint:
        tr.close()
        tr = None
        ta = ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                       level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                       tau_term=wl.tau_term, deterministic=wl.deterministic,
                       max_sources=wl.n_src, enable_adjoint=True, block_size=args.block_size,
                       blocks_per_cu=args.blocks_per_cu, device=dev)
        w_np, v_np = I.random_adjoint_weights(N, seed=7000 + args.workload)
        w = torch.from_numpy(w_np).to(dev)
        v = torch.from_numpy(v_np).to(dev)
        g_nH = torch.empty(N, dtype=torch.float32, device=dev)
        g_xn = torch.empty(N, dtype=torch.float32, device=dev)
        ta.trace(nH, xn, pos, lum, out=out, check=False)
        ta.adjoint(nH, xn, pos, lum, w, v, out=(g_nH, g_xn), check=False)
        rc = ta.sync()
        log("[bench] adjoint leg: warm-up done")
        t_fwd = t_adj = 0.0
        for _ in range(args.steps):
            torch.cuda.synchronize()
            ta0 = time.perf_counter()
            ta.trace(nH, xn, pos, lum, out=out, check=False)
            torch.cuda.synchronize()
            ta1 = time.perf_counter()
            ta.adjoint(nH, xn, pos, lum, w, v, out=(g_nH, g_xn), check=False)
            torch.cuda.synchronize()
            ta2 = time.perf_counter()
            t_fwd += ta1 - ta0
            t_adj += ta2 - ta1
            log(f"[bench] adjoint leg: step {1e3 * (ta1 - ta0):.1f} ms forward, {1e3 * (ta2 - ta1):.1f} ms adjoint")
        rc = rc or ta.sync()
        finite = bool(torch.isfinite(g_nH).all().item() and torch.isfinite(g_xn).all().item())
        graph = None
        if args.graph:
            ref = (rate.clone(), force.clone(), g_nH.clone(), g_xn.clone())

            def fwd_adj():
                ta.trace(nH, xn, pos, lum, out=out, check=False)
                ta.adjoint(nH, xn, pos, lum, w, v, out=(g_nH, g_xn), check=False)

            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                fwd_adj()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            log("[bench] graph: warm-up on the capture stream done")
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fwd_adj()
            torch.cuda.synchronize()
            log("[bench] graph: captured")
            tg0 = time.perf_counter()
            for _ in range(args.steps):
                g.replay()
            torch.cuda.synchronize()
            t_graph = (time.perf_counter() - tg0) / args.steps
            same = all(torch.equal(a, b) for a, b in zip((rate, force, g_nH, g_xn), ref))
            graph = {"ms_per_forward_adjoint": 1e3 * t_graph, "status": ta.sync(),
                     "bitwise_equal_to_eager": same if wl.deterministic else None}
            del g
            log(f"[bench] graph forward+adjoint: {1e3 * t_graph:.2f} ms per replay, equal to eager: {same}")
        ta.close()
        adj_s = t_adj / args.steps
        adj_gbs = segments * ADJOINT_BYTES_PER_SEGMENT / adj_s / 1e9
        adj_traffic = measured_adjoint_traffic(args.workload, wl.deterministic)
        adjoint = {"ms_per_adjoint": 1e3 * adj_s,
                   "ms_per_forward_with_tree": 1e3 * t_fwd / args.steps,
                   "segments_per_s": segments / adj_s,
                   "status": rc, "gradients_finite": finite, "graph": graph,
                   "roofline": {"bound": "hbm", "achieved": adj_gbs, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": adj_gbs / HBM_PEAK_GBS,
                                "traffic": None if adj_traffic is None else adj_traffic / 1e9,
                                "traffic_unit": "GB per adjoint sweep (sum over the per-level k_adjoint "
                                                "launches), rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated",
                                "kernel": "k_adjoint (one launch per level, deepest first; "
                                          "one backward walk over every segment)",
                                "bytes_per_segment": ADJOINT_BYTES_PER_SEGMENT}}
        log(f"[bench] adjoint: {1e3 * adj_s:.2f} ms per adjoint sweep "
            f"({segments / adj_s:.3e} segments/s), forward with tree "
            f"{1e3 * t_fwd / args.steps:.2f} ms, status {rc}")

    # ---- ionization subcycle: the R-type front at 128^3 (one source, C = 0.1) from
    #      t = 0 to 4 t_rec; eager (one synchronisation per substep) and replaying
    #      a HIP graph of 8 substeps until the clock reaches the end ----
    ion = None
    if not args.no_ion:
        if tr is not None:
            tr.close()
            tr = None
        p = I.rtype_problem(128)
        iw = p.wl
        ti = ArtTracer(iw.nx, iw.ny, iw.nz, s_H=iw.s_H, s_d=iw.s_d, n_bins=iw.n_bins,
                       deterministic=True, max_sources=1, device=dev)
        inH = torch.from_numpy(iw.n_H).to(dev)
        ipos = torch.from_numpy(iw.src_pos).to(dev)
        ilum = torch.from_numpy(iw.src_lum).to(dev)
        ix = torch.from_numpy(iw.x_n).to(dev)
        kw = dict(alpha_B=p.alpha_B, gamma_scale=p.gamma_scale, C=0.1)
        ti.ion_subcycle(inH, ix, ipos, ilum, t_end=0.01, **kw)  # warm-up
        ix.copy_(torch.from_numpy(iw.x_n).to(dev))
        torch.cuda.synchronize()
        te = time.perf_counter()
        k_eager, t_eager = ti.ion_subcycle(inH, ix, ipos, ilum, t_end=4.0, **kw)
        torch.cuda.synchronize()
        t_e = time.perf_counter() - te
        r_e = (3.0 * float((ix < 0.5).sum().item()) / (4.0 * math.pi)) ** (1.0 / 3.0)
        r_ref = p.R_S * (1.0 - math.exp(-4.0)) ** (1.0 / 3.0)
        # graph of 8 substeps
        N1 = iw.n_cells
        iout = (torch.empty(N1, device=dev), torch.empty((3, N1), device=dev), torch.empty((1, N1), device=dev))
        t_now = torch.zeros(1, dtype=torch.float64, device=dev)
        chunk = 8

        def steps():
            for _ in range(chunk):
                ti.ion_substep(inH, ix, ipos, ilum, t_end=4.0, t_now=t_now, out=iout, check=False, **kw)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            steps()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            steps()
        ix.copy_(torch.from_numpy(iw.x_n).to(dev))
        t_now.zero_()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        replays = 0
        while float(t_now.item()) < 4.0 and replays < 100000:
            g.replay()
            replays += 1
        torch.cuda.synchronize()
        t_g = time.perf_counter() - tg
        rc = ti.sync()
        del g
        r_g = (3.0 * float((ix < 0.5).sum().item()) / (4.0 * math.pi)) ** (1.0 / 3.0)
        ti.close()
        ion = {"workload": "R-type front: 128^3 uniform n_H, one central source, Method B, C = 0.1, "
                           "t = 0 to 4 t_rec",
               "substeps": k_eager, "eager_ms": 1e3 * t_e, "eager_ms_per_substep": 1e3 * t_e / max(1, k_eager),
               "graph_substeps_run": replays * chunk, "graph_ms": 1e3 * t_g,
               "graph_ms_per_substep": 1e3 * t_g / max(1, replays * chunk),
               "front_radius_rel_err_eager": r_e / r_ref - 1.0, "front_radius_rel_err_graph": r_g / r_ref - 1.0,
               "status": rc}
        log(f"[bench] ion subcycle: {k_eager} substeps to 4 t_rec, eager {1e3 * t_e:.1f} ms "
            f"({1e3 * t_e / max(1, k_eager):.3f} ms/substep), graph {1e3 * t_g:.1f} ms for "
            f"{replays * chunk} substeps; front radius {r_e / r_ref - 1:+.4f} vs analytic")

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read + written")

    # ---- CPU baseline: the FP64 oracle on a bounded sample (one source) ----
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        sample = wl.subset([0])
        tc = time.perf_counter()
        ref = O.trace_workload(sample)
        dt = time.perf_counter() - tc
        seg_cpu = int(ref.segments.sum())
        cpu = {"value": seg_cpu / dt, "unit": "segments/s", "cores": 1, "kind": "oracle",
               "sample": f"source 0 of the {wl.n_src}-source {wl.nx}^3 workload "
                         f"({seg_cpu} segments, {dt:.1f} s, single thread)",
               "ms_per_trace_per_source": 1e3 * dt}
        log(f"[bench] oracle: {seg_cpu / dt:.3e} segments/s on one core ({dt:.1f} s)")

    if tr is not None:
        tr.close()
    traffic = measured_traffic(args.workload, wl.deterministic)
    result = {
        "metric": "ray-cell segments/s (batched, one full trace of all sources per step)",
        "value": seg_per_s,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_trace_per_source": ms_per_source,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 deposits, f64 geometry and optical depth" if not wl.deterministic
                 else "i64 fixed-point deposits, f64 geometry and optical depth",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "n_sources": wl.n_src,
                   "n_bins": wl.n_bins, "level0": wl.level0, "level_max": wl.level_max,
                   "m_ray": wl.phi_c, "tau_term": wl.tau_term,
                   "deposit": "deterministic" if wl.deterministic else "atomic",
                   "segments_per_trace": segments, "waves": st.n_waves},
        "plain": plain,
        "adjoint": adjoint,
        "ion_subcycle": ion,
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / 1e9,
                     "traffic_unit": "GB per trace (sum over the per-level k_sweep launches), "
                                     "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated",
                     "kernel": "k_sweep (one launch per HEALPix level)",
                     "bytes_per_segment": bps,
                     "bytes_per_segment_with_accumulator_width":
                         BYTES_PER_SEGMENT_FIXED_POINT if wl.deterministic else BYTES_PER_SEGMENT,
                     "sweep_ms_per_step": sweep_ms / args.steps,
                     "avg_launch_ms": avg_launch_ms},
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

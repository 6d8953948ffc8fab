"""Benchmark of the ART sweep on one MI355X.

A step is one full batched forward trace (seed, every level's sweep, finalize)
of the 256^3 lognormal workload with 64 sources of log-uniform luminosity and
two frequency bins, inputs resident in HBM.  Prints ONE JSON line with
segments/s (whole job), ms per full trace per source, the plain (one source
per call) comparison, the roofline of the sweep kernel, the adjoint, the
ionization subcycle, the 512^3 / 1024-source forward + adjoint replayed from a
HIP graph, and the FP64 oracle's rate on a bounded sample of the same workload
(one core and all cores).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload 3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# Vector ALU issue of MI355X: 256 CUs x 4 SIMDs, each SIMD 16 lanes wide, so a
# wave64 VALU instruction (FP32 or FP64, not packed) occupies a SIMD for 4 cycles:
# one wave64 instruction per CU per cycle, 64 lane-operations, at 2.4 GHz.
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_PEAK_WAVE_INSTS = N_CU * CLOCK_HZ                  # wave64 VALU instructions / s
VALU_PEAK_TOPS = VALU_PEAK_WAVE_INSTS * 64 / 1e12      # 39.3 T lane-operations / s
# algorithmic bytes per ray-cell segment: the (n_H, x_n) gather (8 B) and a
# read-modify-write of the cell's four FP32 outputs (rate, F_x, F_y, F_z).  The
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


def measured_valu(workload: int, deterministic: bool):
    """VALU wave64 instructions per trace of the forward sweep (rocprofv3
    SQ_INSTS_VALU summed over the sweep launches), or None if stale."""
    if workload != 3:
        return None
    name = "k_sweep_c3_sq_counters.md" if deterministic else "k_sweep_c3_atomic_sq_counters.md"
    return _summary_value(name, "valu_insts_per_trace")


def measured_adjoint_traffic(workload: int, deterministic: bool):
    """HBM bytes per adjoint sweep, likewise (profiled in the fixed-point mode)."""
    if workload != 3 or not deterministic:
        return None
    return _summary_value("k_adjoint_c3_traffic.md", "traffic_bytes_per_adjoint")


def measured_adjoint_valu(workload: int, deterministic: bool):
    if workload != 3 or not deterministic:
        return None
    return _summary_value("k_adjoint_c3_sq_counters.md", "valu_insts_per_adjoint")


def measured_arith(workload: int, deterministic: bool, kernel: str):
    """Floating-point arithmetic VALU instructions (FP64 / FP32 add, mul, fma,
    transcendental) per 64 segments of `kernel` from the committed instruction-mix
    summary (fixed-point mode), or None if stale."""
    if workload != 3 or not deterministic:
        return None
    return _summary_value("k_sweep_k_adjoint_c3_valu_mix.md", f"arith_wave_insts_per_64_segments_{kernel}")


def roofline(kernel_s, segments, bytes_per_segment, traffic_bytes, valu_insts, kernel, traffic_unit, launches,
             arith_per_64=None):
    """The roofline block of a kernel: the method's bytes against HBM, the
    measured HBM traffic, and the measured VALU issue against the chip's issue
    rate.  The bound is whichever measured resource is busiest (HBM traffic or
    VALU issue); its figures are the top-level achieved / peak / frac.  The
    kernel runs as `launches` launches per pass (one per HEALPix level), and
    `traffic` is the measured HBM bytes of an average launch (GB)."""
    model_gbs = segments * bytes_per_segment / kernel_s / 1e9
    hbm = {"achieved": model_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": model_gbs / HBM_PEAK_GBS,
           "bytes_per_segment": bytes_per_segment,
           "measured_GBs": None if traffic_bytes is None else traffic_bytes / kernel_s / 1e9,
           "measured_frac": None if traffic_bytes is None else traffic_bytes / kernel_s / 1e9 / HBM_PEAK_GBS}
    valu = None
    if valu_insts is not None:
        tops = valu_insts * 64 / kernel_s / 1e12
        valu = {"achieved": tops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (VALU lane-operations)",
                "frac": tops / VALU_PEAK_TOPS, "wave_insts_per_segment_x64": valu_insts * 64 / segments}
        if arith_per_64 is not None:
            # the part of those lane-operations that is floating-point arithmetic
            # (one lane-operation per segment per wave instruction per 64 segments)
            at = arith_per_64 * segments / kernel_s / 1e12
            valu["arithmetic"] = {"lane_ops_per_segment": arith_per_64, "achieved": at,
                                  "frac": at / VALU_PEAK_TOPS}
    bound = "hbm"
    if valu is not None and (hbm["measured_frac"] is None or valu["frac"] > hbm["measured_frac"]):
        bound = "alu"
    top = valu if bound == "alu" else hbm
    n = max(1, launches)
    return {"bound": bound, "achieved": top["achieved"], "peak": top["peak"],
            "unit": "TOP/s" if bound == "alu" else "GB/s", "frac": top["frac"],
            "traffic": None if traffic_bytes is None else traffic_bytes / n / 1e9, "traffic_unit": traffic_unit,
            "traffic_per_pass": None if traffic_bytes is None else traffic_bytes / 1e9,
            "launches_per_pass": launches,
            "algorithmic_bytes_per_launch": segments * bytes_per_segment / n,
            "kernel": kernel, "hbm_model": hbm, "valu_issue": valu}


def copy_bandwidth_gbs(dev, mib=2048, repeats=5):
    """Median rate of a device-to-device copy of ``mib`` MiB, counting the bytes
    read and the bytes written."""
    import numpy as np
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del a, b
    return 2 * n * 4 / float(np.median(ts)) / 1e9


_BASELINE_WL = None  # the workload, inherited by the forked workers


def _oracle_worker(args):
    """One source of the bench workload through the oracle's timing build (a
    worker process of the all-cores baseline)."""
    lib, s = args
    from oracle import oracle as O
    with O.using_library(lib):
        t = time.perf_counter()
        ref = O.trace_workload(_BASELINE_WL.subset([s]))
        return int(ref.segments.sum()), time.perf_counter() - t


def cpu_baseline(wl):
    """The FP64 oracle, as it stands, built -O3 -march=native (no FMA contraction,
    no fast math: the same results), on the host's cores: one source on one core,
    then one source per core on all the cores this process may use (at most 16).
    Runs before anything touches the GPU (the workers are forked)."""
    import multiprocessing as mp
    from oracle import oracle as O
    global _BASELINE_WL
    _BASELINE_WL = wl
    lib = os.path.join(ROOT, "oracle", "liboracle_timing.so")
    O.compile_library(os.path.join(ROOT, "oracle", "art_oracle.c"), lib, opt=("-O3", "-march=native"))
    seg1, dt1 = _oracle_worker((lib, 0))
    log(f"[bench] oracle: {seg1 / dt1:.3e} segments/s on one core ({dt1:.1f} s)")
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores, wl.n_src))
    t = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(lib, s) for s in range(cores)])
    dt = time.perf_counter() - t
    seg = sum(r[0] for r in res)
    log(f"[bench] oracle: {seg / dt:.3e} segments/s on {cores} cores ({dt:.1f} s)")
    return {"value": seg / dt, "unit": "segments/s", "cores": cores, "kind": "oracle",
            "sample": f"sources 0..{cores - 1} of the {wl.n_src}-source {wl.nx}^3 workload, one per core "
                      f"({seg} segments, {dt:.1f} s wall); oracle built -O3 -march=native -ffp-contract=off",
            "ms_per_trace_per_source": 1e3 * dt / cores,
            "single_core": {"value": seg1 / dt1, "unit": "segments/s", "cores": 1,
                            "sample": f"source 0 ({seg1} segments, {dt1:.1f} s)",
                            "ms_per_trace_per_source": 1e3 * dt1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true", help="skip the one-source-per-call timing")
    ap.add_argument("--plain-repeats", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint sweep timing")
    ap.add_argument("--no-ion", action="store_true", help="skip the ionization-subcycle timing")
    ap.add_argument("--no-workload5", action="store_true",
                    help="skip the 512^3 / 1024-source forward + adjoint graph step")
    ap.add_argument("--graph", action="store_true",
                    help="also time forward + adjoint captured in one HIP graph (adjoint leg)")
    ap.add_argument("--atomic", action="store_true",
                    help="FP32 atomic deposits instead of the (faster) 64-bit fixed-point ones")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (launch shapes, sources per wave); by default its "
                         "cached result for this GPU and workload is applied, or it runs once and is cached")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the sweep is not "
              "sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    from paper_1711_06277_amd import inputs as I

    t0 = time.time()
    wl = I.config(args.workload)
    # 64-bit fixed-point deposits: integer LDS and global atomics are faster than
    # FP32 ones on this GPU, and the sums are bitwise reproducible
    wl.deterministic = not args.atomic
    log(f"[bench] workload {wl.name}: generated in {time.time() - t0:.1f}s")

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload
    #      (first, while no GPU context exists in this process) ----
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl)

    import torch
    from paper_1711_06277_amd import _abi as A
    from paper_1711_06277_amd.api import ArtTracer

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.device("cuda:0")

    def make_tracer(**kw):
        shape = (args.block_size, args.blocks_per_cu)
        if tuned is not None:
            shape = (tuned["block_size"], tuned["blocks_per_cu"])
        return ArtTracer(wl.nx, wl.ny, wl.nz, s_H=wl.s_H, s_d=wl.s_d, n_bins=wl.n_bins,
                         level0=wl.level0, level_max=wl.level_max, phi_c=wl.phi_c,
                         tau_term=wl.tau_term, deterministic=wl.deterministic,
                         block_size=shape[0], blocks_per_cu=shape[1], device=dev, **kw)

    tuned = None

    tr = make_tracer(max_sources=wl.n_src)
    nH = torch.from_numpy(wl.n_H).to(dev)
    xn = torch.from_numpy(wl.x_n).to(dev)
    pos = torch.from_numpy(wl.src_pos).to(dev)
    lum = torch.from_numpy(wl.src_lum).to(dev)
    N = wl.n_cells
    rate = torch.empty(N, dtype=torch.float32, device=dev)
    force = torch.empty((3, N), dtype=torch.float32, device=dev)
    out = (rate, force, None)

    if not args.no_autotune and not (args.block_size or args.blocks_per_cu):
        ta0 = time.perf_counter()
        bb, bp, bw, ms = tr.autotune(nH, xn, pos, lum, cache=True)
        tuned = {"block_size": bb, "blocks_per_cu": bp, "wave_sources": bw, "ms": ms,
                 "s_spent": time.perf_counter() - ta0}
        log(f"[bench] autotune: {bb} threads x {bp} workgroups per CU, wave cap {bw or 'none'} "
            f"({ms:.1f} ms, {tuned['s_spent']:.1f} s)")

    # ---- batched: all sources in one call ----
    for _ in range(args.warmup):
        tr.trace(nH, xn, pos, lum, out=out, check=False)
    rc = tr.sync()
    if rc != 0:
        log(f"[bench] device status {rc} after warm-up")
        sys.exit(1)

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
    st = tr.stats(wl.n_src)  # of the last timed trace (every trace makes the same segments)
    segments = st.segments
    log(f"[bench] {segments} segments per trace, {st.n_waves} wave(s), "
        f"rays in the largest wave {st.rays_max_wave}")
    ms_per_step = 1e3 * t_total / args.steps
    seg_per_s = segments * args.steps / t_total
    ms_per_source = ms_per_step / wl.n_src
    log(f"[bench] batched: {ms_per_step:.2f} ms/trace, {seg_per_s:.3e} segments/s, "
        f"{ms_per_source:.3f} ms per trace per source")

    # roofline of the sweep kernel: measured per-launch durations (HIP events on
    # the library's stream), summed over a trace
    sweep_s = sweep_ms / 1e3 / args.steps
    avg_launch_ms = sweep_ms / max(1, sweep_launches)
    n_launch_levels = sweep_launches // max(1, args.steps)  # levels launched per trace (and per adjoint)
    roof = roofline(sweep_s, segments, BYTES_PER_SEGMENT, measured_traffic(args.workload, wl.deterministic),
                    measured_valu(args.workload, wl.deterministic),
                    "k_sweep (one launch per HEALPix level)",
                    "GB per k_sweep launch (the average of one trace's per-level launches; traffic_per_pass "
                    "is their sum), rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated",
                    n_launch_levels, measured_arith(args.workload, wl.deterministic, "k_sweep"))
    roof.update({"bytes_per_segment": BYTES_PER_SEGMENT,
                 "bytes_per_segment_with_accumulator_width":
                     BYTES_PER_SEGMENT_FIXED_POINT if wl.deterministic else BYTES_PER_SEGMENT,
                 "sweep_ms_per_step": sweep_ms / args.steps, "avg_launch_ms": avg_launch_ms})
    # what a plain device copy reaches on this GPU (bytes read + written per
    # second, median of 5): the achievable HBM rate beside the published peak
    roof["hbm_model"]["copy_GBs"] = copy_bandwidth_gbs(dev)
    log(f"[bench] roofline: bound {roof['bound']}, frac {roof['frac']:.3f}; HBM model "
        f"{roof['hbm_model']['frac']:.3f}; device copy {roof['hbm_model']['copy_GBs']:.0f} GB/s")

    # ---- plain: one source per call, same kernel and parameters ----
    plain = None
    if not args.no_plain:
        tp = make_tracer(max_sources=1)
        r1 = torch.empty_like(rate)
        f1 = torch.empty_like(force)
        # untimed pass: the sum of the plain traces equals the batched trace
        acc_r = torch.zeros(N, dtype=torch.float64, device=dev)
        for s in range(wl.n_src):
            tp.trace(nH, xn, pos[s:s + 1], lum[s:s + 1], out=(r1, f1, None), check=False)
            acc_r += r1
        m = rate.abs() > 1e-8 * float(wl.src_lum.sum())
        rel = ((acc_r - rate.double()).abs()[m] / rate.double().abs()[m]).max().item() if m.any() else 0.0
        del acc_r
        times = []
        for _ in range(args.plain_repeats):
            torch.cuda.synchronize()
            tp0 = time.perf_counter()
            for s in range(wl.n_src):
                tp.trace(nH, xn, pos[s:s + 1], lum[s:s + 1], out=(r1, f1, None), check=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - tp0)
        rc = tp.sync()
        tp.close()
        t_plain = statistics.median(times)
        plain = {"ms_per_trace": 1e3 * t_plain, "ms_per_trace_min": 1e3 * min(times),
                 "ms_per_trace_max": 1e3 * max(times), "repeats": len(times),
                 "segments_per_s": segments / t_plain,
                 "ms_per_trace_per_source": 1e3 * t_plain / wl.n_src,
                 "speedup_batched_over_plain": t_plain / (t_total / args.steps),
                 "max_rel_diff_rate_vs_batched": rel, "status": rc}
        log(f"[bench] plain: median {1e3 * t_plain:.2f} ms for {wl.n_src} sources "
            f"({1e3 * min(times):.2f}..{1e3 * max(times):.2f}), speedup "
            f"{plain['speedup_batched_over_plain']:.2f}x, max rel diff {rel:.2e}")

    # ---- adjoint: the forward trace records the tree, then the adjoint sweep
    #      walks it back for dL/dn_H and dL/dx_n, L = <w, rate> + <v, force> ----
    adjoint = None
    if not args.no_adjoint:
        tr.close()
        tr = None
        ta = make_tracer(max_sources=wl.n_src, enable_adjoint=True)
        w_np, v_np = I.random_adjoint_weights(N, seed=7000 + args.workload)
        w = torch.from_numpy(w_np).to(dev)
        v = torch.from_numpy(v_np).to(dev)
        if tuned is not None:
            if tuned["wave_sources"]:
                ta.set_wave_sources(tuned["wave_sources"])
            ab, ap, ams = ta.autotune_adjoint(nH, xn, pos, lum, w, v, cache=True)
            tuned["adjoint"] = {"block_size": ab, "blocks_per_cu": ap, "ms": ams}
            log(f"[bench] adjoint autotune: {ab} threads x {ap} workgroups per CU ({ams:.1f} ms)")
        g_nH = torch.empty(N, dtype=torch.float32, device=dev)
        g_xn = torch.empty(N, dtype=torch.float32, device=dev)
        ta.trace(nH, xn, pos, lum, out=out, check=False)
        ta.adjoint(nH, xn, pos, lum, w, v, tape=ta.last_tape or None, out=(g_nH, g_xn), check=False)
        rc = ta.sync()
        log(f"[bench] adjoint leg: warm-up done (tape {'kept' if ta.last_tape else 'not kept'})")
        t_fwd = t_adj = 0.0
        for _ in range(args.steps):
            torch.cuda.synchronize()
            ta0 = time.perf_counter()
            ta.trace(nH, xn, pos, lum, out=out, check=False)
            torch.cuda.synchronize()
            ta1 = time.perf_counter()
            ta.adjoint(nH, xn, pos, lum, w, v, tape=ta.last_tape or None, out=(g_nH, g_xn), check=False)
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
                ta.adjoint(nH, xn, pos, lum, w, v, tape=ta.last_tape or None, out=(g_nH, g_xn), check=False)

            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                fwd_adj()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fwd_adj()
            torch.cuda.synchronize()
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
        adj_roof = roofline(adj_s, segments, ADJOINT_BYTES_PER_SEGMENT,
                            measured_adjoint_traffic(args.workload, wl.deterministic),
                            measured_adjoint_valu(args.workload, wl.deterministic),
                            "k_adjoint (one launch per level, deepest first; one backward walk over every segment)",
                            "GB per k_adjoint launch (the average of one adjoint's per-level launches; "
                            "traffic_per_pass is their sum), rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated",
                            n_launch_levels, measured_arith(args.workload, wl.deterministic, "k_adjoint"))
        adj_roof["bytes_per_segment"] = ADJOINT_BYTES_PER_SEGMENT
        adjoint = {"ms_per_adjoint": 1e3 * adj_s,
                   "ms_per_forward_with_tree": 1e3 * t_fwd / args.steps,
                   "segments_per_s": segments / adj_s,
                   "status": rc, "gradients_finite": finite, "graph": graph, "roofline": adj_roof}
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

    if tr is not None:
        tr.close()
        tr = None

    # ---- 512^3, 1024 sources (dN/dL ~ L^-2), fixed point: forward + adjoint of
    #      L = <w, rate> + <v, force> in one call, captured in a HIP graph; one
    #      eager step, then one replay, bitwise compared ----
    w5 = None
    if not args.no_workload5:
        del nH, xn, pos, lum
        t5 = time.time()
        c5 = I.config(5)
        log(f"[bench] workload {c5.name}: generated in {time.time() - t5:.1f}s")
        # a pool of 80% of the free HBM (72 bytes per ray with the adjoint's tape), and the
        # launch shapes tuned on the 256^3 workload (the same kernels)
        tr5 = ArtTracer(c5.nx, c5.ny, c5.nz, s_H=c5.s_H, s_d=c5.s_d, n_bins=c5.n_bins, deterministic=True,
                        max_sources=c5.n_src, enable_adjoint=True, pool_mem_fraction=0.8, device=dev)
        if tuned is not None:
            A.art_set_launch(tr5._ctx, tuned["block_size"], tuned["blocks_per_cu"])
            if "adjoint" in tuned:
                A.art_set_adjoint_launch(tr5._ctx, tuned["adjoint"]["block_size"], tuned["adjoint"]["blocks_per_cu"])
        a5 = [torch.from_numpy(x).to(dev) for x in (c5.n_H, c5.x_n, c5.src_pos, c5.src_lum, c5.w, c5.v)]
        N5 = c5.n_cells
        o5 = (torch.empty(N5, device=dev), torch.empty((3, N5), device=dev), None,
              torch.empty(N5, device=dev), torch.empty(N5, device=dev))

        def step5():
            tr5.trace_and_adjoint(*a5, out=o5, check=False)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        # the forward trace alone, once (eager)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        with torch.cuda.stream(side):
            tr5.trace(*a5[:4], out=(o5[0], o5[1], None), check=False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        t_fwd5 = time.perf_counter() - tf
        rcf5 = tr5.sync()
        st5f = tr5.stats(c5.n_src)
        log(f"[bench] workload 5 eager forward: {t_fwd5:.2f} s, {st5f.segments} segments, "
            f"{st5f.n_waves} waves, status {rcf5}")
        torch.cuda.synchronize()
        te = time.perf_counter()
        with torch.cuda.stream(side):
            step5()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        t_eager5 = time.perf_counter() - te
        rc5 = tr5.sync()
        st5 = tr5.stats(c5.n_src)
        ref5 = [o.clone() for o in o5 if o is not None]
        log(f"[bench] workload 5 eager forward+adjoint: {t_eager5:.2f} s, {st5.segments} segments, "
            f"{st5.n_waves} waves, status {rc5}")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step5()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        t_graph5 = time.perf_counter() - tg
        same5 = all(torch.equal(a, b) for a, b in zip([o for o in o5 if o is not None], ref5))
        rc5 = rc5 or tr5.sync()
        del g
        tr5.close()
        w5 = {"workload": c5.name, "grid": [c5.nx, c5.ny, c5.nz], "n_sources": c5.n_src,
              "segments_per_pass": st5.segments, "waves": st5.n_waves, "rays_max_wave": st5.rays_max_wave,
              "s_forward_eager": t_fwd5, "waves_forward": st5f.n_waves,
              "segments_per_s_forward": st5f.segments / t_fwd5, "status_forward": rcf5,
              "s_forward_adjoint_eager": t_eager5, "s_forward_adjoint_graph_replay": t_graph5,
              "segments_per_s_forward_plus_adjoint": 2 * st5.segments / t_graph5,
              "graph_bitwise_equal_to_eager": same5, "status": rc5}
        log(f"[bench] workload 5 graph forward+adjoint: {t_graph5:.2f} s per replay, equal to eager: {same5}")

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read + written")

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
        "workload5_forward_adjoint_graph": w5,
        "autotune": tuned,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

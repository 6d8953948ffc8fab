"""Host logic of bench.py (no GPU): the kernel-source hash that decides whether the
committed counter summaries still describe the built kernels, and the lookup of
the measured traffic."""
import os
import shutil

import pytest

import bench


@pytest.fixture
def src_copy(tmp_path, monkeypatch):
    """bench's ROOT pointed at a scratch copy of the two kernel sources."""
    for f in ("paper_1711_06277_amd/csrc/art.hip", "paper_1711_06277_amd/csrc/art_device.h"):
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def _edit(path, fn):
    text = path.read_text()
    path.write_text(fn(text))


def test_hash_ignores_comments_and_blank_space(src_copy):
    h0 = bench.kernel_sources_sha()
    hip = src_copy / "paper_1711_06277_amd/csrc/art.hip"
    _edit(hip, lambda t: "// a new comment line\n" + t.replace("\n\n", "\n\n\n", 3) + "\n/* block\n comment */\n")
    assert bench.kernel_sources_sha() == h0


def test_hash_follows_code_changes(src_copy):
    h0 = bench.kernel_sources_sha()
    dev = src_copy / "paper_1711_06277_amd/csrc/art_device.h"
    _edit(dev, lambda t: t.replace("kStStuck = 4", "kStStuck = 16", 1))
    assert bench.kernel_sources_sha() != h0


def test_measured_traffic_needs_matching_sources(src_copy):
    """A counter summary's traffic is reported for the sources it was taken on,
    and withheld (None) once the code differs."""
    prof = src_copy / "profiles"
    prof.mkdir()
    sha = bench.kernel_sources_sha()
    for name, val in (("k_sweep_c3_traffic.md", 1.5e11), ("k_sweep_c3_atomic_traffic.md", 1.25e11)):
        (prof / name).write_text(f"# summary\n\ntraffic_bytes_per_trace: {val:.6e}\nkernel_sources_sha: {sha}\n")
    assert bench.measured_traffic(3, True) == 1.5e11
    assert bench.measured_traffic(3, False) == 1.25e11
    assert bench.measured_traffic(5, True) is None  # only the 256^3 workload is profiled
    (prof / "k_adjoint_c3_traffic.md").write_text(f"# summary\n\ntraffic_bytes_per_adjoint: 2.5e11\nkernel_sources_sha: {sha}\n")
    assert bench.measured_adjoint_traffic(3, True) == 2.5e11
    assert bench.measured_adjoint_traffic(3, False) is None  # the adjoint is profiled in fixed point
    _edit(src_copy / "paper_1711_06277_amd/csrc/art.hip", lambda t: t + "\nstatic int art_unused_marker = 1;\n")
    assert bench.measured_traffic(3, True) is None
    assert bench.measured_adjoint_traffic(3, True) is None


def test_committed_summaries_are_readable():
    """The committed summaries carry the two fields bench.py reads."""
    for name, key in (("k_sweep_c3_traffic.md", "traffic_bytes_per_trace:"),
                      ("k_sweep_c3_atomic_traffic.md", "traffic_bytes_per_trace:"),
                      ("k_adjoint_c3_traffic.md", "traffic_bytes_per_adjoint:")):
        with open(os.path.join(bench.ROOT, "profiles", name)) as fh:
            text = fh.read()
        assert key in text and "kernel_sources_sha:" in text


def test_roofline_picks_the_busiest_measured_resource():
    """VALU issue above the measured HBM fraction names the bound "alu"; traffic
    is reported per launch (the pass's sum divided by its launches)."""
    seg, t = 1.0e10, 0.1
    valu = 0.6 * bench.VALU_PEAK_WAVE_INSTS * t  # 60% of the issue rate
    r = bench.roofline(t, seg, 40, 2.0e11, valu, "k", "GB per launch", 8)
    assert r["bound"] == "alu" and r["unit"] == "TOP/s"
    assert r["frac"] == pytest.approx(0.6)
    assert r["traffic"] == pytest.approx(2.0e11 / 8 / 1e9)
    assert r["traffic_per_pass"] == pytest.approx(200.0)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(seg * 40 / 8)
    assert r["hbm_model"]["frac"] == pytest.approx(seg * 40 / t / 1e9 / bench.HBM_PEAK_GBS)
    # measured traffic busier than the VALU: "hbm", with the model's figures on top
    r = bench.roofline(t, seg, 40, 0.7 * bench.HBM_PEAK_GBS * 1e9 * t, valu, "k", "u", 8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(r["hbm_model"]["frac"])
    # the arithmetic share of the VALU work, when the instruction mix is known
    r = bench.roofline(t, seg, 40, 2.0e11, valu, "k", "u", 8, arith_per_64=60.0)
    assert r["valu_issue"]["arithmetic"]["achieved"] == pytest.approx(60.0 * seg / t / 1e12)
    assert bench.measured_arith(3, True, "k_sweep") is None or bench.measured_arith(3, True, "k_sweep") > 0
    # no counters: HBM model only, traffic unknown
    r = bench.roofline(t, seg, 40, None, None, "k", "u", 8)
    assert r["bound"] == "hbm" and r["traffic"] is None and r["valu_issue"] is None

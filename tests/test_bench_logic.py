"""Host logic of the measurement record in bench.py (no GPU): the byte counts
the roofline divides by, the hash that ties a counter record to the kernel
sources it was taken on, and the choice of the bound from the counters."""
import json

import pytest

import bench


@pytest.mark.parametrize("elem", [4, 8])
def test_step_bytes_are_the_two_stages_and_the_moments(elem):
    # per step: stage 1 (I^n in, I* out), stage 2 (I*, I^n in, I^n+1 out) and
    # R^(ab) of the new intensity -- 5 intensity transfers per cell-direction
    ns, nc = 162, 128 ** 3
    s1 = bench.algorithmic_bytes("stage1", elem, ns, nc)
    s2 = bench.algorithmic_bytes("stage2", elem, ns, nc)
    assert bench.step_algorithmic_bytes(elem, ns, nc) == s1 + s2 + bench.R_B * nc
    assert s1 + s2 - (16 + 24 + 2 * bench.FIELDS_B) * nc == 5 * elem * ns * nc


def test_bin_step_bytes_scale_with_the_bins():
    ns, nc = 162, 64 ** 3
    one = bench.step_algorithmic_bytes(4, ns, nc, ng=1)
    four = bench.step_algorithmic_bytes(4, ns, nc, ng=4)
    # each further bin adds its 5 intensity transfers and, per stage, its kappa_a
    assert four - one == 3 * (5 * 4 * ns * nc + 2 * 8 * nc)


def test_code_hash_ignores_comments_but_not_code():
    a = "int f(int x) {\n  // twice\n  return 2 * x;  /* doubled */\n}\n"
    b = "/* header\n   text */\nint f(int x) {\n\n  return 2 * x;\n}\n"
    c = "int f(int x) {\n  return 3 * x;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def _record(tmp_path, key, sha, **fields):
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({"per_launch": {key: dict(sources_sha256=sha, **fields)}}))
    return str(path)


def test_counters_are_used_only_on_the_sources_they_were_taken_on(tmp_path, monkeypatch):
    sha = bench.sources_sha256(bench.KERNEL_SOURCES["stage2"])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _record(tmp_path, "w/stage2_fp32", sha, bytes=1.0, valu_insts=2.0))
    assert bench.counters_for("w", "stage2", 4)["bytes"] == 1.0
    assert bench.counters_for("w", "stage2", 8) is None  # no FP64 record
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _record(tmp_path, "w/stage2_fp32", "0" * 64, bytes=1.0))
    assert bench.counters_for("w", "stage2", 4) is None  # taken on other sources


def _run(ms_per_launch, launches=10):
    return {"ktimes": {"stage1": (launches, 0.5 * ms_per_launch * launches),
                       "stage2": (launches, ms_per_launch * launches)},
            "elem": 4, "ns": 162, "nc": 128 ** 3}


@pytest.mark.parametrize("valu_frac, bound", [(0.9, "alu"), (0.1, "hbm")])
def test_bound_is_the_busier_unit(monkeypatch, valu_frac, bound):
    t = 1.4e-3
    traffic = 0.5 * bench.HBM_PEAK_GBS * 1e9 * t  # HBM half busy
    valu = valu_frac * bench.SIMDS * bench.CLOCK_HZ * t / bench.VALU_CYCLES
    monkeypatch.setattr(bench, "counters_for", lambda w, k, e: {"bytes": traffic, "valu_insts": valu})
    blk = bench.roofline_block("w", _run(t * 1e3))
    assert blk["kernel"] == "stage2"  # the longest-running kernel
    assert blk["bound"] == bound
    assert blk["hbm_busy_measured"] == pytest.approx(0.5)
    assert blk["valu_busy"] == pytest.approx(valu_frac)
    assert blk["frac"] == pytest.approx(valu_frac if bound == "alu" else blk["hbm_frac_algorithmic"])
    alg = bench.algorithmic_bytes("stage2", 4, 162, 128 ** 3)
    assert blk["hbm_frac_algorithmic"] == pytest.approx(alg / t / 1e9 / bench.HBM_PEAK_GBS)


def test_bound_without_counters_is_hbm_on_algorithmic_bytes(monkeypatch):
    monkeypatch.setattr(bench, "counters_for", lambda w, k, e: None)
    blk = bench.roofline_block("w", _run(1.4))
    assert blk["bound"] == "hbm" and blk["traffic"] is None and "valu_busy" not in blk

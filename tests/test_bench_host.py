"""Host logic of bench.py: the algorithmic byte and flop model behind the roofline record, the
choice of the bound, the validity of the committed counter records, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_byte_and_flop_model_of_the_16384_position_workload(bench):
    from paper_2205_03902_amd import configs
    geo = configs.CFG4
    byt, flo = bench.model_per_launch(geo)
    # per position: intensities 4 N^2; incident waves written and read back for slices 1..M-1,
    # the M slice-gradient patches and the probe-gradient patch, 8 N^2 each
    n2, M, S = 256 * 256, 12, 16384
    assert byt == S * (4 * n2 + 8 * n2 * (2 * (M - 1) + M + 1))
    # (4M - 2) 2D FFTs of 5 N^2 log2 N^2 = 10 N^2 log2 N flops, plus the pointwise work
    assert flo == pytest.approx(S * ((4 * M - 2) * 10 * n2 * 8 + 30 * n2 * M + 20 * n2), rel=1e-15)
    assert flo / 1e12 == pytest.approx(4.36, abs=0.005)
    # the whole pass with the slices' own traffic: 417 GB
    assert bench.pass_bytes(geo) / 1e9 == pytest.approx(417, abs=0.5)


def test_roofline_takes_the_bound_with_the_larger_fraction(bench):
    from paper_2205_03902_amd import configs
    geo = configs.CFG4
    byt, flo = bench.model_per_launch(geo)
    for ms in (30.0, 120.0, 400.0):
        r = bench.roofline(geo, "lines", ms)
        alu = flo / (ms * 1e-3) / bench.ALU_PEAK
        hbm = byt / (ms * 1e-3) / bench.HBM_PEAK
        assert r["frac"] == pytest.approx(max(alu, hbm))
        assert r["bound"] == ("alu" if alu >= hbm else "hbm")
        assert r["other"]["frac"] == pytest.approx(min(alu, hbm))
        assert r["achieved"] == pytest.approx(r["frac"] * r["peak"])
    # the FP32 peak without packed FP32: 256 CUs x 64 lanes x 2 flops x 2.4 GHz
    assert bench.ALU_PEAK == pytest.approx(256 * 64 * 2 * 2.4e9, rel=1e-3)


def test_counter_records_are_used_only_for_their_workload_path_and_sources(bench, monkeypatch):
    from paper_2205_03902_amd import configs
    for geo, fam in ((configs.CFG4, "lines"), (configs.CFG1, "fused")):
        with open(bench.traffic_file(geo, fam)) as fh:
            rec = json.load(fh)
        assert rec["workload"] == geo.name and rec["family"] == fam
        assert rec["bytes_per_pass"] == pytest.approx(rec["read_bytes_per_pass"] + rec["write_bytes_per_pass"])
        # VALU issue time: instructions x 4 cycles over 1024 SIMDs at 2.4 GHz
        assert rec["valu_issue_ms_per_pass"] == pytest.approx(
            rec["valu_instructions_per_pass"] * 4 / (1024 * 2.4e9) * 1e3, rel=1e-9)
        if bench.traffic_record(geo, fam) is not None:
            assert bench.roofline(geo, fam, 100.0)["traffic"] == rec["bytes_per_pass"]
    # another path, another workload, or changed kernel sources: no record
    assert bench.traffic_record(configs.CFG4, "fused") is None
    assert bench.traffic_record(configs.CFG2, "lines") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda family: "0" * 16)
    assert bench.traffic_record(configs.CFG4, "lines") is None
    assert bench.roofline(configs.CFG4, "lines", 100.0)["traffic"] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr and r.stdout == ""



def test_a_failing_leg_is_recorded_and_the_line_survives(bench):
    out = {"value": 1.0}
    bench.guarded(out, "ok", lambda: {"ratio_median": 0.2})

    def fails():
        raise RuntimeError("out of memory")
    bench.guarded(out, "broken", fails)
    assert out["ok"] == {"ratio_median": 0.2} and out["value"] == 1.0
    assert "out of memory" in out["broken"]["error"]

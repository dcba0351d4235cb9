"""Host logic of the measurement record: the code digest that ties the
committed counter summaries to the collide kernels' sources, the summaries'
format (written from rocprofv3 CSV output by profile_summary, read back by
bench.py), and what each HBM counter stands for after calibration.  Inputs
are small synthetic counter tables in rocprofv3's CSV layout."""
import csv
import os

import pytest

import bench
from paper_2407_19151_amd import profile_summary as P

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "LDS_Block_Size", "Scratch_Size", "Workgroup_Size",
          "Grid_Size"]
K32 = "void mcc::collide_kernel<256, 1024, float, false, 1, false, false, 0>(mcc::CollideArgs)"
K64 = "void mcc::collide_kernel<64, 128, double, false, 1, false, false, 0>(mcc::CollideArgs)"
KDIAG = "void mcc::collide_kernel<64, 128, double, false, 1, false, true, 0>(mcc::CollideArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _csv(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, ctr, val in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": ctr,
                        "Counter_Value": val, "VGPR_Count": 168, "Accum_VGPR_Count": 0,
                        "SGPR_Count": 106, "LDS_Block_Size": 52736, "Scratch_Size": 0,
                        "Workgroup_Size": 256, "Grid_Size": 196608})


def test_code_text_ignores_comments_only():
    a = "int a = 1; // one\n/* two\n   lines */ int b = a;\n"
    b = "int a = 1;\n// another comment\nint b = a; /* more */\n"
    c = "int a = 2; // one\nint b = a;\n"
    assert P.code_text(a) == P.code_text(b) == "int a = 1; int b = a;"
    assert P.code_text(c) != P.code_text(a)


def test_source_hash_covers_the_kernel_sources():
    h = P.source_hash()
    assert len(h) == 64 and h == P.source_hash()
    assert bench.kernel_source_hash() == h


def test_kernel_keys():
    assert P.kernel_key(K32) == ("fp32", "256x1024", "L1")
    assert P.kernel_key(K64) == ("fp64", "64x128", "L1")
    # only the plain order-N forms are keyed (not diagnostics, tangents, ...)
    assert P.kernel_key(KDIAG) is None
    assert P.kernel_key("k_bucket_cells(long)") is None


def test_traffic_summary_round_trip(tmp_path, monkeypatch):
    # two dispatches of the FP32 kernel: the summary keeps their average
    _csv(tmp_path / "f", [(1, K32, "FETCH_SIZE", 1000.0), (2, K32, "FETCH_SIZE", 3000.0),
                          (3, K64, "FETCH_SIZE", 10.0), (4, KDIAG, "FETCH_SIZE", 5.0)])
    _csv(tmp_path / "w", [(1, K32, "WRITE_SIZE", 4000.0), (2, K32, "WRITE_SIZE", 4000.0),
                          (3, K64, "WRITE_SIZE", 20.0)])
    # a 1 GiB copy whose FETCH_SIZE reads half its bytes and WRITE_SIZE all of
    # them (the largest copy dispatch is the calibration one)
    _csv(tmp_path / "cf", [(1, COPY, "FETCH_SIZE", 524288.0), (2, COPY, "FETCH_SIZE", 100.0)])
    _csv(tmp_path / "cw", [(1, COPY, "WRITE_SIZE", 1048576.0)])
    text = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                     str(tmp_path / "cw"), ["the command"])
    assert "fetch_factor 2.0000" in text and "write_factor 1.0000" in text
    out = tmp_path / "traffic.txt"
    out.write_text(text)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    t = bench.read_traffic()
    assert set(t) == {("fp32", "256x1024", "L1"), ("fp64", "64x128", "L1")}
    assert t[("fp32", "256x1024", "L1")] == pytest.approx((2000.0 * 2 + 4000.0) * 1024)
    assert t[("fp64", "64x128", "L1")] == pytest.approx((10.0 * 2 + 20.0) * 1024)
    # counters taken from other sources are not reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.read_traffic() is None


def test_valu_summary_round_trip(tmp_path, monkeypatch):
    a = [(1, K32, "SQ_INSTS_VALU", 1.0e8), (1, K32, "SQ_ACTIVE_INST_VALU", 2.0e9),
         (1, K32, "SQ_THREAD_CYCLES_VALU", 64.0 * 0.75 * 2.0e9), (1, K32, "SQ_WAIT_INST_ANY", 1.0),
         (1, K32, "SQ_WAVE_CYCLES", 10.0), (1, K32, "GRBM_GUI_ACTIVE", 8.0 * 1.0e7),
         (1, K32, "SQ_INSTS_LDS", 5.0), (1, K32, "SQ_WAVES", 3072.0)]
    b = [(1, K32, "SQ_INSTS_VALU_ADD_F64", 10.0), (1, K32, "SQ_INSTS_VALU_MUL_F64", 20.0),
         (1, K32, "SQ_INSTS_VALU_TRANS_F64", 1.0), (1, K32, "SQ_INSTS_VALU_FMA_F64", 30.0),
         (1, K32, "SQ_INSTS_SALU", 7.0)]
    _csv(tmp_path / "a", a)
    _csv(tmp_path / "b", b)
    text = P.valu(str(tmp_path / "a"), str(tmp_path / "b"), ["the command"])
    line = [l for l in text.splitlines() if l.startswith("kernel fp32 256x1024 L1")][0].split()
    # busy: 4 cycles per counted VALU quad-cycle over (GRBM cycles per XCD x 1024 SIMDs)
    assert float(line[line.index("busy") + 1]) == pytest.approx(2.0e9 * 4 / (1.0e7 * 1024),
                                                                abs=1e-3)
    assert float(line[line.index("lanes") + 1]) == pytest.approx(0.75, abs=1e-3)
    out = tmp_path / "valu.txt"
    out.write_text(text)
    monkeypatch.setattr(bench, "VALU_FILE", str(out))
    v = bench.read_valu()
    valu, f64 = v[("fp32", "256x1024", "L1")]
    assert valu == pytest.approx(1.0e8)
    # 64 lanes x (ADD + MUL + TRANS + 2 FMA)
    assert f64 == pytest.approx(64.0 * (10 + 20 + 1 + 2 * 30))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.read_valu() is None


def test_committed_summaries_parse():
    """The committed summaries are in the format bench.py reads, and name
    the dominant kernel of the headline step in both precisions."""
    for path in (bench.TRAFFIC_FILE, bench.VALU_FILE):
        src = [l.split()[1] for l in open(path) if l.startswith("source_sha256")]
        assert len(src) == 1 and len(src[0]) == 64
        keys = {tuple(l.split()[1:4]) for l in open(path) if l.startswith("kernel ")}
        assert ("fp32", "256x1024", "L1") in keys and ("fp64", "256x1024", "L1") in keys

"""The traffic summary behind bench.py's roofline.traffic: counter CSVs are
scaled by the calibration copy, mapped to the sampler's kernel kinds, and a
stored figure is only reported for the kernel sources and register variant
it was measured with."""
import csv
import json

from paper_2403_19854_amd import traffic

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
        "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
        "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
        "Counter_Value", "Start_Timestamp", "End_Timestamp"]
MID = "void fcrkpm::(anonymous namespace)::k_rmid<fcrkpm::(anonymous namespace)::G16, 1, 3, 3>(x)"
X1 = ("void fcrkpm::(anonymous namespace)::k_rpass<fcrkpm::(anonymous namespace)::G16, "
      "fcrkpm::(anonymous namespace)::Lin3, 1, true, true, false, 1, 0, true>(x)")
Y1_G8 = ("void fcrkpm::(anonymous namespace)::k_rpass<fcrkpm::(anonymous namespace)::G8<16>, "
         "fcrkpm::(anonymous namespace)::Lin3, 1, false, false, false, 1, 1, false>(x)")


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for name, val in rows:
            r = ["0"] * len(HEAD)
            r[HEAD.index("Kernel_Name")] = name
            r[HEAD.index("Counter_Name")] = counter
            r[HEAD.index("Counter_Value")] = str(val)
            w.writerow(r)


def _make(tmp_path):
    copy_kib = traffic.COPY_BYTES / 1024
    _csv(tmp_path / "f.csv", "FETCH_SIZE",
         [("__amd_rocclr_copyBuffer", copy_kib / 2), ("__amd_rocclr_copyBuffer", 3.0),
          (MID, 1000.0), (MID, 1100.0), (X1, 500.0), (Y1_G8, 700.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE",
         [("__amd_rocclr_copyBuffer", copy_kib), (MID, 400.0), (MID, 400.0), (X1, 300.0),
          (Y1_G8, 200.0)])
    out = tmp_path / "t.json"
    d = traffic.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "wl", "cmd")
    return d, out


def test_summary_scales_and_maps_kinds(tmp_path):
    d, out = _make(tmp_path)
    assert abs(d["fetch_scale"] - 2.0) < 1e-12 and abs(d["write_scale"] - 1.0) < 1e-12
    mid = d["kinds"]["sep_mid_k_f32"]
    assert mid["dispatches"] == 2 and mid["layout"] == 1
    assert mid["fetch_bytes"] == 1050.0 * 1024 * 2 and mid["write_bytes"] == 400.0 * 1024
    assert d["kinds"]["sep_part1_x_f32"]["layout"] == 1
    assert d["kinds"]["sep_part1_y_f32"]["layout"] == 0
    assert d["source_hash"] == traffic.source_hash()


def test_load_checks_sources_and_variant(tmp_path):
    d, out = _make(tmp_path)
    want = d["kinds"]["sep_mid_k_f32"]["bytes_per_launch"]
    assert traffic.load("wl", "sep_mid_k_f32", 1, path=str(out)) == want
    assert traffic.load("wl", "sep_mid_k_f32", None, path=str(out)) == want
    assert traffic.load("wl", "sep_mid_k_f32", 0, path=str(out)) is None
    assert traffic.load("wl", "sep_mid_k_f64", 1, path=str(out)) is None
    stale = json.loads(out.read_text())
    stale["source_hash"] = "0" * 16
    out.write_text(json.dumps(stale))
    assert traffic.load("wl", "sep_mid_k_f32", 1, path=str(out)) is None
    assert traffic.load("absent", "sep_mid_k_f32", path=str(tmp_path / "none.json")) is None


def test_variant_parsing():
    assert traffic._variant(MID.replace("(anonymous namespace)::", "")) == 1
    assert traffic._variant(Y1_G8) == 0
    assert traffic._variant("k_rmid<fcrkpm::G16, 2, 3, 3>") == 3
    assert traffic._variant("k_rmid2<fcrkpm::G16L, 1>") == 1
    assert traffic._variant("k_cg_xr<float>") is None
    assert traffic._variant("k_smid<fcrkpm::G32, float>") == 1
    assert traffic._variant("k_smid<fcrkpm::GPQ<16, 16>, float>") == 0
    assert traffic._variant("k_rpass<fcrkpm::GPQ<10, 8>, fcrkpm::Lin3, 1, x>") == 1
    assert traffic._variant("k_rpass<fcrkpm::GPQ<5, 16>, fcrkpm::Lin3, 1, x>") == 0


SMID = ("void fcrkpm::(anonymous namespace)::k_smid<fcrkpm::(anonymous namespace)::G16, float>"
        "(fcrkpm::(anonymous namespace)::SArgs<float>)")
X1_T = ("void fcrkpm::(anonymous namespace)::k_rpass<fcrkpm::(anonymous namespace)::G16, "
        "fcrkpm::(anonymous namespace)::Lin3, 1, true, true, false, 1, 0, true, float>(x)")
X1_64 = ("void fcrkpm::(anonymous namespace)::k_rpass<fcrkpm::(anonymous namespace)::G16L, "
         "fcrkpm::(anonymous namespace)::Lin3, 1, true, true, false, 1, 0, false, double>(x)")
Y1_GPQ = ("void fcrkpm::(anonymous namespace)::k_rpass<fcrkpm::(anonymous namespace)::GPQ<6, 16>, "
          "fcrkpm::(anonymous namespace)::Lin3, 1, false, false, false, 1, 1, false, float>(x)")


def test_templated_kernel_names(tmp_path):
    copy_kib = traffic.COPY_BYTES / 1024
    _csv(tmp_path / "f.csv", "FETCH_SIZE",
         [("__amd_rocclr_copyBuffer", copy_kib / 2), (SMID, 1000.0), (X1_T, 500.0), (X1_64, 800.0),
          (Y1_GPQ, 300.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE",
         [("__amd_rocclr_copyBuffer", copy_kib), (SMID, 400.0), (X1_T, 300.0), (X1_64, 600.0),
          (Y1_GPQ, 100.0)])
    out = tmp_path / "t.json"
    d = traffic.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), "wl", "cmd")
    assert d["kinds"]["sep_mid_k_f32"]["layout"] == 1
    assert d["kinds"]["sep_part1_x_f32"]["layout"] == 1
    assert d["kinds"]["sep_part1_x_f64"]["fetch_bytes"] == 800.0 * 1024 * 2
    assert d["kinds"]["sep_part1_y_f32"]["layout"] == 0
    # the line-constant middle pass matches both tile counts of its layout
    want = d["kinds"]["sep_mid_k_f32"]["bytes_per_launch"]
    assert traffic.load("wl", "sep_mid_k_f32", 1, path=str(out)) == want
    assert traffic.load("wl", "sep_mid_k_f32", 3, path=str(out)) == want
    assert traffic.load("wl", "sep_mid_k_f32", 0, path=str(out)) is None

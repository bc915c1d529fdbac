"""Host-side measurement tools: the per-block instruction counter of an AMD
assembly listing, the reducer of rocprofv3 counter CSVs to per-launch
profiles, and bench.py's issue-slot roofline arithmetic."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1402_2773_amd import isa_blocks  # noqa: E402
from synth import codes  # noqa: E402

ASM = """\
\t.text
_Z3fooPi:                               ; @_Z3fooPi
; %bb.0:
\tv_mov_b32_e32 v0, 0
\ts_mov_b32 s0, 0
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
\tv_add_u32_e32 v0, 1, v0
\tds_read_b32 v1, v2
\tglobal_load_dword v3, v[4:5], off
\ts_cbranch_scc1 .LBB0_1
; %bb.2:
\tv_mul_f32_e32 v0, v0, v0
\ts_endpgm
_Z3barPi:                               ; @_Z3barPi
\tv_nop
\ts_endpgm
"""


def test_isa_blocks_counts_each_block(tmp_path):
    f = tmp_path / "k.s"
    f.write_text(ASM)
    bl = isa_blocks.blocks(isa_blocks.function_lines(str(f), "foo"))
    by = {b["label"]: b for b in bl}
    assert [b["label"] for b in bl] == ["entry", "0", "1", "2"]
    assert (by["0"]["v"], by["0"]["s"]) == (1, 1)
    assert (by["1"]["v"], by["1"]["lds"], by["1"]["mem"], by["1"]["s"]) == (1, 1, 1, 1)
    assert by["1"]["branches"] == ["scc1>1"] and "Depth=1" in by["1"]["note"]
    assert (by["2"]["v"], by["2"]["s"]) == (1, 1)  # the listing ends at s_endpgm
    # the second function is not part of the first
    assert sum(b["v"] for b in bl) == 3


def _write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Workgroup_Size", "Counter_Name", "Counter_Value"])
        # rocprofv3 names each dispatch's threads per workgroup in its rows
        w.writerows([(d, k, 1024 if "<1, 4," in k else 256, c, v) for d, k, c, v in rows])


def test_profile_summary_medians_and_copy_scaling(tmp_path):
    k14 = "void ngdbf::decode_kernel<1, 4, 0, false, true, 0>(ngdbf::DecodeArgs)"
    k44 = "void ngdbf::decode_kernel<4, 4, 0, false, true, 0>(ngdbf::DecodeArgs)"
    cls = tmp_path / "c.csv"
    # counters split over two dimensions are summed per dispatch; the median
    # over a kernel's dispatches is its per-launch figure
    _write_counters(cls, [
        (1, k14, "SQ_INSTS_VALU", 4), (1, k14, "SQ_INSTS_VALU", 6), (1, k14, "GRBM_GUI_ACTIVE", 8),
        (2, k14, "SQ_INSTS_VALU", 30), (2, k14, "GRBM_GUI_ACTIVE", 8),
        (3, k14, "SQ_INSTS_VALU", 20), (3, k14, "GRBM_GUI_ACTIVE", 9),
        (4, k44, "SQ_INSTS_VALU", 7), (4, k44, "GRBM_GUI_ACTIVE", 1),
        (5, "some_other_kernel", "SQ_INSTS_VALU", 99),
    ])
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fetch, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0),
                            (2, k14, "FETCH_SIZE", 100.0), (3, k44, "FETCH_SIZE", 10.0)])
    _write_counters(write, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0),
                            (2, k14, "WRITE_SIZE", 50.0), (3, k44, "WRITE_SIZE", 5.0)])
    iss = tmp_path / "i.csv"
    _write_counters(iss, [(1, k14, "SQ_ACTIVE_INST_VALU", 21), (1, k14, "SQ_ACTIVE_INST_VALU2", 5),
                          (1, k14, "GRBM_GUI_ACTIVE", 8)])
    out = subprocess.run([sys.executable, "-m", "paper_1402_2773_amd.profile_summary", "--workload", "mix4",
                          "--classes", str(cls), "--issue", str(iss), "--fetch", str(fetch), "--write", str(write),
                          "--copy-bytes", "1024"], cwd=ROOT, capture_output=True, text=True, check=True)
    d = json.loads(out.stdout)
    assert d["kernel_sources_sha256"] == bench.kernel_sources_digest()
    c1008, c4000 = d["instances"]["C1008"], d["instances"]["C4000"]
    assert c1008["SQ_INSTS_VALU"] == 20 and c1008["GRBM_GUI_ACTIVE"] == 8
    assert d["dispatches_per_instance"] == {"C1008": 3, "C4000": 1}
    # 1024 bytes copied read 512 FETCH units and 1024 WRITE units
    assert d["copy_calibration"]["fetch_bytes_per_unit"] == 2.0
    assert d["copy_calibration"]["write_bytes_per_unit"] == 1.0
    assert (c1008["fetch_bytes"], c1008["write_bytes"], c1008["traffic_bytes"]) == (200.0, 50.0, 250.0)
    assert c4000["traffic_bytes"] == 25.0
    assert (c1008["SQ_ACTIVE_INST_VALU"], c1008["SQ_ACTIVE_INST_VALU2"]) == (21, 5)
    assert "SQ_ACTIVE_INST_VALU" not in c4000
    assert "C96" not in d["instances"]
    assert c1008["workgroup_size"] == 1024 and c4000["workgroup_size"] == 256


def test_issue_slots_count_dual_issued_pairs_once():
    # 100 instructions issued, 30 of the 4-clock slots held two of them
    c = {"SQ_INSTS_VALU": 100.0, "SQ_ACTIVE_INST_VALU": 100.0, "SQ_ACTIVE_INST_VALU2": 30.0}
    assert bench.issue_slots(c) == pytest.approx(70.0)
    assert bench.issue_slots({"SQ_INSTS_VALU": 100.0}) is None
    assert bench.PEAK_ISSUE_TSLOTS == pytest.approx(256 * 4 * 2.4e9 / 4 * 64 / 1e12)


def test_roofline_fractions():
    code = codes.named_code("C1008")
    frames, ms = 1000, 2.0
    c = {"SQ_INSTS_VALU": 1e9, "SQ_ACTIVE_INST_VALU": 1.01e9, "SQ_ACTIVE_INST_VALU2": 2.5e8,
         "traffic_bytes": 5e6, "source": "test"}
    r = bench.roofline(code, frames, "f32", ms, 1e9, c, False, "k")
    slots = 1.01e9 - 2.5e8
    assert r["achieved"] == pytest.approx(slots * 64 / 2e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["dual_issued_fraction"] == pytest.approx(0.5)
    per_frame = 4 * code.n + (code.n + 7) // 8 + 4 + 1
    assert r["algorithmic_bytes"] == frames * per_frame
    assert r["hbm_frac"] == pytest.approx(frames * per_frame / 2e-3 / 8e12)
    assert r["traffic"] == 5e6 and r["bound"] == "alu"
    # the method's LDS ratio: bit-iterations/s against 256 CUs x 32 banks x
    # 2.4 GHz / (2 d_v); no LDS counters, no busy fraction
    assert r["lds_method_ratio"] == pytest.approx(1e9 / 2e-3 / (256 * 32 * 2.4e9 / 6))
    assert r["lds_busy_frac"] is None
    # LDS busy: SQ_LDS_IDX_ACTIVE over GRBM_GUI_ACTIVE x 32 CUs per XCD
    rl = bench.roofline(code, frames, "f32", ms, 1e9,
                        {**c, "lds": {"SQ_LDS_IDX_ACTIVE": 16.0, "GRBM_GUI_ACTIVE": 2.0}}, False, "k")
    assert rl["lds_busy_frac"] == pytest.approx(0.25)
    # without a profile of the current kernel the counter figures are null
    r0 = bench.roofline(code, frames, "f32", ms, 1e9, None, False, "k")
    assert r0["frac"] is None and r0["traffic"] is None and r0["hbm_frac"] == r["hbm_frac"]
    assert r0["lds_busy_frac"] is None

"""Host logic of bench.py (CPU): the stored counter figures are used only while
they were taken on the current kernel source, and the roofline arithmetic."""
import json

import bench


def test_particle_kernel_bytes():
    # 24 B of state read and written per particle, 6 seen-field reads and 3
    # current writes of 4 B per cell
    assert bench.particle_kernel_bytes(10, 3) == 2 * 24 * 10 + 9 * 4 * 3
    assert bench.particle_kernel_bytes(10, 3, word=8, state_bytes=44) == 2 * 44 * 10 + 9 * 8 * 3


def test_stored_counters_follow_the_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    sha = bench.kernel_sha()
    (tmp_path / "t.json").write_text(json.dumps({"kernel_source_sha": sha, "hbm_bytes_per_launch": 123.0}))
    assert bench.stored_traffic("t.json") == 123.0
    (tmp_path / "t.json").write_text(json.dumps({"kernel_source_sha": "0" * 16, "hbm_bytes_per_launch": 123.0}))
    assert bench.stored_traffic("t.json") is None
    assert bench.stored_traffic("missing.json") is None
    doc = {"kernel_source_sha": sha, "cases": {"w": {"valu_lane_instr_per_particle": 200.0}}}
    (tmp_path / "valu_k_particles.json").write_text(json.dumps(doc))
    v = bench.valu_issue("w", 1000, 1e-3)          # 2e5 lane instructions in 1 us
    assert v["bound"] == "alu" and abs(v["achieved"] - 0.2) < 1e-12
    assert abs(v["frac"] - 2e11 / bench.VALU_PEAK_LANE_INSTR) < 1e-15
    assert bench.valu_issue("other", 1000, 1e-3) is None
    doc["kernel_source_sha"] = "0" * 16
    (tmp_path / "valu_k_particles.json").write_text(json.dumps(doc))
    assert bench.valu_issue("w", 1000, 1e-3) is None


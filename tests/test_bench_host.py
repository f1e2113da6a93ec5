"""Host logic of bench.py (CPU): the stored counter figures are used only while
they were taken on the current kernel source, and the roofline arithmetic."""
import json

import bench


def test_particle_kernel_bytes():
    # 24 B of state read and written per particle, 6 seen-field reads and 3
    # current writes of 4 B per cell
    assert bench.particle_kernel_bytes(10, 3) == 2 * 24 * 10 + 9 * 4 * 3
    assert bench.particle_kernel_bytes(10, 3, word=8, state_bytes=44) == 2 * 44 * 10 + 9 * 8 * 3


def test_step_bytes_of_the_batch():
    # 8 ppc: 48 B of particle state and 24 words of 4 B per cell shared by 8 particles
    assert bench.step_bytes(8, 1) == 2 * 24 * 8 + 24 * 4
    assert bench.step_bytes(8, 1) / 8 == 60


def test_batch_is_64_instances_accepted_by_the_oracle():
    insts = bench.batch_instances(bench._oracle_accepts)
    assert len(insts) == 64
    assert len({w["name"] for w in insts}) == 64
    assert all(0.3 <= w["alpha"] <= 0.7 and w["ppc"] == 8 for w in insts)


def test_gpus_above_one_exit_with_a_message():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_stored_counters_follow_the_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    sha = bench.kernel_sha()
    (tmp_path / "t.json").write_text(json.dumps({"kernel_source_sha": sha, "hbm_bytes_per_launch": 123.0}))
    assert bench.stored_traffic("t.json") == (123.0, "profiles/t.json")
    (tmp_path / "t.json").write_text(json.dumps({"kernel_source_sha": "0" * 16, "hbm_bytes_per_launch": 123.0}))
    assert bench.stored_traffic("t.json") == (None, None)
    assert bench.stored_traffic("missing.json") == (None, None)
    doc = {"kernel_source_sha": sha, "cases": {"w": {"valu_lane_instr_per_particle": 200.0}}}
    (tmp_path / "valu_k_particles.json").write_text(json.dumps(doc))
    v = bench.valu_issue("w", 1000, 1e-3)          # 2e5 lane instructions in 1 us
    assert v["bound"] == "alu" and abs(v["achieved"] - 0.2) < 1e-12
    assert abs(v["frac"] - 2e11 / bench.VALU_PEAK_LANE_INSTR) < 1e-15
    assert bench.valu_issue("other", 1000, 1e-3) is None
    doc["kernel_source_sha"] = "0" * 16
    (tmp_path / "valu_k_particles.json").write_text(json.dumps(doc))
    assert bench.valu_issue("w", 1000, 1e-3) is None



def test_tune_cache_has_the_timed_workloads():
    # the shipped cache (written by `bench.py --tune` on the GPU) holds a pick for
    # the headline batch and the adjoint workload, and keys tell schemes apart
    import pic_inputs as pi
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd import tune
    wls = bench.batch_instances(lambda c: L.pic_psi_coeffs(L.PIC_GALERKIN, c["alpha"], 4)[0] == L.PIC_OK)
    for w, prec in ((wls, "fp32"), ([pi.workload("beam2d_256_adjoint")], "fp32"),
                    ([pi.workload("beam3d_128x128x256")], "fp32"),
                    ([pi.workload("beam2d_512", alpha=0.5, precision="fp64")], "fp64")):
        pick = tune.lookup(w, prec)
        assert pick is not None, tune.key(w, prec)
        assert len(pick["tile"]) == 3 and pick["block"] in (256, 512) and pick["schedule"] in ("batched", "plain")
        assert set(pick["options"]) <= {"seen_tile_z", "yee_tile_z", "particle_defer", "particle_prefetch",
                                        "particle_waves4", "resort_every"}
    base = pi.workload("beam2d_512", alpha=0.5)
    keys = {tune.key([pi.workload("beam2d_512", alpha=0.5, **kw)], "fp32")
            for kw in ({}, {"interp": "uniform"}, {"solver": "ck"}, {"correction": "ratio"}, {"correction": False})}
    assert len(keys) == 5 and tune.key([base], "fp32") != tune.key([base], "fp64")
    assert tune.lookup([base], "fp32", cache=None) is None

"""CPU tests of bench.py's work model (the algorithmic counts its roofline
figures divide by) and of its refusal to run on more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pass_a_slots_scale_with_the_disk_rows():
    # 2r - 1 rows, two prefix reads each, plus one: 19 at r = 5, 31 at r = 8
    assert bench.pass_a_slots("f16", 5) == 122
    assert bench.pass_a_slots("f16", 8) == 134
    assert bench.pass_a_slots("f64", 8) - bench.pass_a_slots("f64", 5) == 12


def test_step_bound_counts_algorithmic_work_only():
    # the larger of the step's VALU time and the HBM time of the state read
    # and written (8 B per FP16 update); the two-pass spill is not counted
    assert bench.STATE_BYTES == {"f64": 32, "f32": 16, "f16": 8, "bf16": 8}
    for dt in ("f64", "f32", "f16", "bf16"):
        v = (bench.pass_a_slots(dt, 5) + bench.RESAMPLE_SLOTS) / bench.PEAK_LANE_OPS
        m = bench.STATE_BYTES[dt] / bench.PEAK_HBM
        one = max(v, m)
        assert abs(bench.step_bound_s(dt, 5, 1) - one) < 1e-24
        assert abs(bench.step_bound_s(dt, 5, 1 << 20) - (1 << 20) * one) < 1e-15
        # every mode's step is VALU-bound on its algorithmic work
        assert v > m
    # 130 slots per FP16 update at r = 5: 3.47 us for 2^20 particles
    assert abs(bench.step_bound_s("f16", 5, 1 << 20) - 130 * (1 << 20) / bench.PEAK_LANE_OPS) < 1e-15


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_ablation_variants_are_valid_step_parameters():
    # every row of the naive-vs-optimised table must name a variant the
    # binding accepts (the table is only exercised on a GPU otherwise)
    import paper_2308_00763_amd as pf
    assert bench.ABLATION and bench.ABLATION[0] == ("optimised", {})
    names = [name for name, _ in bench.ABLATION]
    assert len(set(names)) == len(names)
    for _, var in bench.ABLATION:
        p = pf.make_params(1 << 20, 1024, 1024, "f16", **var)
        assert pf.pf_workspace_bytes(p) > 0

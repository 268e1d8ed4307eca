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


def test_step_bound_is_pass_a_roof_plus_pass_c_bytes():
    for dt in ("f64", "f32", "f16", "bf16"):
        a = max(bench.pass_a_slots(dt, 5) / bench.PEAK_LANE_OPS, bench.PASS_A_BYTES[dt] / bench.PEAK_HBM)
        one = a + bench.PASS_C_BYTES[dt] / bench.PEAK_HBM
        assert abs(bench.step_bound_s(dt, 5, 1) - one) < 1e-24
        assert abs(bench.step_bound_s(dt, 5, 1 << 20) - (1 << 20) * one) < 1e-15
    # every pass-A roof here is the VALU's; FP64 moves the most bytes
    assert bench.PASS_C_BYTES["f64"] > bench.PASS_C_BYTES["f32"] > bench.PASS_C_BYTES["f16"]


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
        assert p.n_particles == 1 << 20

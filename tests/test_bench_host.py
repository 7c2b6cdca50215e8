"""bench.py's host-side contract: one GPU only (a request for more exits with
a message and status 2, before any device work), and the instruction counts
its ALU rooflines are priced with are consistent with their definitions."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert p.returncode == 2, (p.returncode, p.stdout, p.stderr)
    assert "one GPU" in p.stdout + p.stderr
    assert '"metric"' not in p.stdout


def test_alu_roofline_constants():
    import bench
    # Huygens: 90 VALU instructions per 2 pairs, one v_rsq_f32 and one
    # v_rcp_f32 per pair, each taking four issue slots
    assert bench.HUYGENS_OPS == 45
    assert bench.HUYGENS_TRANSCENDENTALS == 2
    assert bench.HUYGENS_SLOTS == 45 + 2 * 3
    # the fit step's two loops, per pair
    assert bench.SINUSOID_FIT_OPS == (22.5, 27.125)
    # the peak: 256 CUs x 128 lanes x 2.4 GHz, one op per lane per instruction
    assert abs(bench.VALU_PEAK_TOPS - 256 * 128 * 2.4e9 / 1e12) < 0.1
    r = bench.alu_roofline(39.325, 45, 70.0)
    assert r["bound"] == "alu" and abs(r["frac"] - 0.5) < 1e-3

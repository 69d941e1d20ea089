"""bench.py's command line without a GPU: more than one GPU is refused with a
message, and the traffic figure is read only for the kernel source it was
measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stdout


def test_traffic_only_for_the_profiled_kernel_source(monkeypatch, tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    got = bench.measured_traffic(1)
    assert got is None or got > 5.9e8          # at least the algorithmic bytes of one launch
    # a different kernel source (another root with a changed kernel) reads no figure
    csrc = tmp_path / "paper_1307_5310_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("residual_kernel.h", "residual_inst.hip"):
        text = open(os.path.join(ROOT, "paper_1307_5310_amd", "csrc", f)).read()
        (csrc / f).write_text(text + ("\n// changed\n" if f == "residual_inst.hip" else ""))
    (tmp_path / "profiles").mkdir()
    prof = "residual_apply_cavity32_p4q3_hbm_traffic.md"
    (tmp_path / "profiles" / prof).write_text(open(os.path.join(ROOT, "profiles", prof)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(1) is None

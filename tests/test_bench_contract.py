"""Host-side contract of bench.py (no GPU): more than one GPU is refused with a message, and
the measured HBM traffic of the cyclic-reduction kernel is reported only while the kernel
source is the one the counters were taken on."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_follows_the_kernel_source(tmp_path):
    """A traffic record is used only for the kernel source whose SHA-256 it carries."""
    import hashlib
    bench = _bench_module()
    src = open(os.path.join(ROOT, "paper_2105_11993_amd", "csrc", "kernels_prec.hip"), "rb").read()
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_2105_11993_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "kernels_prec.hip").write_bytes(src)
    rec = {"hbm_bytes_per_launch": 7.0e7, "kernels_prec_sha256": hashlib.sha256(src).hexdigest()}
    (tmp_path / "profiles" / "k_bcr_mfma_c2_traffic.json").write_text(json.dumps(rec))
    bench.ROOT = str(tmp_path)
    assert bench.measured_traffic(63.5e6) == 7.0e7
    # the source differs by one byte: no traffic figure
    (csrc / "kernels_prec.hip").write_bytes(src + b"\n")
    assert bench.measured_traffic(63.5e6) is None
    # no record at all: none either
    (tmp_path / "profiles" / "k_bcr_mfma_c2_traffic.json").unlink()
    assert bench.measured_traffic(63.5e6) is None

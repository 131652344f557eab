"""bench.py's command line without a GPU: more than one GPU is refused with a message and a
non-zero status (the benchmark runs one process on one GPU)."""
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, cwd=ROOT,
                         timeout=300)
    assert out.returncode == 2
    assert "one GPU only" in out.stdout and "--gpus 2" in out.stdout

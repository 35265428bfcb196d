"""The library shares PyTorch's HIP runtime whatever the import order (no GPU needed).

One process holds one working HSA runtime: if the library mapped the system's
HIP runtime beside the one a PyTorch ROCm wheel carries, whichever started
second would find no device.  Checked in a fresh interpreter that imports the
binding before anything else."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_1210_5128_amd import bnos  # first: before any explicit torch import
import torch  # noqa: F401
hip = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l})
hsa = sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libhsa-runtime64' in l})
print(len(hip), len(hsa))
"""


def test_binding_maps_one_hip_runtime():
    out = subprocess.run([sys.executable, "-c", PROBE, ROOT], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout

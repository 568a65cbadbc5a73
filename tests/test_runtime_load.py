"""The Python binding must leave a process with ONE HIP runtime.

torch ships its own HIP runtime; a library opened before torch would bind to
the system one, and torch would then load a second runtime for the same GPU.
The binding imports torch first, so whichever order a program uses, the
library binds to torch's runtime.  Checked here on the CPU (no GPU needed):
loading libraries maps them whether or not a device is present.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import sys
import paper_1811_08282_amd as sw
if sys.argv[1] == 'library_first':
    sw.load()
    import torch
else:
    import torch
    sw.load()
maps = set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)
print(len(maps))
"""


@pytest.mark.parametrize("order", ["library_first", "torch_first"])
def test_one_hip_runtime_per_process(order):
    pytest.importorskip("torch")
    env = dict(os.environ, PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", PROBE, order], env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1", (order, out.stdout)

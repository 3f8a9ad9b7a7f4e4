"""The binding binds the library to torch's HIP runtime whatever the
caller imported first: a fresh interpreter that calls into the library
before importing torch still finds torch loaded, and the library's HIP
runtime is the copy torch ships (one runtime in the process)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r'''
import sys
sys.path.insert(0, sys.argv[1])
from paper_1911_08158_amd import binding
assert "torch" not in sys.modules
n = binding.workspace_bytes(binding.Params.of(None, problem="pwave", nelem=(8, 8, 8), p=2, tau=0.01))
assert n > 0 and "torch" in sys.modules
import os, torch
lib = os.path.realpath(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
maps = open("/proc/self/maps").read()
hip = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
print(sorted(hip))
assert len(hip) == 1, hip
'''


def test_library_binds_to_torch_runtime_when_loaded_first():
    r = subprocess.run([sys.executable, "-c", PROBE, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr

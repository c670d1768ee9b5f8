"""The HIP library and torch share one HIP runtime in the process."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_binds_to_the_runtime_torch_loaded():
    # load the library before anything imports torch explicitly; the loader
    # must still end with a single libamdhip64 mapped into the process
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1503_08718_amd import load\n"
        "load()\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
        "print(len(libs), libs)\n"
        "assert len(libs) == 1, libs\n" % ROOT
    )
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr


def test_missing_library_is_an_error_not_a_fallback():
    # with the shared library absent the binding raises; nothing computes on the CPU instead
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1503_08718_amd import _lib\n"
        "_lib.LIB_PATH = '/nonexistent/libmrtlbm.so'\n"
        "try:\n"
        "    _lib.load()\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % ROOT
    )
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and "not built" in out.stdout, out.stdout + out.stderr

"""The product path has no CPU fallback: the package never imports the oracle,
and without its HIP library the binding raises instead of computing anything."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2510_19764_amd")


def test_package_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), f


def test_missing_library_raises():
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2510_19764_amd import build, binding\n"
        "build.LIB = '/nonexistent/libragsnn.so'\n"
        "def no_build(*a, **k):\n"
        "    raise RuntimeError('library missing')\n"
        "build.build = no_build\n"
        "try:\n"
        "    binding.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "raised library missing" in r.stdout, r.stdout + r.stderr

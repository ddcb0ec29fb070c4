"""The HIP library builds for gfx950, loads on a host without a GPU, and
exports every entry point include/ragsnn.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ragsnn.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    from paper_2510_19764_amd import binding
    assert declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2510_19764_amd import binding, build
    if not os.path.exists(build.LIB) or build.stale():
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", build.LIB], capture_output=True, text=True, check=True).stdout
    syms = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [s for s in declared() if s not in syms]
    assert not missing, missing
    L = ctypes.CDLL(build.LIB)
    for s in declared():
        assert hasattr(L, s)


def test_last_error_is_empty_string_initially():
    from paper_2510_19764_amd import binding
    L = binding.lib()
    assert isinstance(L.rs_last_error(), bytes)


def test_invalid_params_rejected_without_gpu_work():
    # validation happens before any device call
    from paper_2510_19764_amd import binding
    cfg = binding.EpropConfig(n_in=10, n_rec=0, n_out=2, batch=1)
    h = ctypes.c_void_p()
    code = binding.lib().rs_eprop_create(ctypes.byref(cfg.c()), None, ctypes.byref(h))
    assert code == binding.RS_EINVAL and not h.value
    assert b"n_rec" in binding.lib().rs_last_error()

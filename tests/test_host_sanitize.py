"""The library's host layer (context, argument and batch checks, staging,
checkpoint save and load) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host_sanitize/host_abi_check, the host code
of csrc/tlda_api.hip instrumented (device code as usual), built by
__graft_entry__.build() through tests/host_sanitize/build.py.  The checkpoint
loader is fed truncations of a valid checkpoint, each in a buffer of exactly
that length, so a read past the given length is reported as a heap overflow.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "host_sanitize", "_build", "host_abi_check")
# leaks of the HIP runtime's own allocations at exit are not the library's
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(mode):
    assert os.path.exists(EXE), "host_abi_check is not built: run __graft_entry__.build()"
    r = subprocess.run([EXE, mode], env=ENV, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.returncode == 0, out
    assert f"host_abi_check {mode}: 0 failed expectations" in r.stdout, out


def test_host_layer_under_sanitizers_without_device():
    """Status strings (any int), configuration checks and a context request
    that fails cleanly without a device (on a GPU host it succeeds).  Builds
    the driver first if it is missing (on the CPU, like the library test)."""
    if not os.path.exists(EXE):
        import importlib.util

        from paper_2511_07809_amd.build import build as lib_build
        lib_build()
        spec = importlib.util.spec_from_file_location(
            "host_sanitize_build", os.path.join(HERE, "host_sanitize", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    _run("cpu")


@pytest.mark.gpu
def test_host_layer_under_sanitizers_on_device():
    """Argument checks on a live context, staging from pinned host memory,
    moments, a refresh and a step, then the checkpoint round trip,
    truncations and corrupted headers."""
    _run("gpu")

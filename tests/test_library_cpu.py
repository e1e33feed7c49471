"""Host-only checks of the C ABI: the library loads, exports every function
the header declares, and its structs have the header's layout.  No call here
touches a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlda.h")
LIB = os.path.join(ROOT, "paper_2511_07809_amd", "libtlda.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tlda_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2511_07809_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_every_declared_function_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2511_07809_amd import tlda
    assert sorted(tlda.EXPORTED) == names


def test_status_strings(lib):
    lib.tlda_status_str.restype = ctypes.c_char_p
    lib.tlda_status_str.argtypes = [ctypes.c_int]
    assert lib.tlda_status_str(0) == b"ok"
    assert lib.tlda_status_str(3) == b"invalid CSR content"
    assert lib.tlda_status_str(99) == b"unknown status"
    lib.tlda_last_error.restype = ctypes.c_char_p
    lib.tlda_last_error.argtypes = [ctypes.c_void_p]
    assert lib.tlda_last_error(None) == b""


def test_create_rejects_null_arguments_before_touching_a_device(lib):
    lib.tlda_create.restype = ctypes.c_int
    lib.tlda_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.tlda_create(None, None, None) == 1   # TLDA_ERR_ARG


def test_create_validates_config_before_touching_a_device(lib):
    from paper_2511_07809_amd import tlda
    lib.tlda_create.restype = ctypes.c_int
    lib.tlda_create.argtypes = [ctypes.POINTER(tlda.tlda_config), ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_void_p)]
    out = ctypes.c_void_p()

    def create(V, K, D, flags, alpha0=1.0, theta=0.0):
        cfg = tlda.tlda_config(V, K, D, flags, alpha0, theta, 0, 0, 0, 0)
        return lib.tlda_create(ctypes.byref(cfg), None, ctypes.byref(out))

    assert create(100, 10, 10, 0x8) == 1                       # unknown flag
    assert create(100, 10, 10, 0, alpha0=0.0) == 1             # alpha0 must be > 0
    assert create(100, 10, 10, 0, theta=-1.0) == 1             # theta must be >= 0
    assert create(2, 1, 1, 0) == 2                             # V < 3
    assert create(100, 10, 101, 0) == 2                        # D > V
    assert create(300, 257, 10, 0) == 2                        # K above the limit
    assert create(300, 10, 129, tlda.TLDA_BF16) == 2           # BF16 path: D <= 128
    assert create(300, 129, 10, tlda.TLDA_BF16) == 2           # BF16 path: K <= 128
    assert create(300, 10, 129, tlda.TLDA_CLASSIC) == 2        # classic rung: D <= 128
    assert create(300, 129, 10, tlda.TLDA_CLASSIC) == 2        # classic rung: K <= 128
    cfg = tlda.tlda_config(1000, 10, 10, 0, 1.0, 0.0, 0, 513, 0, 0)   # subspace width <= 512
    assert lib.tlda_create(ctypes.byref(cfg), None, ctypes.byref(out)) == 2
    assert out.value is None
    lib.tlda_set_timing_events.restype = ctypes.c_int
    lib.tlda_set_timing_events.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int]
    assert lib.tlda_set_timing_events(None, None, None, 0) == 1


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "tlda.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        " sizeof(tlda_config),"
        " offsetof(tlda_config, alpha0), offsetof(tlda_config, eig_iters),"
        " offsetof(tlda_config, eig_seed), offsetof(tlda_config, eig_warm_iters),"
        " sizeof(tlda_csr_batch),"
        " offsetof(tlda_csr_batch, row_ptr), offsetof(tlda_csr_batch, slot),"
        " offsetof(tlda_csr_batch, first_doc), sizeof(tlda_csr_batch_u16),"
        " offsetof(tlda_csr_batch_u16, first_doc));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    from paper_2511_07809_amd import tlda
    cfg, b, h = tlda.tlda_config, tlda.tlda_csr_batch, tlda.tlda_csr_batch_u16
    assert got == [ctypes.sizeof(cfg), cfg.alpha0.offset, cfg.eig_iters.offset,
                   cfg.eig_seed.offset, cfg.eig_warm_iters.offset, ctypes.sizeof(b),
                   b.row_ptr.offset, b.slot.offset, b.first_doc.offset, ctypes.sizeof(h),
                   h.first_doc.offset]


def test_header_compiles_as_c_and_cxx(tmp_path):
    for comp, ext in (("gcc", "c"), ("g++", "cpp")):
        src = tmp_path / f"h.{ext}"
        src.write_text('#include "tlda.h"\nint main(void){return TLDA_OK;}\n')
        subprocess.run([comp, "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(tmp_path / f"h_{ext}")], check=True)


def test_bench_runs_on_one_gpu_only():
    """bench.py --gpus N with N > 1 exits at once with a message (the
    benchmark measures one GPU's share; the sharding is a design note)."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stdout + r.stderr

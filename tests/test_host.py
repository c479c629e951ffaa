"""CPU-only checks of the C ABI library: it loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swalign.h")
LIB = os.path.join(ROOT, "paper_2208_12350_amd", "libswalign.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sw_create", "sw_destroy", "sw_last_error", "sw_align_batch", "sw_set_option"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libswalign.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n
    from paper_2208_12350_amd import binding
    assert set(binding.EXPORTED) == set(_declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libswalign.so not built")
def test_null_handle_is_rejected():
    from paper_2208_12350_amd import binding as B
    lib = B.load_library()
    assert lib.sw_align_batch(None, None, None, 1, None, None) == B.SW_EINVAL
    assert lib.sw_set_option(None, b"mode", 0) == B.SW_EINVAL
    assert lib.sw_last_error(None) == b"null handle"
    lib.sw_destroy(None)


def test_pool_allocator_native(tmp_path):
    """Device-pool bookkeeping used for serving admission, tested on the host."""
    import subprocess
    src = os.path.join(ROOT, "tests", "native", "pool_test.cpp")
    exe = str(tmp_path / "pool_test")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_2208_12350_amd", "csrc"),
                           src, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "pool ok" in out.stdout


PROBE_LIB = os.path.join(ROOT, "paper_2208_12350_amd", "libswprobe.so")


@pytest.mark.skipif(not os.path.exists(PROBE_LIB), reason="libswprobe.so not built")
def test_probe_library_exports_and_rejects_bad_arguments():
    lib = ctypes.CDLL(PROBE_LIB)
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "swprobe.h")).read(), flags=re.S)
    for n in set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)):
        assert hasattr(lib, n), n
    lib.sw_probe_valu.restype = ctypes.c_int
    v = ctypes.c_double(0)
    assert lib.sw_probe_valu(0, 9, 10, 1, ctypes.byref(v)) == -1       # unknown kind
    assert lib.sw_probe_valu(0, 0, 0, 1, ctypes.byref(v)) == -1        # no iterations
    assert lib.sw_probe_valu(0, 0, 10, 1, None) == -1


STENCIL_LIB = os.path.join(ROOT, "paper_2208_12350_amd", "libswstencil.so")


@pytest.mark.skipif(not os.path.exists(STENCIL_LIB), reason="libswstencil.so not built")
def test_stencil_library_exports_and_rejects_bad_arguments():
    lib = ctypes.CDLL(STENCIL_LIB)
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "swstencil.h")).read(), flags=re.S)
    names = set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text))
    from paper_2208_12350_amd import stencil
    assert names == set(stencil.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n
    L = stencil.load_library()
    # argument errors are reported before any launch
    assert L.sw_diffuse_padded(None, None, 4, 4, 6, 0.5, None) == -1
    assert L.sw_diffuse_padded(1, 2, 4, 4, 5, 0.5, None) == -1            # pitch < nx + 2
    assert L.sw_diffuse_padded(1, 2, 4, 4, 6, 1.5, None) == -1            # D outside [0, 1]
    assert L.sw_diffuse_checked(1, 2, 0, 4, 0.5, None) == -1
    assert L.sw_pad_grid(1, 2, 4, 4, 3, None) == -1


def test_bench_reads_committed_traffic_summaries():
    """bench.py takes roofline.traffic from the committed counter summaries:
    the dominant kernel of each summary is found under its profiled name
    (with or without the namespace), rescaled to another run's cells per
    launch, and ignored once the kernel sources no longer match."""
    import glob
    import bench
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "sweep_*_traffic.txt")))
    assert paths
    for path in paths:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        kernel, workload = kv["kernel"], kv["workload"]
        per_launch = float(kv["traffic_bytes_per_launch"])
        cells = float(kv["cells_per_launch"])
        sha = kv["sources_sha256"]
        assert bench.stored_traffic(kernel, workload, sha) == round(per_launch)
        assert bench.stored_traffic(kernel.replace("sw::", ""), workload, sha) == round(per_launch)
        assert bench.stored_traffic(kernel, workload, sha, cells_per_launch=cells / 2) == round(per_launch / 2)
        assert bench.stored_traffic(kernel, workload, "0" * 64) is None
        assert bench.stored_traffic(kernel, "no_such_workload", sha) is None

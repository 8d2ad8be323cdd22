"""C-ABI checks that need no GPU: the library loads, exports every symbol declared in
include/dtws.h, reports no device here, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re

import pytest

import paper_1812_10302_amd as dtws

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dtws.h")


def declared_symbols():
    text = open(HEADER).read()
    return re.findall(r"DTWS_API\s+[\w\s\*]+?\b(dtws_\w+)\s*\(", text)


def test_header_declares_the_boundary():
    names = set(declared_symbols())
    for must in ("dtws_create", "dtws_destroy", "dtws_search", "dtws_search_batch", "dtws_znorm_stats",
                 "dtws_lb_cascade", "dtws_dtw_band", "dtws_bsf_update", "dtws_strerror", "dtws_last_error",
                 "dtws_get_counters", "dtws_device_count"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = dtws.library()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_strerror():
    lib = dtws.library()
    assert lib.dtws_strerror(0) == b"ok"
    assert lib.dtws_strerror(dtws.ENODEV) == b"no HIP device"
    assert lib.dtws_strerror(12345) == b"unknown error"


def test_argument_errors_before_any_device_work():
    lib = dtws.library()
    h = ctypes.c_void_p()
    assert lib.dtws_create(0, 1000, 64, 1, None) == dtws.EINVAL
    assert lib.dtws_create(0, 1, 64, 1, ctypes.byref(h)) == dtws.EINVAL          # max_n < 2
    assert lib.dtws_create(0, 1000, 1, 1, ctypes.byref(h)) == dtws.EINVAL        # max_m < 2
    assert lib.dtws_create(0, 1000, 4096, 1, ctypes.byref(h)) == dtws.EINVAL     # max_m over the limit
    assert lib.dtws_create(0, 1 << 31, 64, 1, ctypes.byref(h)) == dtws.EINVAL    # max_n too large
    out = dtws.Match()
    assert lib.dtws_search(None, None, 100, None, 8, 1, 0, 0, None, ctypes.byref(out)) == dtws.EINVAL
    assert lib.dtws_dtw_band(None, None, 100, None, 8, 1, None, 4, 0.0, None, None) == dtws.EINVAL
    assert lib.dtws_bsf_update(None, None, None, None, 4, None) == dtws.EINVAL
    assert lib.dtws_get_counters(None, None) == dtws.EINVAL
    cfg = dtws.TrainCfg()
    assert lib.dtws_model_train(None, None, 100, ctypes.byref(cfg), None, None, None) == dtws.EINVAL
    size = ctypes.c_size_t(0)
    assert lib.dtws_model_save(None, None, ctypes.byref(size)) == dtws.EINVAL
    assert lib.dtws_model_load(None, None, 0) == dtws.EINVAL
    lib.dtws_destroy(None)   # accepted


@pytest.mark.skipif(dtws.device_count() > 0, reason="a HIP device is present")
def test_no_device_reports_enodev():
    assert dtws.device_count() == 0
    with pytest.raises(dtws.DtwsError) as e:
        dtws.Context(0, max_n=1000, max_m=64)
    assert e.value.code == dtws.ENODEV


def test_exports_are_only_the_c_abi():
    """Everything the shared object exports with a dtws_ prefix is declared in the header."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", dtws.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.split()[-1].startswith("dtws_")}
    assert exported == set(declared_symbols())


def test_single_hip_runtime_in_process():
    """The binding loads torch before libdtws.so, so exactly one HIP runtime is mapped."""
    import subprocess
    import sys
    code = ("import paper_1812_10302_amd as d; d.library(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT).stdout
    libs = eval(out.strip().splitlines()[-1])
    assert len(libs) == 1, libs

"""The C-ABI library without a GPU: it loads, exports every declared symbol,
and reports errors instead of computing (no compute calls are made here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpbatch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(lp_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1802_08557_amd import lpbatch
    return lpbatch.load()


def test_header_declares_the_binding_exports():
    from paper_1802_08557_amd import lpbatch
    assert declared_functions() == sorted(lpbatch.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_options_defaults(lib):
    from paper_1802_08557_amd.lpbatch import LPOptions
    o = LPOptions()
    o.precision = 7
    lib.lp_options_init(ctypes.byref(o))
    assert o.precision == 0 and o.k_deg == 50 and o.max_iters == 0 and o.flags == 0
    assert o.stats is None and o.stream is None and o.scaling == 0 and o.pricing == 0


def _c_layout(tmp_path, struct, fields):
    """sizeof and field offsets of a struct of lpbatch.h, from the C compiler."""
    src = tmp_path / f"layout_{struct}.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lpbatch.h"\nint main(void){'
                   f'printf("%zu", sizeof({struct}));'
                   + "".join(f'printf(" %zu", offsetof({struct}, {f}));' for f in fields)
                   + "return 0;}\n")
    exe = tmp_path / f"layout_{struct}"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    return [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]


@pytest.mark.parametrize("struct,cls", [("lp_options", "LPOptions"), ("lp_peaks", "LPPeaks")])
def test_struct_layouts_match_the_header(tmp_path, struct, cls):
    # The ctypes mirrors of lp_options and lp_peaks have the C structs' sizes and offsets.
    from paper_1802_08557_amd import lpbatch
    C = getattr(lpbatch, cls)
    fields = [f[0] for f in C._fields_]
    got = _c_layout(tmp_path, struct, fields)
    assert got[0] == ctypes.sizeof(C)
    assert got[1:] == [getattr(C, f).offset for f in fields]


def test_null_context_and_bad_arguments_are_errors(lib):
    from paper_1802_08557_amd import lpbatch
    assert lib.lp_batch_solve_ex(None, 1, *([None] * 9), None) == lpbatch.LP_ERR_ARG
    assert "ctx" in lpbatch.last_error()
    assert lib.lp_ctx_create(None, 0) == lpbatch.LP_ERR_ARG
    assert lib.lp_ctx_kernel_times(None, None, None, 0) == lpbatch.LP_ERR_ARG
    assert lib.lp_batch_scale(None, 1, *([None] * 5), 4, 0, *([None] * 6)) == lpbatch.LP_ERR_ARG
    assert lib.lp_measure_peaks(None, None) == lpbatch.LP_ERR_ARG


@pytest.mark.skipif(os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK),
                    reason="a GPU is present")
def test_without_gpu_context_creation_fails_cleanly(lib):
    from paper_1802_08557_amd import lpbatch
    h = ctypes.c_void_p()
    rc = lib.lp_ctx_create(ctypes.byref(h), 0)
    assert rc in (lpbatch.LP_ERR_HIP, lpbatch.LP_ERR_ARG)
    assert not h.value
    assert lpbatch.last_error() != ""


def test_header_enums_match_the_binding():
    # The binding's copies of the header's enum values (precision, placement,
    # pricing) and of the stats layout.
    from paper_1802_08557_amd import lpbatch
    text = open(HEADER).read()
    val = lambda name: int(re.search(r"\b" + name + r"\s*=\s*(-?\d+)", text).group(1))
    assert (lpbatch.PREC_FP64, lpbatch.PREC_FP32_CERT64) == (val("LP_PREC_FP64"), val("LP_PREC_FP32_CERT64"))
    assert (lpbatch.PRICE_DANTZIG, lpbatch.PRICE_STEEPEST_EDGE) == (val("LP_PRICE_DANTZIG"),
                                                                    val("LP_PRICE_STEEPEST_EDGE"))
    width = int(re.search(r"#define LP_STATS_WIDTH (\d+)", text).group(1))
    assert lpbatch.STATS_WIDTH == width


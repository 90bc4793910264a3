"""The C-ABI library loads and exports every entry point include/swmi.h declares (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swmi.h")
LIB = os.path.join(ROOT, "paper_1304_5966_amd", "libswmi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sw_score", "sw_align", "sw_batch", "sw_score_dev", "sw_context_create",
                 "sw_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libswmi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sw_\w+)", out))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libswmi.so not built")
def test_library_holds_gfx950_code_only():
    data = open(LIB, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-[a-z]*-(gfx[0-9a-z]+)", data))
    assert targets == {b"gfx950"}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libswmi.so not built")
def test_binding_reports_errors_without_gpu():
    from paper_1304_5966_amd import swmi
    assert "gfx950" in swmi.version()
    h = ctypes.c_void_p()
    st = swmi.lib.sw_context_create(0, None, ctypes.byref(h))
    assert st != swmi.SW_OK or h.value  # a context needs a GPU; either way no abort
    if st != swmi.SW_OK:
        assert swmi.lib.sw_last_error()
        assert swmi.lib.sw_score(None, b"A", 1, b"A", 1, None, None, None) == swmi.SW_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libswmi.so not built")
def test_batch_results_view_matches_the_result_structs():
    """BatchResults reads the library's sw_score_result array through a numpy view;
    its field layout must match the C struct field by field."""
    from paper_1304_5966_amd import swmi
    raw = (swmi.ScoreResult * 3)()
    for i, r in enumerate(raw):
        r.score, r.threshold, r.end_a, r.end_b = 10 * i + 1, i, 1000 + i, 2 ** 40 + i
        r.cells_computed, r.fallback = 3 ** 30 + i, i % 2
    res = swmi.BatchResults(raw, 3)
    assert len(res) == 3
    assert res[1] == swmi.Score(11, 1001, 2 ** 40 + 1, 3 ** 30 + 1, 1, 1)
    assert res[-1].key() == (21, 1002, 2 ** 40 + 2)
    assert [r.key() for r in res] == res.keys() == [(1, 1000, 2 ** 40), (11, 1001, 2 ** 40 + 1),
                                                   (21, 1002, 2 ** 40 + 2)]
    assert res[1:] == [res[1], res[2]]
    assert swmi.BatchResults((swmi.ScoreResult * 1)(), 0) == []

"""The C-ABI library loads and exports every symbol include/sdcsz.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2010_03144_amd import sdcsz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "sdcsz.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdcsz_[a-z_]+)\s*\(", text)))


def test_header_lists_the_binding_functions():
    assert declared() == sorted(sdcsz.FUNCTIONS)


@pytest.mark.skipif(not os.path.exists(sdcsz.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sdcsz.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(sdcsz.LIB_PATH), reason="library not built")
def test_size_queries_without_gpu():
    L = sdcsz.lib()
    p = sdcsz.make_params((512, 512, 512), True, (6, 6, 6), 1e-3)
    assert L.sdcsz_compress_workspace_size(ctypes.byref(p)) > 512**3 * 6
    assert L.sdcsz_max_compressed_size(ctypes.byref(p)) > 512**3 * 4
    bad = sdcsz.make_params((8, 8), True, (0, 8), 1e-3)
    assert L.sdcsz_compress_workspace_size(ctypes.byref(bad)) == 0
    assert sdcsz.strerror(sdcsz.ESDC) == "uncorrectable silent data corruption"

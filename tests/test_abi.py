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


@pytest.mark.skipif(not os.path.exists(sdcsz.LIB_PATH), reason="library not built")
def test_launch_shape_table_round_trip_and_validation():
    try:
        assert sdcsz.tune_set(3, 1, 0, [(1000, 64), (50000, 128)]) == sdcsz.OK
        assert sdcsz.tune_get(3, 1, 0) == [(1000, 64), (50000, 128)]
        assert sdcsz.tune_get(3, 0, 0) == []
        assert sdcsz.tune_set(0, 0, 0, [(10, 96)]) == sdcsz.EINVAL  # lanes 64, 128 or 256
        assert sdcsz.tune_set(0, 0, 0, [(10, 64), (10, 128)]) == sdcsz.EINVAL  # strictly ascending
        assert sdcsz.tune_set(4, 0, 0, []) == sdcsz.EINVAL
        assert sdcsz.tune_set(0, 2, 0, []) == sdcsz.EINVAL
        assert sdcsz.tune_set(0, 0, 2, []) == sdcsz.EINVAL
        assert sdcsz.tune_set(0, 0, 0, [(i + 1, 64) for i in range(sdcsz.TUNE_MAX + 1)]) == sdcsz.EINVAL
    finally:
        assert sdcsz.tune_set(3, 1, 0, []) == sdcsz.OK
    assert sdcsz.tune_get(3, 1, 0) == []


def test_tuner_table_from_measurements():
    from paper_2010_03144_amd import tune
    best = {256: 64, 1024: 64, 4096: 128, 16384: 256, 65536: 256}
    assert tune.entries_from_best(best) == [(2048, 64), (8192, 128), (tune.UNBOUNDED, 256)]
    assert tune.entries_from_best({256: 128}) == [(tune.UNBOUNDED, 128)]
    assert tune.pick({64: 0.97, 128: 0.99, 256: 1.0}) == 256  # within the noise margin
    assert tune.pick({64: 0.80, 128: 0.90, 256: 1.0}) == 64
    # the tuning fields have about the requested number of blocks, partial blocks included
    for block in ((6, 6, 6), (16, 16)):
        for n in tune.SIZES:
            shape = tune.class_shape(block, n)
            nb = 1
            for d, b in zip(shape, block):
                nb *= -(-d // b)
            assert 0.5 * n <= nb <= 2 * n, (block, n, shape, nb)

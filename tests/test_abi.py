"""C-ABI contract checks that need no GPU: the library loads, exports every
declared symbol, and its host-only entry points behave."""

import ctypes
import os
import re

import pytest

from paper_2404_01585_amd import flexis as fx
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "flexis.h")).read()
    return sorted(set(re.findall(r"^(?:fx_status|const char \*|uint64_t)\s*(fx_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fx.library_path()):
        pytest.skip("libflexis.so not built")
    return fx.load_library()


def test_exports_every_declared_symbol(lib):
    declared = _declared_symbols()
    assert set(declared) == set(fx.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_version(lib):
    assert b"gfx950" in lib.fx_version()


@pytest.mark.parametrize("sigma,lam,n", [(3, 1.0, 3), (2, 1.0, 3), (2, 0.25, 3), (375, 0.57, 5), (3550, 0.37, 7),
                                         (200, 0.3, 4), (2000, 0.1, 6), (1, 0.0, 16), (10 ** 15, 0.999999, 16)])
def test_tau_matches_oracle(lib, sigma, lam, n):
    assert fx.tau(sigma, lam, n) == O.tau(sigma, lam, n)


def test_tau_errors(lib):
    out = ctypes.c_int64(0)
    assert lib.fx_tau(5, 1.5, 3, ctypes.byref(out)) == fx.FX_EINVAL
    assert lib.fx_tau(5, -0.1, 3, ctypes.byref(out)) == fx.FX_EINVAL
    assert lib.fx_tau(5, 0.5, 0, ctypes.byref(out)) == fx.FX_EINVAL
    assert lib.fx_tau(-1, 0.5, 3, ctypes.byref(out)) == fx.FX_EINVAL
    assert lib.fx_tau(5, 0.5, 3, None) == fx.FX_EINVAL
    assert b"lambda" in lib.fx_last_error() or len(lib.fx_last_error()) > 0


def test_null_arguments(lib):
    assert lib.fx_ctx_create(None, None) == fx.FX_EINVAL
    assert lib.fx_ctx_destroy(None) == fx.FX_EINVAL
    assert lib.fx_graph_destroy(None) == fx.FX_EINVAL
    assert lib.fx_support(None, None, 1, 0.5, 0, None, None, 0) == fx.FX_EINVAL
    assert lib.fx_enumerate(None, None, None, 0, None) == fx.FX_EINVAL
    assert lib.fx_ctx_set(None, b"lanes", 1) == fx.FX_EINVAL
    assert lib.fx_ctx_get(None, b"lanes", None) == fx.FX_EINVAL
    assert lib.fx_support_noalloc(None, None, 1, 0.5, 0, None) == fx.FX_EINVAL


def test_result_layout_matches_header(lib):
    # the numpy view of fx_result used for batches has the ctypes struct's layout
    assert fx.RESULT_DTYPE.itemsize == ctypes.sizeof(fx.ResultC)
    for name, _ in fx.ResultC._fields_:
        assert fx.RESULT_DTYPE.fields[name][1] == getattr(fx.ResultC, name).offset, name


def test_bench_refuses_more_than_one_gpu():
    # the benchmark is single-GPU: asking for more exits with a message before
    # touching any device
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 2
    line = json.loads(out.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]

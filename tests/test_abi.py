"""The C ABI library builds, loads on the host and exports every function
declared in include/eqfmm.h (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eqfmm.h")
LIB = os.path.join(ROOT, "paper_2212_13080_amd", "libeqfmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eqfmm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libeqfmm.so is not built: run __graft_entry__.build()")
    import torch  # noqa: F401  (the library binds to the HIP runtime torch loads)
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("eqfmm_plan_create", "eqfmm_forward", "eqfmm_backward", "eqfmm_workspace_bytes",
                     "eqfmm_plan_destroy", "eqfmm_strerror"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_python_binding_wraps_every_symbol():
    from paper_2212_13080_amd import native
    assert sorted(native.EXPORTS) == declared_functions()


def test_host_only_calls(lib):
    # plan creation, sizes and error strings need no GPU
    from paper_2212_13080_amd import native
    p = native.Params()
    p.levels, p.order, p.boundary, p.precision, p.box = 3, 4, 3, 1, 1.0
    h = native.eqfmm_plan_create(p)
    assert native.eqfmm_plan_device_bytes(h) > 0
    assert native.eqfmm_workspace_bytes(h, 1000) > native.eqfmm_workspace_bytes(h, 10)
    native.eqfmm_plan_destroy(h)
    assert native.lib().eqfmm_strerror(-2).decode().startswith("position outside")
    bad = native.Params()
    bad.levels, bad.order, bad.box = 1, 4, 1.0
    with pytest.raises(native.EqfmmError) as e:
        native.eqfmm_plan_create(bad)
    assert e.value.code == -1
    bad.levels, bad.order, bad.split_d = 3, 4, 0.1      # 2d >= leaf side
    with pytest.raises(native.EqfmmError):
        native.eqfmm_plan_create(bad)


def test_bench_refuses_more_than_one_gpu():
    # bench.py measures one GPU; a request for more exits with a message
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

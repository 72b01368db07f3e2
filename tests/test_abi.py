"""The C-ABI library loads, exports every symbol its header declares, and validates
arguments on the host (no GPU needed: invalid calls return before any HIP call)."""
import ctypes
import os
import re

import pytest

from oracle import fmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fc2t2.h")
LIB = os.path.join(ROOT, "paper_2111_00110_amd", "libfc2t2.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfc2t2.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fc2t2_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (the binding loads torch's HIP runtime first)
    from paper_2111_00110_amd import fc2t2
    return fc2t2.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_multi_index_order_matches_checker(lib):
    from paper_2111_00110_amd import fc2t2
    for d in (2, 3):
        for K in range(0, 7):
            assert fc2t2.multi_indices(d, K) == fmm.multi_indices(d, K)
    assert lib.fc2t2_multi_indices(4, 2, None) == -1


def test_supported_orders(lib):
    assert lib.fc2t2_supported(2, 6) and lib.fc2t2_supported(3, 5)
    assert not lib.fc2t2_supported(3, 6) and not lib.fc2t2_supported(2, 0)


def test_status_strings(lib):
    for s in range(6):
        assert lib.fc2t2_status_string(s)


def test_plan_create_rejects_bad_arguments_on_host(lib):
    from paper_2111_00110_amd.fc2t2 import _Grid, _Kernel
    out = ctypes.c_void_p()
    good_g = _Grid(3, 64, -1.0, 1.0)
    good_k = _Kernel(0, 0.02, 0, None)

    def create(g, k, K=4, prec=1, io=0, C=1):
        return lib.fc2t2_plan_create(ctypes.byref(g), ctypes.byref(k), K, prec, io, C, None, ctypes.byref(out))

    assert create(_Grid(4, 64, -1, 1), good_k) == 1           # dim
    assert create(_Grid(3, 48, -1, 1), good_k) == 1           # n not a power of two
    assert create(_Grid(3, 2, -1, 1), good_k) == 1            # n < 4
    assert create(_Grid(3, 64, 1, -1), good_k) == 1           # hi <= lo
    assert create(good_g, _Kernel(0, -1.0, 0, None)) == 1     # sigma <= 0
    assert create(good_g, _Kernel(7, 1.0, 0, None)) == 1      # unknown kernel
    assert create(good_g, _Kernel(2, 0.0, 5, None)) == 1      # poly without coefficients
    assert create(good_g, good_k, K=0) == 1
    assert create(good_g, good_k, K=6) == 2                   # unsupported order in 3-D
    assert create(good_g, good_k, C=0) == 1
    assert create(good_g, good_k, prec=9) == 1
    assert create(good_g, good_k, prec=0, io=0) == 2          # FP64 contraction needs FP64 IO
    assert create(good_g, _Kernel(1, 0.02, 0, None), prec=5) == 2   # separable M2L: Gaussian only
    assert create(good_g, good_k, prec=8) == 1
    assert create(good_g, good_k, prec=5 | 0x100) == 2           # the fitted tensor is not separable
    assert out.value is None
    assert lib.fc2t2_plan_create(None, ctypes.byref(good_k), 4, 1, 0, 1, None, ctypes.byref(out)) == 1


def test_null_plan_calls_fail_cleanly(lib):
    assert lib.fc2t2_workspace_size(None, 0, 10) == 0
    assert lib.fc2t2_local_numel(None) == 0
    assert lib.fc2t2_plan_destroy(None) == 1
    assert lib.fc2t2_expand(None, None, None, 0, None, None, 0, None) == 1
    assert lib.fc2t2_eval(None, None, None, 0, None, None, None, None) == 1
    assert lib.fc2t2_stage_timing(None, 1) == 1
    assert lib.fc2t2_stage_time(None, 0, None, None) == 1
    assert lib.fc2t2_out_of_domain(None, None, 0, None) == 1
    assert lib.fc2t2_eval_backward_ex(None, None, None, 0, None, None, None, None, 0, 0, None) == 1
    assert lib.fc2t2_expand_backward_ex(None, None, None, None, 0, None, None, None, 0, 0, None) == 1

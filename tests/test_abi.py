"""The C ABI without a GPU: the library loads, exports every function that
include/fse.h declares, and rejects bad plans and block lists on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from synth import losses, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fse.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fse_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    from paper_2204_14193_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES)


def test_struct_layouts():
    from paper_2204_14193_amd import _lib, fse
    assert C.sizeof(_lib.fse_block_t) == 24 and fse.BLOCK_DTYPE == losses.BLOCK_DTYPE
    assert C.sizeof(_lib.fse_trace_t) == 16
    assert C.sizeof(_lib.fse_plan_desc_t) == 16


@pytest.mark.parametrize("rho,gamma,iters", [(0.0, 0.5, 10), (1.5, 0.5, 10), (0.8, -0.1, 10),
                                             (0.8, 1.5, 10), (0.8, 0.5, -1), (0.8, 0.5, 5000),
                                             (float("nan"), 0.5, 10)])
def test_plan_rejects_bad_parameters(rho, gamma, iters):
    import paper_2204_14193_amd as fse
    with pytest.raises(fse.FseError) as e:
        fse.Plan(rho, gamma, iters)
    assert e.value.code == -1


def test_plan_accepts_edges():
    import paper_2204_14193_amd as fse
    fse.Plan(1.0, 0.0, 0).close()
    fse.Plan(1e-3, 1.0, 4096).close()


def _check(plan, blocks, nf=1, H=256, W=256):
    return plan.validate(losses.blocks_to_array(blocks), nf, H, W)


def test_validation_cases():
    import paper_2204_14193_amd as fse
    plan = fse.Plan(0.8, 0.5, 500)
    B = losses.Block
    good = B(0, 16, 16, 16, 16, 16, 64, 100)
    assert _check(plan, [good]) == (0, -1)
    assert _check(plan, []) == (0, -1)
    cases = {
        -2: [B(0, 16, 16, 16, 16, 16, 48, 10),          # unsupported F
             B(0, 16, 16, 16, 16, 25, 64, 10),          # 66x66 area > 64
             B(0, 16, 16, 40, 8, 16, 64, 10)],          # 72 rows > 64
        -1: [B(0, 16, 16, 16, 16, 16, 64, 501),         # iters > max
             B(0, 16, 16, 16, 16, 16, 64, -1),
             B(1, 16, 16, 16, 16, 16, 64, 10),          # frame out of range
             B(0, 250, 16, 16, 16, 16, 64, 10),         # B leaves the frame
             B(0, -1, 16, 8, 8, 8, 32, 10),
             B(0, 16, 16, 0, 16, 16, 64, 10),           # empty block
             B(0, 16, 16, 16, 16, -1, 64, 10)],
    }
    for code, bad in cases.items():
        for b in bad:
            st, idx = _check(plan, [good, b])
            assert (st, idx) == (code, 1), b
    st, idx = _check(plan, [good, B(0, 31, 31, 4, 4, 8, 32, 10)])
    assert (st, idx) == (-5, 1)
    # areas may overlap (they are independent); only B regions may not
    assert _check(plan, [good, B(0, 33, 16, 8, 8, 16, 64, 10)]) == (0, -1)


def test_validation_of_workloads():
    import paper_2204_14193_amd as fse
    plan = fse.Plan(0.8, 0.5, 500)
    for wl in (workloads.isolated_256(), workloads.random_1080p_8x8()):
        assert plan.validate(wl.blocks, *wl.frames.shape) == (0, -1)

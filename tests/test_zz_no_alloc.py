"""The entry point that allocates nothing: mclbm_create_static builds a context
over the library's static workspace (one array per device in the code object).
Through the C ABI it must give the same results as mclbm_create over a
caller-allocated workspace, bit for bit (the same kernels on the same inputs),
on two contexts in a row, the second smaller than the first (the array keeps the
first context's contents); it refuses a context larger than the array and a
second context while one holds it."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import FIELDS
from paper_2004_11286_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11286_amd import mclbm

    return mclbm


def run(mc, params, fields, precision, steps, static):
    s = mc.Sim(params, precision, static_workspace=static)
    s.init_fields(**fields)
    s.step(steps)
    out = s.read_moments()
    cons = s.conservation()
    buf = bytes(s.save())
    s.close()
    return out, cons, buf


def test_static_context_matches_the_allocating_one_twice(mc):
    cases = [(W.ternary_tube(nx=96, ny=4, nz=4), mc.MCLBM_FP32, 60),
             (W.ternary_tube(nx=40, ny=2, nz=2), mc.MCLBM_FP64, 45)]
    for k, ((params, fields), prec, steps) in enumerate(cases):
        print("case", k, params["nx"], params["ny"], params["nz"], "precision", prec, flush=True)
        got, gc, gbuf = run(mc, params, fields, prec, steps, static=True)
        want, wc, wbuf = run(mc, params, fields, prec, steps, static=False)
        for f in FIELDS:
            np.testing.assert_array_equal(got[f], want[f], err_msg=f"case {k} {f}")
        np.testing.assert_array_equal(gc, wc)
        assert gbuf == wbuf


def test_static_context_limits(mc):
    params, fields = W.ternary_tube(nx=64, ny=4, nz=4)
    s = mc.Sim(params, mc.MCLBM_FP32, static_workspace=True)
    with pytest.raises(mc.MclbmError) as e:                   # the array is held
        mc.Sim(params, mc.MCLBM_FP32, static_workspace=True)
    assert "held" in str(e.value)
    s.close()
    big, _ = W.shear_layer(nx=64, ny=64, nz=64)
    need = mc.mclbm_workspace_bytes(big, mc.MCLBM_FP32)
    assert need > mc.MCLBM_STATIC_WORKSPACE_BYTES
    with pytest.raises(mc.MclbmError) as e:                   # too large for the array
        mc.Sim(big, mc.MCLBM_FP32, static_workspace=True)
    assert str(need) in str(e.value)
    s = mc.Sim(params, mc.MCLBM_FP32, static_workspace=True)  # released by close
    s.init_fields(**fields)
    s.step(3)
    assert s.step_count == 3
    s.close()

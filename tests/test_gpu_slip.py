"""GPU parity of free-slip y walls (wall_y = 1: specular reflection at the y ends,
mirrored stencil ghosts with Phi_y odd) against the oracle, through the C ABI.
The oracle's free-slip walls are pinned on the CPU (tests/test_oracle_slip.py).
Compared here with strong coupling and constant properties, and under weak
coupling and/or temperature-dependent heat capacities and transport.
"""
import numpy as np
import pytest

from gpu_common import FIELDS, OTHER_MODES, decode_checkpoint, field_errors, stored_population_error, with_mode
from paper_2004_11286_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11286_amd import mclbm

    return mclbm


def _case(M, nx, ny, nz, walls, seed):
    if M == 2:
        params, _ = W.binary_interdiffusion(nx=nx, ny=ny, nz=nz)
        X0 = [0.4, 0.6]
    elif M == 3:
        params, _ = W.ternary_tube(nx=nx, ny=ny, nz=nz)
        X0 = [0.3, 0.3, 0.4]
    else:
        params, _ = W.ternary_tube(nx=nx, ny=ny, nz=nz, masses=(2.0, 16.0, 28.0, 40.0),
                                   x_left=(0.2, 0.2, 0.1, 0.5), x_right=(0.1, 0.2, 0.2, 0.5),
                                   Doff={(0, 1): 0.08, (0, 2): 0.07, (0, 3): 0.06, (1, 2): 0.03,
                                         (1, 3): 0.02, (2, 3): 0.04})
        X0 = [0.2, 0.2, 0.15, 0.45]
    params = dict(params, wall_x=int(walls), wall_y=1)
    f = W.random_near_equilibrium(params, nx, ny, nz, seed=seed, X0=X0, p0=params["P0"], T0=0.3,
                                  amp=0.05, uamp=0.03)
    return params, f


@pytest.mark.parametrize("M", [2, 3, 4])
@pytest.mark.parametrize("walls", [0, 1])
def test_slip_ragged_grid_fp64(mc, oracle_mod, M, walls):
    """13 x 7 x 5 nodes, 20 steps in FP64 with free-slip y walls (and x walls or
    periodic x): fields, mass and energy sums and the stored populations against
    the oracle."""
    params, f = _case(M, 13, 7, 5, walls, seed=111 + 2 * M + walls)
    s = mc.Sim(params, mc.MCLBM_FP64)
    s.init_fields(**f)
    s.step(20)
    g, gc = s.read_moments(), s.conservation()
    hdr, vals = decode_checkpoint(s.save())
    s.close()
    o = oracle_mod.OracleSim(params)
    o.init_fields(**f)
    o.step(20)
    om, oc, op = o.read_moments(), o.conservation(), o.populations()
    errs = field_errors(g, om)
    gp = np.stack([hdr["ref"][l][:, None, None, None] + vals[l].astype(np.float64) / hdr["scale"][l]
                   for l in range(M + 1)])
    ref = np.concatenate([op[:M - 1], op[M:M + 2]])
    pop_err = float(np.abs(gp - ref).max() / np.abs(ref).max())
    print("slip fp64", M, walls, errs, "populations", pop_err)
    for k in FIELDS:
        assert errs[k] < 1e-12, (k, errs[k])
    assert pop_err < 1e-12
    np.testing.assert_allclose(gc[:M + 1], oc[:M + 1], rtol=1e-12)
    np.testing.assert_allclose(gc[M + 4], oc[M + 4], rtol=1e-12)


def test_slip_plug_flow_fp64(mc):
    """A plug flow parallel to the free-slip walls stays put."""
    params, _ = W.ternary_tube(nx=8, ny=16, nz=4)
    X, P0, T0, u = [0.3, 0.3, 0.4], params["P0"], 1 / 3, (0.05, 0.0, 0.02)
    params = dict(params, wall_x=0, wall_y=1)
    f = W.uniform_state(params, 8, 16, 4, X=X, p=P0, T=T0, u=u)
    s = mc.Sim(params, mc.MCLBM_FP64)
    s.init_fields(**f)
    s.step(200)
    g = s.read_moments()
    s.close()
    for k in ("X", "p", "T", "u"):
        np.testing.assert_allclose(g[k], f[k], rtol=1e-13, atol=1e-15)


def test_slip_ternary_fp32_1000_steps(mc, oracle_mod):
    """The ternary tube's interface (64 x 16 x 4, walls at the x ends, free-slip y
    walls, a shear flow u_x along y), FP32 storage, FP64 collision, 1000 steps."""
    params, f = W.ternary_tube(nx=64, ny=16, nz=4)
    params = dict(params, wall_y=1)
    f = dict(f, u=f["u"].copy())
    y = np.arange(16, dtype=np.float64) + 0.5
    f["u"][2] += 0.02 * np.cos(np.pi * y / 16)[None, :, None]
    o = oracle_mod.OracleSim(params)
    o.init_fields(**f)
    o.step(1000)
    om = o.read_moments()
    s = mc.Sim(params, mc.MCLBM_FP32)
    s.init_fields(**f)
    s.step(1000)
    g = s.read_moments()
    s.close()
    errs = field_errors(g, om)
    print("slip fp32 1000", errs)
    for k in FIELDS:
        assert errs[k] < 1e-5, (k, errs[k])


def test_slip_checkpoint_resume_and_mismatch(mc):
    """A free-slip checkpoint resumes bit for bit, and a context with periodic y
    refuses it."""
    params, f = _case(3, 16, 8, 4, 1, seed=5)
    s = mc.Sim(params, mc.MCLBM_FP32)
    s.init_fields(**f)
    s.step(7)
    buf = s.save()
    s.step(5)
    a = s.read_moments()
    s.load(buf)
    s.step(5)
    b = s.read_moments()
    s.close()
    for k in FIELDS:
        np.testing.assert_array_equal(a[k], b[k])
    other = mc.Sim(dict(params, wall_y=0), mc.MCLBM_FP32)
    with pytest.raises(mc.MclbmError):
        other.load(buf)
    other.close()


@pytest.mark.parametrize("weak,props", OTHER_MODES)
@pytest.mark.parametrize("M", [2, 3, 4])
@pytest.mark.parametrize("walls", [0, 1])
def test_slip_other_modes_ragged_grid_fp64(mc, oracle_mod, M, walls, weak, props):
    """Weak coupling and/or C_v(T) with T-dependent transport: 13 x 7 x 5 nodes,
    20 steps in FP64, fields, mass and energy sums and every stored population
    against the oracle."""
    params, f = _case(M, 13, 7, 5, walls, seed=151 + 2 * M + walls + 10 * weak + 20 * props)
    params = with_mode(params, weak, props)
    s = mc.Sim(params, mc.MCLBM_FP64)
    s.init_fields(**f)
    s.step(20)
    g, gc = s.read_moments(), s.conservation()
    hdr, vals = decode_checkpoint(s.save())
    s.close()
    o = oracle_mod.OracleSim(params)
    o.init_fields(**f)
    o.step(20)
    om, oc, op = o.read_moments(), o.conservation(), o.populations()
    errs = field_errors(g, om)
    pop_err = stored_population_error(hdr, vals, op, M, weak)
    print("slip modes fp64", M, walls, weak, props, errs, "populations", pop_err)
    for k in FIELDS:
        assert errs[k] < 1e-12, (k, errs[k])
    assert pop_err < 1e-12
    np.testing.assert_allclose(gc[:M + 1], oc[:M + 1], rtol=1e-12)
    np.testing.assert_allclose(gc[M + 4], oc[M + 4], rtol=1e-12)


def test_slip_weak_cv_of_T_fp32_1000_steps(mc, oracle_mod):
    """The 64 x 16 x 4 walled interface with free-slip y walls and a shear flow,
    weak coupling with C_v(T) and T-dependent transport, FP32 storage, 1000 steps."""
    params, f = W.ternary_tube(nx=64, ny=16, nz=4)
    params = with_mode(dict(params, wall_y=1), 1, True, T=1 / 3)
    f = dict(f, u=f["u"].copy())
    y = np.arange(16, dtype=np.float64) + 0.5
    f["u"][2] += 0.02 * np.cos(np.pi * y / 16)[None, :, None]
    o = oracle_mod.OracleSim(params)
    o.init_fields(**f)
    o.step(1000)
    om = o.read_moments()
    s = mc.Sim(params, mc.MCLBM_FP32)
    s.init_fields(**f)
    s.step(1000)
    g = s.read_moments()
    s.close()
    errs = field_errors(g, om)
    print("slip weak cvt fp32 1000", errs)
    for k in FIELDS:
        assert errs[k] < 1e-5, (k, errs[k])

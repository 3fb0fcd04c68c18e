"""GPU parity of open x ends (wall_x = 2: equilibrium inlet at x = 0, zero-gradient
outlet at x = nx - 1) against the oracle, through the C ABI. The oracle's open
ends are pinned on the CPU (tests/test_oracle_open.py). Compared here: fields
and stored populations on ragged grids with an inlet state different from the
interior (FP64), the uniform through-flow fixed point, the inflow front of the
advection-diffusion pin (FP64 and FP32), and a walled-tube-sized ternary
through-flow over 1000 steps (FP32); the same ragged grids under weak coupling
and with temperature-dependent heat capacities and transport, and the
through-flow with both (FP32).
"""
import numpy as np
import pytest

from gpu_common import FIELDS, OTHER_MODES, decode_checkpoint, field_errors, stored_population_error, with_mode
import physics_cases as pc
from paper_2004_11286_amd import workloads as W

pytestmark = pytest.mark.gpu
T0 = 1.0 / 3.0


@pytest.fixture(scope="module")
def mc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11286_amd import mclbm

    return mclbm


def _case(M, nx, ny, nz, seed):
    if M == 2:
        params, _ = W.binary_interdiffusion(nx=nx, ny=ny, nz=nz)
        X0, Xin = [0.4, 0.6], [0.7, 0.3]
    elif M == 3:
        params, _ = W.ternary_tube(nx=nx, ny=ny, nz=nz)
        X0, Xin = [0.3, 0.3, 0.4], [0.1, 0.4, 0.5]
    else:
        params, _ = W.ternary_tube(nx=nx, ny=ny, nz=nz, masses=(2.0, 16.0, 28.0, 40.0),
                                   x_left=(0.2, 0.2, 0.1, 0.5), x_right=(0.1, 0.2, 0.2, 0.5),
                                   Doff={(0, 1): 0.08, (0, 2): 0.07, (0, 3): 0.06, (1, 2): 0.03,
                                         (1, 3): 0.02, (2, 3): 0.04})
        X0, Xin = [0.2, 0.2, 0.15, 0.45], [0.1, 0.3, 0.1, 0.5]
    inlet = np.array(Xin + [1.02 * params["P0"], 0.31, 0.04, 0.01, -0.02])
    params = dict(params, wall_x=2, inlet=inlet)
    f = W.random_near_equilibrium(params, nx, ny, nz, seed=seed, X0=X0, p0=params["P0"], T0=0.3,
                                  amp=0.05, uamp=0.03)
    f["u"][0] += 0.03                                   # a mean flow from inlet to outlet
    return params, f


@pytest.mark.parametrize("M", [2, 3, 4])
def test_open_ragged_grid_fp64(mc, oracle_mod, M):
    """13 x 7 x 5 nodes, 20 steps in FP64 with an inlet state unlike the interior:
    fields, the mass and energy sums and every stored population against the
    oracle (the inflow crosses several nodes in that time)."""
    params, f = _case(M, 13, 7, 5, seed=71 + M)
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
    print("open fp64", M, errs, "populations", pop_err)
    for k in FIELDS:
        assert errs[k] < 1e-12, (k, errs[k])
    assert pop_err < 1e-12
    np.testing.assert_allclose(gc[:M + 1], oc[:M + 1], rtol=1e-12)
    np.testing.assert_allclose(gc[M + 4], oc[M + 4], rtol=1e-12)


def test_open_uniform_through_flow_fp64(mc):
    """A uniform equilibrium flowing through the domain, fed with itself, stays put."""
    params, _ = W.ternary_tube(nx=24, ny=4, nz=4)
    X, P0, u = [0.3, 0.3, 0.4], params["P0"], (0.05, 0.01, -0.02)
    params = dict(params, wall_x=2, inlet=np.array(X + [P0, T0] + list(u)))
    f = W.uniform_state(params, 24, 4, 4, X=X, p=P0, T=T0, u=u)
    s = mc.Sim(params, mc.MCLBM_FP64)
    s.init_fields(**f)
    s.step(200)
    g = s.read_moments()
    s.close()
    for k in FIELDS:
        np.testing.assert_allclose(g[k], f[k] if k != "rho" else g[k], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_open_inflow_front(mc, oracle_mod, prec, tol):
    """The advection-diffusion inflow front of the oracle pin (equal molar masses,
    nx = 256, 1600 steps) on the GPU against the oracle."""
    nx, t, u, D = 256, 1600, 0.025, 0.05
    P = T0 / 20.0
    params = {"nx": nx, "ny": 1, "nz": 1, "wall_x": 2,
              **pc.species_block([20.0, 20.0], [1.5, 1.5], [0.5, 0.5], P, D),
              "inlet": np.array([0.8, 0.2, P, T0, u, 0.0, 0.0])}
    f = pc.line_fields(2, nx, [0.2, 0.8], P, T0, (u, 0, 0))
    s = mc.Sim(params, mc.PRECISIONS[prec])
    s.init_fields(**f)
    s.step(t)
    g = s.read_moments()
    s.close()
    o = oracle_mod.OracleSim(params)
    o.init_fields(**f)
    o.step(t)
    errs = field_errors(g, o.read_moments())
    print("open front", prec, errs)
    for k in FIELDS:
        assert errs[k] < tol, (k, errs[k])


def test_open_ternary_through_flow_fp32_1000_steps(mc, oracle_mod):
    """The ternary tube's sharp interface (256 x 4 x 4) carried by a mean flow of
    0.02 through open ends, the inlet at the left half's state, FP32 storage,
    1000 steps."""
    params, f = W.ternary_tube()
    Xl = [float(v) for v in f["X"][:, 0, 0, 0]]
    params = dict(params, wall_x=2, inlet=np.array(Xl + [params["P0"], T0, 0.02, 0.0, 0.0]))
    f = dict(f, u=f["u"].copy())
    f["u"][0] += 0.02
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
    print("open C2 fp32 1000", errs)
    for k in FIELDS:
        assert errs[k] < 1e-5, (k, errs[k])


@pytest.mark.parametrize("weak,props", OTHER_MODES)
@pytest.mark.parametrize("M", [2, 3, 4])
def test_open_other_modes_ragged_grid_fp64(mc, oracle_mod, M, weak, props):
    """Weak coupling and/or C_v(T) with T-dependent transport: 13 x 7 x 5 nodes,
    20 steps in FP64, fields, mass and energy sums and every stored population
    against the oracle."""
    params, f = _case(M, 13, 7, 5, seed=131 + M + 5 * weak + 10 * props)
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
    print("open modes fp64", M, weak, props, errs, "populations", pop_err)
    for k in FIELDS:
        assert errs[k] < 1e-12, (k, errs[k])
    assert pop_err < 1e-12
    np.testing.assert_allclose(gc[:M + 1], oc[:M + 1], rtol=1e-12)
    np.testing.assert_allclose(gc[M + 4], oc[M + 4], rtol=1e-12)


def test_open_weak_cv_of_T_through_flow_fp32_1000_steps(mc, oracle_mod):
    """The ternary tube's interface carried through open ends by a mean flow of
    0.02, weak coupling with C_v(T) and T-dependent transport, FP32 storage,
    1000 steps."""
    params, f = W.ternary_tube()
    Xl = [float(v) for v in f["X"][:, 0, 0, 0]]
    params = with_mode(dict(params, wall_x=2, inlet=np.array(Xl + [params["P0"], T0, 0.02, 0.0, 0.0])), 1, True,
                       T=T0)
    f = dict(f, u=f["u"].copy())
    f["u"][0] += 0.02
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
    print("open weak cvt fp32 1000", errs)
    for k in FIELDS:
        assert errs[k] < 1e-5, (k, errs[k])


def test_open_weak_cv_of_T_checkpoint_resume_and_mismatch(mc):
    """A weakly coupled context with C_v(T) and open x ends resumes bit for bit
    from its checkpoint (all M + 2 lattices); contexts that differ in coupling or
    in the kind of heat capacities refuse it."""
    params, f = _case(3, 16, 6, 4, seed=9)
    params = with_mode(params, 1, True)
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
    for other_params in (dict(params, weak=0), {k: v for k, v in params.items() if k not in ("cv_coef", "transport_exp")}):
        other = mc.Sim(other_params, mc.MCLBM_FP32)
        with pytest.raises(mc.MclbmError):
            other.load(buf)
        other.close()

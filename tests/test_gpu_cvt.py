"""GPU parity of temperature-dependent specific heats (Sec. 3.1) against the
oracle, through the C ABI.

C_{a,v}(T) = sum_k c_ak T^k; the temperature is the root of eq temperature
(Newton's method in the moments and read-back kernels), H_a(T) enters the
energy collision, and the correction flux takes the gradients of the mass
fractions. The oracle's polynomial mode is pinned on the CPU
(tests/test_oracle_cvt.py). Compared here: fields and the stored populations on
ragged grids (FP64), a walled ternary tube in FP32 over 1000 steps, windows of
the full-size shear layer, and the temperature read back after initialisation.
"""
import numpy as np
import pytest

from gpu_common import FIELDS, decode_checkpoint, field_errors, oracle_window
from paper_2004_11286_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11286_amd import mclbm

    return mclbm


def with_cv_of_T(params, T0):
    """Heat capacities rising with T, differently per species (linear, quadratic
    and cubic parts; C_v about doubles at T0 for the first species)."""
    cv = np.asarray(params["cv"], dtype=np.float64)
    shapes = [[1.0, 0.6 / T0, 0.1 / T0 ** 2, 0.3 / T0 ** 3], [1.0, 0.0, 0.4 / T0 ** 2, 0.0],
              [1.0, 0.2 / T0, 0.0, 0.1 / T0 ** 3], [1.0, 0.3 / T0, 0.3 / T0 ** 2, 0.0]]
    return dict(params, cv_coef=np.stack([cv[a] * np.asarray(shapes[a]) for a in range(len(cv))]))


def _case(M, nx, ny, nz, walls, seed):
    T0 = 0.3
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
    params = with_cv_of_T(dict(params, wall_x=int(walls)), T0)
    f = W.random_near_equilibrium(params, nx, ny, nz, seed=seed, X0=X0, p0=params["P0"], T0=T0,
                                  amp=0.05, uamp=0.03)
    return params, f


@pytest.mark.parametrize("M", [2, 3, 4])
@pytest.mark.parametrize("walls", [0, 1])
def test_cvt_ragged_grid_fp64(mc, oracle_mod, M, walls):
    """13 x 7 x 5 nodes, 20 steps in FP64: fields, conservation sums and the stored
    populations against the oracle; the result differs from constant heat
    capacities."""
    params, f = _case(M, 13, 7, 5, walls, seed=51 + 2 * M + walls)
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
    # stored lattices: species 1..M-1, f, g (the slaved species is not stored)
    gp = np.stack([hdr["ref"][l][:, None, None, None] + vals[l].astype(np.float64) / hdr["scale"][l]
                   for l in range(M + 1)])
    ref = np.concatenate([op[:M - 1], op[M:M + 2]])
    pop_err = float(np.abs(gp - ref).max() / np.abs(ref).max())
    print("cvt fp64", M, walls, errs, "populations", pop_err)
    for k in FIELDS:
        assert errs[k] < 1e-12, (k, errs[k])
    assert pop_err < 1e-12
    np.testing.assert_allclose(gc[:M + 1], oc[:M + 1], rtol=1e-12)
    np.testing.assert_allclose(gc[M + 4], oc[M + 4], rtol=1e-12)
    const = mc.Sim({k: v for k, v in params.items() if k != "cv_coef"}, mc.MCLBM_FP64)
    const.init_fields(**f)
    const.step(20)
    gk = const.read_moments()
    const.close()
    assert np.abs(gk["T"] - g["T"]).max() > 1e-6 * np.abs(g["T"]).max()


def test_cvt_temperature_read_back(mc):
    """Initialised at (X, p, T, u), the state reads back T and p: the energy held
    by the energy lattice is rho (U(T) + u^2/2) and Newton's method inverts it."""
    params, f = _case(3, 16, 8, 4, 0, seed=2)
    f["T"] = f["T"] * (1.0 + 0.3 * np.random.default_rng(0).uniform(-1, 1, f["T"].shape))
    s = mc.Sim(params, mc.MCLBM_FP64)
    s.init_fields(**f)
    g = s.read_moments()
    s.close()
    np.testing.assert_allclose(g["T"], f["T"], rtol=1e-13)
    np.testing.assert_allclose(g["p"], f["p"], rtol=1e-13)


def test_cvt_ternary_tube_fp32_1000_steps(mc, oracle_mod):
    """256 x 4 x 4 tube with walls, FP32 storage, FP64 collision, 1000 steps."""
    params, f = W.ternary_tube()
    params = with_cv_of_T(params, 1 / 3)
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
    print("cvt C2 fp32 1000", errs)
    for k in FIELDS:
        assert errs[k] < 1e-5, (k, errs[k])


def test_cvt_full_size_shear_layer_windows(mc, oracle_mod):
    """The 256^3 shear layer with polynomial heat capacities, FP32 storage: the
    GPU state after 20 steps, cut into 9^3 periodic windows, advanced one step
    by the oracle, matches the GPU's step 21 at the window centres."""
    params, f = W.shear_layer()
    params = with_cv_of_T(params, 1.0)
    s = mc.Sim(params, mc.MCLBM_FP32)
    s.init_fields(**f)
    c0 = s.conservation()
    s.step(20)
    hdr, vals = decode_checkpoint(s.save())
    s.step(1)
    g = s.read_moments()
    c1 = s.conservation()
    s.close()
    M = params["M"]
    np.testing.assert_allclose(c1[:M + 1], c0[:M + 1], rtol=1e-6)
    np.testing.assert_allclose(c1[M + 4], c0[M + 4], rtol=1e-6)
    worst = {k: 0.0 for k in FIELDS}
    rng = np.random.default_rng(11)
    centers = [(0, 0, 0), (255, 64, 128), (17, 63, 200)]
    centers += [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(4)]
    r = 4
    for (x, y, z) in centers:
        win = oracle_window(hdr, vals, (x, y, z), r)
        wp = dict(params, nx=2 * r + 1, ny=2 * r + 1, nz=2 * r + 1, wall_x=0)
        o = oracle_mod.OracleSim(wp)
        o.set_populations(win)
        o.step(1)
        om = o.read_moments()
        for k in FIELDS:
            ov = om[k][..., r, r, r]
            gv = g[k][..., z, y, x]
            scale = max(np.abs(f[k]).max(), 1e-3) if k == "u" else np.abs(ov).max()
            worst[k] = max(worst[k], float(np.abs(gv - ov).max() / scale))
            assert np.abs(gv - ov).max() <= 1e-6 * scale, (k, (x, y, z), gv, ov)
    print("cvt fp32 worst window error", worst)


def with_transport(params, T_ref):
    """Transport coefficients as powers of T / T_ref (viscosity 0.7, 0.8, ...;
    conductivity 0.75, 0.85, ...; diffusivity 1.75)."""
    M = params["M"]
    tex = np.concatenate([0.7 + 0.1 * np.arange(M), 0.75 + 0.1 * np.arange(M), [1.75, T_ref]])
    return dict(params, transport_exp=tex)


@pytest.mark.parametrize("M,walls,cvt", [(2, 0, False), (3, 1, False), (3, 1, True), (4, 0, True)])
def test_transport_of_T_ragged_grid_fp64(mc, oracle_mod, M, walls, cvt):
    """Temperature-dependent transport (T about 1.4 T_ref), alone and with C_v(T):
    13 x 7 x 5 nodes, 20 steps in FP64, fields against the oracle; the result
    differs from constant transport."""
    params, f = _case(M, 13, 7, 5, walls, seed=91 + M)
    if not cvt:
        params = {k: v for k, v in params.items() if k != "cv_coef"}
    params = with_transport(params, 0.3 / 1.4)
    s = mc.Sim(params, mc.MCLBM_FP64)
    s.init_fields(**f)
    s.step(20)
    g, gc = s.read_moments(), s.conservation()
    s.close()
    o = oracle_mod.OracleSim(params)
    o.init_fields(**f)
    o.step(20)
    om, oc = o.read_moments(), o.conservation()
    errs = field_errors(g, om)
    print("transport fp64", M, walls, cvt, errs)
    for k in FIELDS:
        assert errs[k] < 1e-12, (k, errs[k])
    np.testing.assert_allclose(gc[:M + 1], oc[:M + 1], rtol=1e-12)
    const = mc.Sim({k: v for k, v in params.items() if k != "transport_exp"}, mc.MCLBM_FP64)
    const.init_fields(**f)
    const.step(20)
    gk = const.read_moments()
    const.close()
    assert np.abs(gk["X"] - g["X"]).max() > 1e-9


def test_transport_of_T_ternary_tube_fp32_1000_steps(mc, oracle_mod):
    """256 x 4 x 4 walled tube with C_v(T) and temperature-dependent transport,
    FP32 storage, FP64 collision, 1000 steps."""
    params, f = W.ternary_tube()
    params = with_transport(with_cv_of_T(params, 1 / 3), 0.25)
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
    print("transport C2 fp32 1000", errs)
    for k in FIELDS:
        assert errs[k] < 1e-5, (k, errs[k])

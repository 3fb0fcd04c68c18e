"""Batched engine: many independent tubes of uneven length in one context.

Parity: every tube of a batch against the FP64 oracle run on that tube alone;
bit-for-bit equality of a batch with single-tube contexts; bit-for-bit equality
of every launch choice within a step path (occupancy variant, XCD order, tube
order, sequential per-tube launches, replayed HIP graphs), agreement of the
two-read and three-pass paths to rounding; the autotuner; the FP32 trajectory
read-back; per-tube conservation; the full 512-tube ensemble (18.9 M nodes)
sampled through whole tubes advanced by the oracle.
"""
import numpy as np
import pytest

from gpu_common import FIELDS, field_errors
from paper_2004_11286_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11286_amd import mclbm

    return mclbm


def small_ensemble(n=6, seed=5):
    return W.tube_ensemble(ntubes=n, ny=4, nz=4, lmin=8, lmax=40, seed=seed)


def run_batch(mc, tubes, precision, steps, **launch):
    b = mc.Batch([p for p, _ in tubes], precision)
    if launch:
        b.set_launch(**launch)
    b.init_fields([f for _, f in tubes])
    b.step(steps)
    out = b.read_moments()
    buf = bytes(b.save())
    b.close()
    return out, buf


def test_batch_matches_oracle_fp64(mc, oracle_mod):
    """Six ragged tubes (8..40 x 4 x 4, walls), 40 steps in FP64: each tube
    against the oracle run on that tube alone."""
    tubes = small_ensemble()
    g, _ = run_batch(mc, tubes, mc.MCLBM_FP64, 40)
    for t, (params, f) in enumerate(tubes):
        o = oracle_mod.OracleSim(params)
        o.init_fields(**f)
        o.step(40)
        errs = field_errors(g[t], o.read_moments())
        print("batch fp64 tube", t, params["nx"], errs)
        for k in FIELDS:
            assert errs[k] < 1e-12, (t, k, errs[k])


@pytest.mark.parametrize("prec", ["fp32", "fp16", "i16"])
def test_batch_is_bitwise_single_contexts(mc, prec):
    tubes = small_ensemble(seed=6)
    g, _ = run_batch(mc, tubes, mc.PRECISIONS[prec], 30)
    for t, (params, f) in enumerate(tubes):
        s = mc.Sim(params, mc.PRECISIONS[prec])
        s.init_fields(**f)
        s.step(30)
        r = s.read_moments()
        s.close()
        for k in FIELDS:
            np.testing.assert_array_equal(g[t][k], r[k], err_msg=f"tube {t} {k}")


LAUNCHES = [dict(variant=1), dict(swizzle=1), dict(order=1), dict(sequential=1), dict(graph_steps=4),
            dict(graph_steps=2, swizzle=1, order=1, variant=1),
            # block shapes (tiles of 64x4, 32x8, 16x16, 64x2x2, 32x4x2 nodes), alone and with
            # the other choices: the ragged tubes leave idle threads in edge tiles
            dict(shape=1), dict(shape=2, sequential=1), dict(shape=3, swizzle=1), dict(shape=4, order=1),
            dict(shape=5, graph_steps=2, swizzle=1, variant=1)]


@pytest.mark.parametrize("three_pass", [0, 1])
@pytest.mark.parametrize("prec", ["fp32", "fp16", "i16"])
def test_launch_choices_are_bitwise_equal(mc, prec, three_pass):
    """Within each step path (two-read, three-pass) every launch choice computes
    the same step bit for bit. The graph runs start from an odd step (one eager
    step first) and are interleaved with reads, so several replays follow eager
    work; 16-bit storage checks the replayed step counter of the stochastic
    rounding."""
    tubes = small_ensemble(n=9, seed=7)
    P = mc.PRECISIONS[prec]

    def run(**launch):
        b = mc.Batch([p for p, _ in tubes], P)
        b.set_launch(**launch)
        b.init_fields([f for _, f in tubes])
        outs = []
        for n in (1, 9, 8, 3):
            b.step(n)
            outs.append(bytes(b.save()))
        assert b.step_count == 21
        b.close()
        return outs

    ref = run(three_pass=three_pass)
    for launch in LAUNCHES:
        got = run(three_pass=three_pass, **launch)
        for k, (a, r) in enumerate(zip(got, ref)):
            assert a == r, (launch, k)


@pytest.mark.parametrize("prec,rtol", [("fp32", 1e-5), ("fp16", 2e-3), ("i16", 2e-3)])
def test_step_paths_agree_to_rounding(mc, prec, rtol):
    """The two-read step, the three-pass step and its split collision (species
    lattices, then momentum and energy lattices, in two launches) compute the
    same step. The three-pass step carries the node state through the record in
    the record precision, and the split kernels are compiled separately and may
    fuse a multiply-add differently, so the fields agree to rounding (16-bit
    storage: to the stochastic rounding that a last-bit difference can flip)."""
    tubes = small_ensemble(n=9, seed=7)
    P = mc.PRECISIONS[prec]
    out = []
    for launch in (dict(), dict(three_pass=1), dict(three_pass=1, split=1),
                   dict(three_pass=1, split=1, graph_steps=2, swizzle=1, sequential=1)):
        b = mc.Batch([p for p, _ in tubes], P)
        b.set_launch(**launch)
        b.init_fields([f for _, f in tubes])
        b.step(21)
        out.append(b.read_moments())
        b.close()
    for j, got in enumerate(out[1:]):
        worst = 0.0
        for t in range(len(tubes)):
            for k in FIELDS:
                scale = max(np.abs(out[0][t][k]).max(), 1e-3 if k == "u" else 0.0)
                err = np.abs(got[t][k] - out[0][t][k]).max() / scale
                worst = max(worst, err)
                assert err <= rtol, (j, t, k, err)
        print(prec, "launch", j + 1, "largest relative difference from the two-read step", worst)


def test_autotune_picks_a_choice_and_keeps_the_trajectory(mc):
    tubes = small_ensemble(n=8, seed=8)
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP32)
    b.init_fields([f for _, f in tubes])
    rep = b.autotune(4)
    print(rep)
    lines = rep.strip().splitlines()
    assert lines[-1].startswith("chosen")
    # header, 6 paths x 2 x 2 x 2 candidates in the linear numbering, the fastest with 5 tiled shapes, choice
    assert len(lines) == 1 + 48 + 5 + 1
    assert sorted(int(r.split()[6]) for r in lines[49:54]) == [1, 2, 3, 4, 5]
    chosen = [int(v) for v in lines[-1].split()[1:8]]
    lc = b.launch()
    assert [lc["three_pass"], lc["variant"], lc["split"], lc["swizzle"], lc["order"], lc["graph_steps"],
            lc["shape"]] == chosen
    n = b.step_count
    b.step(5)
    got = b.read_moments()
    b.close()
    ref, _ = run_batch(mc, tubes, mc.MCLBM_FP32, n + 5)
    for t in range(len(tubes)):
        for k in FIELDS:
            # bitwise within a step path; across paths and with the split collision, to rounding
            scale = max(np.abs(ref[t][k]).max(), 1e-3 if k == "u" else 0.0)
            assert np.abs(got[t][k] - ref[t][k]).max() <= 1e-5 * scale, (t, k)


def test_trajectory_fields_f32(mc):
    tubes = small_ensemble(n=4, seed=9)
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP32)
    b.init_fields([f for _, f in tubes])
    b.step(12)
    flat = b.read_fields_f32().cpu().numpy()
    mom = b.read_moments()
    M = b.M
    parts = b.split(flat, M + 5)
    b.close()
    for t in range(len(tubes)):
        want = np.concatenate([mom[t]["X"], mom[t]["T"][None], mom[t]["u"], mom[t]["p"][None]]).astype(np.float32)
        np.testing.assert_array_equal(parts[t], want)


def test_conservation_per_tube(mc):
    tubes = small_ensemble(n=5, seed=10)
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP32)
    b.init_fields([f for _, f in tubes])
    c0 = b.conservation()
    b.step(200)
    c1 = b.conservation()
    b.close()
    M = b.M
    assert c0.shape == (5, M + 5)
    # walls: species masses, total mass and energy are conserved per tube
    for t in range(5):
        np.testing.assert_allclose(c1[t, :M + 1], c0[t, :M + 1], rtol=1e-6)
        np.testing.assert_allclose(c1[t, M + 4], c0[t, M + 4], rtol=1e-6)
    # different mixtures: the tubes really hold different states
    assert np.unique(np.round(c0[:, 0], 6)).size == 5


def test_full_size_ensemble_sampled_tubes(mc, oracle_mod):
    """The 512-tube ensemble (L ~ U{32..256} x 16 x 16, 18.9 M nodes, FP32) in one
    context, 20 steps; the shortest, the longest and two random tubes are run
    whole by the oracle and compared field by field. The velocity in a tube is
    driven by diffusion alone and can be tiny, so its error is taken relative to
    max(max |u|, 1e-3) and bounded by the FP32 target 1e-5 (FP32 storage resolves
    the momentum populations to about 1e-8 absolute); the other fields to 1e-6."""
    tubes = W.tube_ensemble()
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP32)
    assert b.n == sum(p["nx"] for p, _ in tubes) * 256
    b.init_fields([f for _, f in tubes])
    b.step(20)
    g = b.read_moments()
    b.close()
    lens = np.array([p["nx"] for p, _ in tubes])
    rng = np.random.default_rng(3)
    picks = sorted({int(lens.argmin()), int(lens.argmax()), *[int(v) for v in rng.integers(0, 512, 2)]})
    for t in picks:
        params, f = tubes[t]
        o = oracle_mod.OracleSim(params)
        o.init_fields(**f)
        o.step(20)
        om = o.read_moments()
        errs = field_errors(g[t], om)
        errs["u"] = float(np.abs(g[t]["u"] - om["u"]).max() / max(np.abs(om["u"]).max(), 1e-3))
        print("ensemble tube", t, params["nx"], errs)
        for k in FIELDS:
            assert errs[k] < (1e-5 if k == "u" else 1e-6), (t, k, errs[k])


def test_batch_checkpoint_resume_is_bitwise(mc):
    tubes = small_ensemble(n=5, seed=12)
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP16)
    b.init_fields([f for _, f in tubes])
    b.step(7)
    buf = b.save()
    b.step(6)
    a = b.read_moments()
    b.load(buf)
    assert b.step_count == 7
    b.step(6)
    c = b.read_moments()
    b.close()
    for t in range(len(tubes)):
        for k in FIELDS:
            np.testing.assert_array_equal(a[t][k], c[t][k])
    # a checkpoint does not load into a batch of other tubes
    other = mc.Batch([p for p, _ in small_ensemble(n=5, seed=13)], mc.MCLBM_FP16)
    with pytest.raises(mc.MclbmError):
        other.load(buf)
    other.close()


def test_launch_arguments_are_checked(mc):
    tubes = small_ensemble(n=2, seed=14)
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP32)
    for bad in (dict(variant=2), dict(graph_steps=3), dict(swizzle=2), dict(split=2), dict(order=2)):
        with pytest.raises(mc.MclbmError):
            b.set_launch(**bad)
    b.set_launch(variant=1, split=1)
    b.set_launch(variant=0, split=0)
    b.close()


@pytest.mark.gpu
def test_stream_copy_is_exact(mc):
    import torch

    for n in (4, 1000, (1 << 20) + 12):               # float counts: multiples of 4 (16 bytes)
        a = torch.randn(n, device="cuda")
        b = torch.full_like(a, float("nan"))
        mc.stream_copy(b, a)
        torch.cuda.synchronize()
        assert torch.equal(a, b), n


@pytest.mark.parametrize("model", ["weak", "cv_of_T", "weak_cv_of_T_open", "weak_cv_of_T_slip"])
def test_batch_models_match_oracle_and_single_contexts(mc, oracle_mod, model):
    """Weak coupling and temperature-dependent heat capacities, apart and together
    (between open x ends, each tube fed at its own left-end state, or between
    free-slip y walls), in a batch of ragged tubes (each with its own species
    data): every tube bit for bit equal to its own single-tube context, and
    within 1e-12 of the oracle (FP64, 30 steps)."""
    tubes = []
    for p, f in small_ensemble(n=4, seed=21):
        if model.startswith("weak"):
            p = dict(p, weak=1)
        if "cv_of_T" in model:
            cv = np.asarray(p["cv"], dtype=np.float64)
            p = dict(p, cv_coef=np.stack([cv[a] * np.array([1.0, 0.5 * 3, 0.0, 0.2 * 27]) for a in range(p["M"])]))
        if model.endswith("open"):
            Xl = [float(v) for v in f["X"][:, 0, 0, 0]]
            p = dict(p, wall_x=2, inlet=np.array(Xl + [float(f["p"][0, 0, 0]), float(f["T"][0, 0, 0]), 0.02, 0.0, 0.0]))
            f = dict(f, u=f["u"] + np.array([0.02, 0.0, 0.0])[:, None, None, None])
        if model.endswith("slip"):
            p = dict(p, wall_y=1)
        tubes.append((p, f))
    g, _ = run_batch(mc, tubes, mc.MCLBM_FP64, 30)
    for t, (params, f) in enumerate(tubes):
        s = mc.Sim(params, mc.MCLBM_FP64)
        s.init_fields(**f)
        s.step(30)
        r = s.read_moments()
        s.close()
        o = oracle_mod.OracleSim(params)
        o.init_fields(**f)
        o.step(30)
        om = o.read_moments()
        for k in FIELDS:
            np.testing.assert_array_equal(g[t][k], r[k], err_msg=f"{model} tube {t} {k}")
            scale = max(np.abs(om[k]).max(), 1e-3 if k == "u" else 0.0)
            assert np.abs(g[t][k] - om[k]).max() <= 1e-12 * scale, (model, t, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_block_shapes_are_bitwise_equal_single_contexts(mc, prec):
    """Every block shape gives the same step bit for bit on single contexts with
    ragged grids: a walled ternary tube with free-slip y walls and the opposed
    jets (their edge tiles leave threads idle in x, y and z)."""
    cases = []
    params, f = W.ternary_tube(nx=13, ny=7, nz=5)
    cases.append((dict(params, wall_y=1), f))
    P0 = params["P0"]
    jets = dict(params, nx=13, ny=11, nz=3, wall_x=3, wall_y=2, nozzle=(2, 9),
                inlet=np.array([0.1, 0.4, 0.5, P0, 1.0 / 3.0, 0.04, 0.0, 0.0]),
                inlet_right=np.array([0.3, 0.2, 0.5, P0, 1.0 / 3.0, -0.04, 0.0, 0.0]))
    cases.append((jets, W.random_near_equilibrium(jets, 13, 11, 3, seed=5, X0=[0.2, 0.3, 0.5], p0=P0, T0=1.0 / 3.0)))
    for params, f in cases:
        outs = []
        for shape in range(6):
            s = mc.Sim(params, mc.PRECISIONS[prec])
            s.set_launch(shape=shape)
            s.init_fields(**f)
            s.step(7)
            outs.append(bytes(s.save()))
            s.close()
        for shape in range(1, 6):
            assert outs[shape] == outs[0], (params["wall_x"], shape)

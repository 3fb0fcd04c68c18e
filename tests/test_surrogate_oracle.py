"""Pins of the surrogate's FP64 reference against what the definitions fix:
brute-force index loops, the adjoint identity of the convolution, central
finite differences of the loss, the closed-form first Adam step, and
equivariance under periodic shifts in y and z."""
import numpy as np
import pytest

from oracle import surrogate_oracle as S


def brute_conv(x, W, b):
    Cin, nz, ny, nx = x.shape
    Cout = W.shape[1]
    y = np.zeros((Cout, nz, ny, nx))
    for o in range(Cout):
        for z in range(nz):
            for yy in range(ny):
                for xx in range(nx):
                    s = b[o]
                    for tap in range(27):
                        dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
                        xi = min(max(xx + dx, 0), nx - 1)   # replicate padding at the walls
                        zi, yi = (z + dz) % nz, (yy + dy) % ny
                        for i in range(Cin):
                            s += W[tap, o, i] * x[i, zi, yi, xi]
                    y[o, z, yy, xx] = s
    return y


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 3, 4, 5))
    W = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=2)
    np.testing.assert_allclose(S.conv(x, W, b), brute_conv(x, W, b), rtol=1e-12, atol=1e-12)


def test_conv_single_tap_is_a_shift():
    """One unit weight on tap (dz, dy, dx) = (0, 0, +1): y(x) = in(x + 1), the wall
    value itself at the last x."""
    x = np.arange(2 * 2 * 3 * 4, dtype=float).reshape(2, 2, 3, 4)
    W = np.zeros((27, 2, 2))
    W[9 * 1 + 3 * 1 + 2, 0, 0] = 1.0            # tap (0, 0, +1)
    assert S.tap_offset(14) == (0, 0, 1)
    y = S.conv(x, W, None)
    np.testing.assert_array_equal(y[0, :, :, :-1], x[0, :, :, 1:])
    np.testing.assert_array_equal(y[0, :, :, -1], x[0, :, :, -1])
    np.testing.assert_array_equal(y[1], 0.0)


def test_conv_sees_no_wall_in_an_x_uniform_field():
    """Replicate padding: a field constant along x gives wall outputs equal to the
    interior ones (zero padding would not)."""
    rng = np.random.default_rng(7)
    x = np.repeat(rng.normal(size=(3, 2, 3, 1)), 6, axis=3)
    W = rng.normal(size=(27, 2, 3))
    y = S.conv(x, W, rng.normal(size=2))
    np.testing.assert_allclose(y, np.repeat(y[..., 2:3], 6, axis=3), rtol=1e-12, atol=1e-12)


def test_conv_with_mirror_symmetric_weights_is_the_method_of_images():
    """With weights symmetric under dx -> -dx, the convolution of a tube equals the
    circular convolution of its mirror image doubled domain (x, then x reversed)
    restricted to the tube: the half-way wall as a mirror."""
    rng = np.random.default_rng(8)
    x = rng.normal(size=(2, 3, 4, 5))
    W = rng.normal(size=(27, 3, 2))
    for tap in range(27):
        dz, dy, dx = S.tap_offset(tap)
        if dx == 1:
            W[tap] = W[tap - 2]                      # tap (dz, dy, -1)
    b = rng.normal(size=3)
    ext = np.concatenate([x, x[..., ::-1]], axis=3)
    circ = np.zeros((3,) + ext.shape[1:])
    for tap in range(27):
        dz, dy, dx = S.tap_offset(tap)
        circ += np.tensordot(W[tap], np.roll(ext, (-dz, -dy, -dx), axis=(1, 2, 3)), axes=(1, 0))
    circ += b[:, None, None, None]
    np.testing.assert_allclose(S.conv(x, W, b), circ[..., :5], rtol=1e-12, atol=1e-12)


def test_conv_input_grad_is_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(4, 3, 5, 6))
    W = rng.normal(size=(27, 3, 4))
    dy = rng.normal(size=(3, 3, 5, 6))
    lhs = np.sum(S.conv(x, W, None) * dy)
    rhs = np.sum(x * S.conv_input_grad(dy, W))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_conv_is_equivariant_to_periodic_shifts():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 5, 6))
    W = rng.normal(size=(27, 3, 2))
    b = rng.normal(size=3)
    y = S.conv(x, W, b)
    xs = np.roll(x, (1, 2), axis=(1, 2))
    np.testing.assert_allclose(S.conv(xs, W, b), np.roll(y, (1, 2), axis=(1, 2)), rtol=1e-12, atol=1e-12)


def _tiny_problem(seed=3, C=3, depth=3, width=4):
    rng = np.random.default_rng(seed)
    shapes = [(C, 3, 2, 5), (C, 2, 3, 4)]
    fs = [rng.uniform(0.2, 1.0, size=s) for s in shapes]
    tg = [f + 0.05 * rng.normal(size=f.shape) for f in fs]
    norm = {"in_shift": np.full(C, 0.5), "in_scale": np.full(C, 2.0), "out_scale": np.full(C, 0.1)}
    p = S.he_init(C, depth, seed, width=width, gain=3.0).astype(np.float64)
    p += 0.1 * rng.normal(size=p.size)         # biases non-zero, ReLUs mixed
    return fs, tg, norm, p


def test_loss_gradient_matches_central_differences():
    C, depth, width = 3, 3, 4
    fs, tg, norm, p = _tiny_problem(C=C, depth=depth, width=width)
    w = np.array([1.0, 0.5, 2.0])
    L, g = S.loss_and_grad(p, fs, tg, norm, C, depth, width, weight=w)
    rng = np.random.default_rng(4)
    idx = rng.choice(p.size, 40, replace=False)
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        Lp, _ = S.loss_and_grad(pp, fs, tg, norm, C, depth, width, weight=w)
        Lm, _ = S.loss_and_grad(pm, fs, tg, norm, C, depth, width, weight=w)
        fd = (Lp - Lm) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_gradient_with_second_terms_and_conditioning():
    """Tied second-term weights and conditioning channels: the folded gradient
    still matches central differences."""
    C, depth, width, P = 3, 3, 4, 2
    fs, tg, norm, _ = _tiny_problem(C=C, depth=depth, width=width)
    cond = [np.array([0.3, -0.7]), np.array([1.1, 0.2])]
    p = S.he_init(C, depth, 9, width=width, gain=3.0, S=2).astype(np.float64)
    p += 0.1 * np.random.default_rng(10).normal(size=p.size)
    L, g = S.loss_and_grad(p, fs, tg, norm, C, depth, width, tubes_cond=cond, P=P)
    idx = list(range(0, 27 * width * (C + 2), 7))[:40]          # layer-0 weights, all column kinds
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        Lp, _ = S.loss_and_grad(pp, fs, tg, norm, C, depth, width, tubes_cond=cond, P=P)
        Lm, _ = S.loss_and_grad(pm, fs, tg, norm, C, depth, width, tubes_cond=cond, P=P)
        assert g[k] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5, abs=1e-9), k


def test_second_terms_carry_the_fields_exactly():
    """With tied weights, a layer-0 output equals the convolution of hi + lo / 256."""
    rng = np.random.default_rng(11)
    v = rng.normal(size=(3, 2, 3, 5))
    W = rng.normal(size=(27, 4, 3))
    hi, lo = S.two_term(v)
    a = np.concatenate([hi, lo])
    np.testing.assert_allclose(S.conv(a, S.expand_first(W, 3, 3), None), S.conv(hi + lo / 256, W, None),
                               rtol=1e-12, atol=1e-12)


def test_loss_is_zero_for_a_perfect_prediction():
    """All weights zero and the target equal to the fields: y = 0 = r."""
    C, depth, width = 3, 3, 4
    fs, _, norm, p = _tiny_problem(C=C, depth=depth, width=width)
    L, g = S.loss_and_grad(np.zeros_like(p), fs, fs, norm, C, depth, width)
    assert L == 0.0 and np.all(g == 0.0)


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = S.adam(p0, g, np.zeros(50), np.zeros(50), 1, 1e-3, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding():
    """BF16 keeps 7 fraction bits: the spacing at 1 is 2^-7."""
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -2.5, 3.0e-5])
    r = S.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                            # halfway: to the even neighbour 1
    assert r[2] == 1.0                            # below halfway
    assert r[3] == 1.0 + 2 ** -7                  # above halfway
    assert r[4] == 1.0 + 2 ** -6                  # halfway: to the even neighbour 1 + 2^-6
    assert r[5] == -2.5
    assert abs(r[6] - 3.0e-5) <= 3.0e-5 * 2 ** -8


def test_mole_residual_definition():
    """Fields X_1..X_3, T, u (3), p: the moles are sum p X_s / T."""
    rng = np.random.default_rng(6)
    a = rng.uniform(0.1, 1.0, size=(8, 2, 2, 7))
    assert S.mole_residual(a, a, 3) == 0.0
    b = a.copy()
    b[1] *= 1.01                                  # species 2 gains 1 % everywhere
    assert S.mole_residual(a, b, 3) == pytest.approx(0.01, rel=1e-12)
    c = a.copy()
    c[3] *= 2.0                                   # doubling T halves every species' moles
    assert S.mole_residual(a, c, 3) == pytest.approx(0.5, rel=1e-12)
    d = a.copy()
    d[7] *= 2.0
    d[3] *= 2.0                                   # p and T doubled together: same moles
    assert S.mole_residual(a, d, 3) == pytest.approx(0.0, abs=1e-14)


def test_two_term_encoding_resolves_16_bits():
    rng = np.random.default_rng(7)
    v = rng.normal(0, 2, 10000)
    hi, lo = S.two_term(v)
    v32 = v.astype(np.float32).astype(np.float64)
    assert np.all(S.bf16(hi) == hi) and np.all(S.bf16(lo) == lo)
    assert np.abs(v32 - hi).max() <= np.abs(v32).max() * 2 ** -8          # one term: ~8 bits
    assert np.all(np.abs(v32 - (hi + lo / 256)) <= np.abs(v32) * 2 ** -15)  # two terms: ~16 bits


def _cons_problem(seed=12, M=3, shape=(3, 4, 6)):
    rng = np.random.default_rng(seed)
    f = np.concatenate([rng.dirichlet([2.0] * M, size=shape).transpose(3, 0, 1, 2),
                        rng.uniform(0.3, 0.4, (1,) + shape), rng.normal(0, 1e-3, (3,) + shape),
                        rng.uniform(0.02, 0.03, (1,) + shape)])
    y = rng.normal(size=(3 * M + 4,) + shape)
    scale = np.concatenate([np.full(3 * M, 1e-4), [1e-3, 1e-4, 1e-4, 1e-4]])
    return f, y, scale


def test_conservative_output_keeps_moles_exactly():
    M = 3
    f, y, scale = _cons_problem(M=M)
    fo, n1 = S.conservative_fields(f, y, scale, M)
    moles = lambda g: np.array([np.sum(g[M + 4] * g[s] / g[M]) for s in range(M)])
    np.testing.assert_allclose(moles(fo), moles(f), rtol=1e-12)
    np.testing.assert_allclose(fo[:M].sum(axis=0), 1.0, rtol=1e-14)
    np.testing.assert_allclose(fo[M + 4], fo[M] * n1.sum(axis=0), rtol=1e-14)
    assert S.mole_residual(f, fo, M) < 1e-12
    # a flux on the wall face (x = nx - 1, +x direction) changes nothing
    y2 = np.zeros_like(y)
    y2[0][..., -1] = 5.0
    fo2, _ = S.conservative_fields(f, y2, scale, M)
    np.testing.assert_allclose(fo2, f, rtol=1e-14, atol=1e-16)
    # an interior +x flux moves moles from x to x + 1 only
    y3 = np.zeros_like(y)
    y3[0][1, 2, 3] = 1.0
    _, n3 = S.conservative_fields(f, y3, scale, M)
    n0 = f[M + 4] * f[:M] / f[M]
    d = n3[0] - n0[0]
    assert d[1, 2, 3] == pytest.approx(-1e-4) and d[1, 2, 4] == pytest.approx(1e-4)
    assert np.count_nonzero(np.abs(d) > 1e-15) == 2


@pytest.mark.parametrize("wf", [0.0, 3e5])
def test_conservative_loss_gradient_matches_central_differences(wf):
    """The adjoint of the divergence and of p = T sum n, X = n / sum n, and of the
    x-flux term (weight in the p slot)."""
    M = 3
    f, y, scale = _cons_problem(seed=13, M=M)
    tgt, _ = S.conservative_fields(f, 0.3 * np.random.default_rng(14).normal(size=y.shape), scale, M)
    w = np.array([1e6, 2e6, 5e5, 1e4, 1e5, 1e5, 1e5, wf])
    N = f[0].size
    L, dy = S.conservative_loss(f, y, tgt, w, scale, M, N)
    rng = np.random.default_rng(15)
    h = 1e-4                     # loss ~0.2, gradients ~1e-6: a smaller step is round-off
    for _ in range(40):
        idx = tuple(int(rng.integers(0, s)) for s in y.shape)
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        fd = (S.conservative_loss(f, yp, tgt, w, scale, M, N)[0] - S.conservative_loss(f, ym, tgt, w, scale, M, N)[0]) / (2 * h)
        assert dy[idx] == pytest.approx(fd, rel=1e-5, abs=1e-12), idx


def test_flux_target_reconstructs_the_fluxes_of_a_walled_tube():
    """Fields uniform in y and z, a target made by known x fluxes (none through the
    walls) and known T, u changes: the target fluxes, minus the change summed from
    the left wall, are those fluxes, so predicting them gives zero loss; a uniform
    offset on every interior face (invisible to the interior divergence) does not."""
    M = 3
    rng = np.random.default_rng(21)
    f, _, scale = _cons_problem(seed=22, M=M, shape=(1, 1, 9))
    f = np.repeat(np.repeat(f, 2, axis=1), 3, axis=2)          # [C][2][3][9], uniform in y, z
    y = np.zeros((3 * M + 4,) + f.shape[1:])
    for s in range(M):
        y[3 * s] = rng.normal(size=9)[None, None, :]
    y[3 * M:] = rng.normal(size=(4, 1, 1, 1))
    for s in range(M):
        y[3 * s][..., -1] = 0.0                               # the wall face
    tgt, _ = S.conservative_fields(f, y, scale, M)
    w = np.array([1e6, 2e6, 5e5, 1e4, 1e5, 1e5, 1e5, 3e5])
    L, dy = S.conservative_loss(f, y, tgt, w, scale, M, f[0].size)
    assert L < 1e-18 and np.abs(dy).max() < 1e-9
    y2 = y.copy()
    y2[0][..., :-1] += 0.1                                    # uniform offset, species 0
    _, n2 = S.conservative_fields(f, y2, scale, M)
    _, n1 = S.conservative_fields(f, y, scale, M)
    assert np.abs(n2 - n1)[..., 1:-1].max() < 1e-15           # the interior does not see it
    L2, _ = S.conservative_loss(f, y2, tgt, w * np.r_[np.zeros(7), 1.0], scale, M, f[0].size)
    assert L2 == pytest.approx(3e5 * (0.1 * 1e-4) ** 2 * 8 / 9, rel=1e-9)   # 8 open faces of 9 per row


def test_network_gradient_conservative_form():
    C, depth, width, M = 8, 3, 4, 3
    rng = np.random.default_rng(16)
    fs, tg = [], []
    for shape in [(2, 3, 5), (3, 2, 4)]:
        f, _, scale = _cons_problem(seed=int(rng.integers(100)), M=M, shape=shape)
        t, _ = S.conservative_fields(f, 0.5 * rng.normal(size=(3 * M + 4,) + shape), scale, M)
        fs.append(f)
        tg.append(t)
    norm = {"in_shift": np.full(C, 0.2), "in_scale": np.full(C, 3.0), "out_scale": scale}
    p = S.he_init(C, depth, 17, width=width, gain=3.0, species=M).astype(np.float64)
    p += 0.1 * rng.normal(size=p.size)
    w = np.array([1e6, 1e6, 1e6, 1e4, 1e5, 1e5, 1e5, 2e5])
    L, g = S.loss_and_grad(p, fs, tg, norm, C, depth, width, weight=w, species=M)
    h = 1e-6
    for k in rng.choice(p.size, 30, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        Lp, _ = S.loss_and_grad(pp, fs, tg, norm, C, depth, width, weight=w, species=M)
        Lm, _ = S.loss_and_grad(pm, fs, tg, norm, C, depth, width, weight=w, species=M)
        assert g[k] == pytest.approx((Lp - Lm) / (2 * h), rel=2e-5, abs=1e-10), k


def test_clip_grad_norm_definition():
    """Clipping by global norm: the clipped gradient has the limit as its norm and
    the direction of the original; below the limit, or with limit 0, nothing
    changes and the norm is reported."""
    g = np.array([3.0, -4.0, 12.0])                      # norm 13
    c, n = S.clip_grad_norm(g, 6.5)
    assert n == 13.0
    np.testing.assert_allclose(c, g / 2.0, rtol=1e-15)
    assert np.sqrt(np.sum(c * c)) == pytest.approx(6.5, rel=1e-15)
    c2, n2 = S.clip_grad_norm(g, 20.0)
    np.testing.assert_array_equal(c2, g)
    c3, n3 = S.clip_grad_norm(g, 0.0)
    np.testing.assert_array_equal(c3, g)
    assert n2 == n3 == 13.0

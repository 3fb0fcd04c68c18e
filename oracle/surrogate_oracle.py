"""FP64 reference of the learned surrogate (test infrastructure only).

Plain numpy, written from the definitions, not from the GPU kernels:

- a 3x3x3 convolution, output o = b[o] + sum over taps (dz, dy, dx) and input
  channels i of W[tap][o][i] * in[i](z + dz, y + dy, x + dx), tap = 9 (dz+1) +
  3 (dy+1) + (dx+1), with periodic wrapping in y and z and, at the x ends of a
  tube (its walls), replicate padding: the value outside a wall is that of the
  wall node, the mirror image that a wall without flux implies;
- the network: layer 0 maps C field channels to the hidden width, ReLU between
  layers, the last layer maps back to C; its input is the normalised fields
  (f - shift) * scale, its output the change of the normalised fields;
- the conservative output form: the network predicts, per species, the fluxes
  of the molar density n_s = p X_s / T through the faces between x and x + e_a
  (none through the walls); n_s changes by minus their discrete divergence;
  then p = T sum n and X_s = n_s / sum n;
- the mean squared error and its gradient by the chain rule (the gradient of a
  convolution with respect to its input is the adjoint gather, the transposed
  weights scattered back along the tap offsets; with respect to the weights, the
  correlation of the output gradient with the shifted input); in the
  conservative form also the error of the fluxes through the x faces against
  those the target change implies on a walled tube with fields uniform in y and
  z, which fixes the uniform flux offset that the divergence cannot see;
- Adam as published by Kingma and Ba (bias-corrected first and second moments),
  optionally after clipping the gradient by its global Euclidean norm;
- the mole residual: with R_U = 1 the molar density of species s is
  rho_s / m_s = p X_s / T, so a tube's moles are sum_x p X_s / T.

Optionally the forward and backward passes round to BF16 (round to nearest
even) at the points where the GPU kernels store BF16 (the packed input, the
weights, the hidden activations, the activation gradients), so that a
comparison isolates the FP32-versus-FP64 accumulation.

Pins (tests/test_surrogate_oracle.py): brute-force loops, the adjoint identity,
central finite differences of the loss, the closed-form first Adam step,
equivariance under periodic shifts.
"""
from __future__ import annotations

import numpy as np

NTAP = 27


def tap_offset(tap: int):
    return tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to BF16 (nearest even) through FP32, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[..., z, y, x] = x[..., z + dz, y + dy, clamp(x + dx)]: periodic in z and
    y, the x index clamped to [0, nx - 1] (replicate padding at the walls)."""
    s = np.roll(x, shift=(-dz, -dy), axis=(-3, -2))
    nx = s.shape[-1]
    idx = np.clip(np.arange(nx) + dx, 0, nx - 1)
    return s[..., idx]


def shift_adjoint(g: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """Adjoint of shift: out[..., z + dz, y + dy, clamp(x + dx)] += g[..., z, y, x],
    so the values gathered twice at a wall (its own and its ghost's) send both
    contributions back to the wall node."""
    nx = g.shape[-1]
    idx = np.clip(np.arange(nx) + dx, 0, nx - 1)
    out = np.zeros_like(g)
    np.add.at(out, (Ellipsis, idx), g)        # scatter along x (repeated indices add)
    return np.roll(out, shift=(dz, dy), axis=(-3, -2))


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray | None) -> np.ndarray:
    """x [Cin][nz][ny][nx], W [27][Cout][Cin], b [Cout] -> [Cout][nz][ny][nx]."""
    y = np.zeros((W.shape[1],) + x.shape[1:])
    for tap in range(NTAP):
        y += np.tensordot(W[tap], shift(x, *tap_offset(tap)), axes=(1, 0))
    if b is not None:
        y += b[:, None, None, None]
    return y


def conv_input_grad(dy: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv with respect to x: sum_tap shift_adjoint(W[tap]^T dy, d_tap)."""
    dx = np.zeros((W.shape[2],) + dy.shape[1:])
    for tap in range(NTAP):
        dx += shift_adjoint(np.tensordot(W[tap].T, dy, axes=(1, 0)), *tap_offset(tap))
    return dx


def conv_weight_grad(dy: np.ndarray, x: np.ndarray):
    """dW[tap][o][i] = sum_nodes dy[o] x[i](. + d_tap); db[o] = sum_nodes dy[o]."""
    Cout, Cin = dy.shape[0], x.shape[0]
    dW = np.zeros((NTAP, Cout, Cin))
    dyf = dy.reshape(Cout, -1)
    for tap in range(NTAP):
        dW[tap] = dyf @ shift(x, *tap_offset(tap)).reshape(Cin, -1).T
    return dW, dyf.sum(axis=1)


# ------------------------------------------------------------------ network
def layer_shapes(C: int, depth: int, width: int = 64, S: int = 0, species: int = 0):
    """S counts the conditioning channels of layer 0 (the tied second terms add no
    parameters); species > 0: conservative output, 3 species + 4 channels."""
    ins = [C + S] + [width] * (depth - 1)
    outs = [width] * (depth - 1) + [3 * species + 4 if species else C]
    return list(zip(outs, ins))


def param_count(C: int, depth: int, width: int = 64, S: int = 0, species: int = 0) -> int:
    return sum(NTAP * o * i + o for o, i in layer_shapes(C, depth, width, S, species))


def unflatten(params: np.ndarray, C: int, depth: int, width: int = 64, S: int = 0, species: int = 0):
    """Flat parameters (layer by layer: W[tap][out][in], then b[out]) -> list of (W, b)."""
    out, k = [], 0
    for o, i in layer_shapes(C, depth, width, S, species):
        W = params[k:k + NTAP * o * i].reshape(NTAP, o, i)
        k += NTAP * o * i
        b = params[k:k + o]
        k += o
        out.append((np.asarray(W, dtype=np.float64), np.asarray(b, dtype=np.float64)))
    assert k == params.size
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def he_init(C: int, depth: int, seed: int, width: int = 64, gain: float = 1.0, S: int = 0,
            species: int = 0) -> np.ndarray:
    """Seeded He-normal weights, zero biases (the starting point of training)."""
    rng = np.random.default_rng(seed)
    layers = []
    for k, (o, i) in enumerate(layer_shapes(C, depth, width, S, species)):
        std = np.sqrt(2.0 / (NTAP * i)) * (gain if k < depth - 1 else 0.1 * gain)
        layers.append((rng.normal(0.0, std, (NTAP, o, i)), np.zeros(o)))
    return flatten(layers).astype(np.float32)


def two_term(v: np.ndarray):
    """hi = bf16(v), lo = bf16((v - hi) 256), v taken in FP32 first: hi + lo / 256
    carries about 16 significant bits of v."""
    v32 = np.asarray(v, dtype=np.float32).astype(np.float64)
    hi = bf16(v32)
    return hi, bf16((v32 - hi) * 256.0)


def expand_first(W: np.ndarray, C: int, P: int) -> np.ndarray:
    """Layer-0 weights over the input columns [fields, second terms, conditioning]:
    a second term reuses its field's weights divided by 256."""
    if P == 0:
        return W
    return np.concatenate([W[:, :, :C], W[:, :, :P] / 256.0, W[:, :, C:]], axis=2)


def fold_first(g: np.ndarray, C: int, P: int) -> np.ndarray:
    """Gradient with respect to the expanded layer-0 weights -> the parameters."""
    if P == 0:
        return g
    out = np.concatenate([g[:, :, :C], g[:, :, C + P:]], axis=2)
    out[:, :, :P] += g[:, :, C:C + P] / 256.0
    return out


def _down(F, a):
    """F(x - e_a): zero below x = 0 (walls), periodic in y (a = 1) and z (a = 2)."""
    if a == 0:
        out = np.zeros_like(F)
        out[..., 1:] = F[..., :-1]
        return out
    return np.roll(F, 1, axis=-2 if a == 1 else -3)


def _up(g, a):
    """g(x + e_a) (the value at x = nx - 1 for a = 0 is never used: that face is a wall)."""
    if a == 0:
        out = np.zeros_like(g)
        out[..., :-1] = g[..., 1:]
        return out
    return np.roll(g, -1, axis=-2 if a == 1 else -3)


def conservative_fields(f, y, out_scale, M):
    """New fields [X_1..X_M, T, u, p] from fields f (same layout) and the raw
    output y [3M + 4][...] of the conservative form; also returns n' [M][...]."""
    T, p = f[M], f[M + 4]
    n = p * f[:M] / T
    n1 = np.empty_like(n)
    for s in range(M):
        div = np.zeros_like(T)
        for a in range(3):
            F = y[3 * s + a] * out_scale[3 * s + a]
            if a == 0:
                F = F.copy()
                F[..., -1] = 0.0                      # the face at the wall carries no flux
            div += F - _down(F, a)
        n1[s] = n[s] - div
    T1 = T + y[3 * M] * out_scale[3 * M]
    u1 = f[M + 1:M + 4] + y[3 * M + 1:3 * M + 4] * out_scale[3 * M + 1:3 * M + 4, None, None, None]
    tot = n1.sum(axis=0)
    return np.concatenate([n1 / tot, T1[None], u1, (T1 * tot)[None]]), n1


def conservative_loss(f, y, target, w, out_scale, M, N):
    """Loss contribution of one tube (sum over its nodes, divided by the total N)
    and its gradient with respect to y."""
    fo, n1 = conservative_fields(f, y, out_scale, M)
    nt = target[M + 4] * target[:M] / target[M]
    e = n1 - nt
    loss = float(np.sum(w[:M, None, None, None] * e * e))
    g = 2.0 * w[:M, None, None, None] * e / N
    dy = np.zeros_like(y)
    for s in range(M):
        for a in range(3):
            d = (_up(g[s], a) - g[s]) * out_scale[3 * s + a]
            if a == 0:
                d[..., -1] = 0.0
            dy[3 * s + a] = d
    for k in range(4):
        e = fo[M + k] - target[M + k]
        loss += float(np.sum(w[M + k] * e * e))
        dy[3 * M + k] = 2.0 * w[M + k] * e * out_scale[3 * M + k] / N
    # the x-flux term, weight w[M + 4] (the p slot, which this form does not fit):
    # on a tube with walls and fields uniform in y and z, the flux of n_s through
    # the face between x and x + 1 that the target change implies is minus the
    # change summed from the left wall up to x (nothing enters through the wall)
    wf = w[M + 4] if len(w) > M + 4 else 0.0
    if wf:
        n0 = f[M + 4] * f[:M] / f[M]
        Fstar = -np.cumsum(nt - n0, axis=-1)
        for s in range(M):
            e = y[3 * s] * out_scale[3 * s] - Fstar[s]
            e[..., -1] = 0.0                          # the wall face: no flux, not fitted
            loss += float(np.sum(wf * e * e))
            dy[3 * s] += 2.0 * wf * e * out_scale[3 * s] / N
    return loss / N, dy


def forward(params, f, norm, C, depth, width=64, round_bf16=False, cond=None, P=0, species=0):
    """One tube: f [C][nz][ny][nx] fields, cond [S] constants of the tube, P
    leading field channels also given as a second BF16 term (tied weights) ->
    (y raw output, pred fields, cache)."""
    S = 0 if cond is None else len(cond)
    layers = unflatten(np.asarray(params, dtype=np.float64), C, depth, width, S, species)
    rnd = bf16 if round_bf16 else (lambda a: a)
    v = (f - norm["in_shift"][:, None, None, None]) * norm["in_scale"][:, None, None, None]
    if P:
        hi, lo = two_term(v)
        a = np.concatenate([hi, lo[:P]])
    else:
        a = rnd(v)
    if S:
        a = np.concatenate([a, np.broadcast_to(np.asarray(cond, dtype=np.float64)[:, None, None, None],
                                               (S,) + f.shape[1:])])
    a = rnd(a)
    acts = [a]
    for k, (W, b) in enumerate(layers):
        if k == 0:
            W = expand_first(W, C, P)
        z = conv(acts[-1], rnd(W), b)
        if k < depth - 1:
            acts.append(rnd(np.maximum(z, 0.0)))
        else:
            y = z
    if species:
        pred, _ = conservative_fields(f, y, norm["out_scale"], species)
    else:
        pred = f + y * norm["out_scale"][:, None, None, None]
    return y, pred, acts


def loss_and_grad(params, tubes_f, tubes_target, norm, C, depth, width=64, weight=None, round_bf16=False,
                  tubes_cond=None, P=0, species=0):
    """Mean over all nodes of all tubes of sum_c w_c (y_c - r_c)^2 with
    r = (target - f) / out_scale, and its gradient with respect to the flat
    parameters (same order)."""
    S = 0 if tubes_cond is None else len(tubes_cond[0])
    layers = unflatten(np.asarray(params, dtype=np.float64), C, depth, width, S, species)
    w = np.ones(C) if weight is None else np.asarray(weight, dtype=np.float64)
    rnd = bf16 if round_bf16 else (lambda a: a)
    N = sum(f[0].size for f in tubes_f)
    total = 0.0
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    for t, (f, tgt) in enumerate(zip(tubes_f, tubes_target)):
        cond = None if tubes_cond is None else tubes_cond[t]
        y, _, acts = forward(params, f, norm, C, depth, width, round_bf16, cond, P, species)
        if species:
            lt, d = conservative_loss(f, y, tgt, w, norm["out_scale"], species, N)
            total += lt * N
            d = rnd(d)
        else:
            r = (tgt - f) / norm["out_scale"][:, None, None, None]
            e = y - r
            total += float(np.sum(w[:, None, None, None] * e * e))
            d = rnd(2.0 * w[:, None, None, None] * e / N)
        for k in range(depth - 1, -1, -1):
            W, _ = layers[k]
            dW, db = conv_weight_grad(d, acts[k])
            if k == 0:
                dW = fold_first(dW, C, P)
            grads[k][0][...] += dW
            grads[k][1][...] += db
            if k > 0:
                d = rnd(conv_input_grad(d, rnd(W)) * (acts[k] > 0))
    return total / N, flatten(grads)


def clip_grad_norm(grad, max_norm):
    """Clipping by global norm: (grad scaled by max_norm / |grad| when |grad| >
    max_norm > 0, else grad unchanged; |grad|), |.| the Euclidean norm over all
    parameters."""
    g = np.asarray(grad, dtype=np.float64)
    norm = float(np.sqrt(np.sum(g * g)))
    if max_norm > 0.0 and np.isfinite(norm) and norm > max_norm:
        return g * (max_norm / norm), norm
    return g.copy(), norm


def adam(params, grad, m, v, step, lr, b1, b2, eps):
    """One Adam step (Kingma and Ba): returns new (params, m, v); step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def mole_residual(a: np.ndarray, b: np.ndarray, M: int) -> float:
    """max_s |S_s(b) - S_s(a)| / S_s(a), S_s = sum p X_s / T, for one tube's fields
    [C][...] laid out X_1..X_M, T, u_x, u_y, u_z, p."""
    sa = np.array([np.sum(a[M + 4] * a[s] / a[M]) for s in range(M)])
    sb = np.array([np.sum(b[M + 4] * b[s] / b[M]) for s in range(M)])
    return float(np.max(np.abs(sb - sa) / np.abs(sa)))

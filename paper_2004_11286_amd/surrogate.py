"""The learned surrogate end to end: trajectories from a batched ensemble of
tubes, normalisation from the data, training, and evaluation against the
lattice Boltzmann step (the judge of its error).

Only orchestration lives here: every field read-back, forward and backward
pass, loss, optimiser step, residual and lattice step is a call into the C ABI
of libmclbm (include/mclbm.h, include/mclbm_nn.h); torch holds the snapshot
tensors on the device.
"""
from __future__ import annotations

import time

import numpy as np

from . import mclbm as mc

DEPTH = 6
K_DEFAULT = 100
LR = 1e-4          # larger rates let one late, heavily weighted pair's gradient spike kill the
                   # ReLUs (the loss jumps to that of predicting no change and stays there)


def channels(M: int) -> int:
    return M + 5                      # X_1..X_M, T, u_x, u_y, u_z, p


def conditioning(params: dict) -> np.ndarray:
    """Per-tube constants the evolution depends on but the fields do not show:
    molar masses / 40 and the off-diagonal diffusivities / 0.1."""
    M = int(params["M"])
    m = np.asarray(params["molar_mass"], dtype=np.float64) / 40.0
    D = np.asarray(params["D"], dtype=np.float64)
    iu = np.triu_indices(M, 1)
    return np.concatenate([m, D[iu] / 0.1]).astype(np.float32)


def trajectories(tubes: list, K: int = K_DEFAULT, nsnap: int = 50, precision: int = mc.MCLBM_FP32):
    """Run the tubes as one batched context and keep the FP32 fields every K
    steps: a device tensor [nsnap + 1][(M+5) n] and the tube sizes."""
    import torch

    b = mc.Batch([p for p, _ in tubes], precision)
    b.init_fields([f for _, f in tubes])
    C = channels(b.M)
    snaps = torch.empty((nsnap + 1, C * b.n), dtype=torch.float32, device=b.device)
    b.read_fields_f32(out=snaps[0])
    for j in range(nsnap):
        b.step(K)
        b.read_fields_f32(out=snaps[j + 1])
    torch.cuda.synchronize()
    dims = [(s[2], s[1], s[0]) for s in b.shapes]
    b.close()
    # a tube whose state left the lattice's stable range shows as non-finite fields
    last = snaps[-1].cpu().numpy()
    off, bad = 0, []
    for t, (nx, ny, nz) in enumerate(dims):
        n = nx * ny * nz
        if not np.all(np.isfinite(last[C * off:C * (off + n)])):
            bad.append(t)
        off += n
    if bad:
        raise ValueError(f"tubes {bad} became non-finite within {K * nsnap} steps; leave them out of the ensemble")
    return snaps, dims


def molar_densities(x: np.ndarray, M: int) -> np.ndarray:
    """n_s = p X_s / T from fields [..., C, n] (X_1..X_M, T, u, p)."""
    return x[..., M + 4:M + 5, :] * x[..., :M, :] / x[..., M:M + 1, :]


def _tube_views(x, dims, C, stride=256):
    """Per tube: [snapshots][C][subsampled nodes] views of the flat snapshots."""
    sizes = [nx * ny * nz for nx, ny, nz in dims]
    off = np.concatenate([[0], np.cumsum(sizes)])
    for t, n in enumerate(sizes):
        yield x[:, C * off[t]:C * off[t + 1]].reshape(x.shape[0], C, n)[:, :, ::max(1, n // stride)]


def x_flux_targets(x: np.ndarray, dims, C: int, M: int) -> np.ndarray:
    """The x fluxes the snapshot changes imply along the first x row of each tube,
    F*_s(x) = -sum_{x' <= x} dn_s(x') (the target of the x-flux loss term; exact for
    fields uniform in y and z, as in these tubes): [pairs][M][sum of nx] (host)."""
    sizes = [nx * ny * nz for nx, ny, nz in dims]
    off = np.concatenate([[0], np.cumsum(sizes)])
    rows = []
    for t, (nx, ny, nz) in enumerate(dims):
        seg = x[:, C * off[t]:C * off[t + 1]].reshape(x.shape[0], C, sizes[t])[:, :, :nx]
        n = molar_densities(seg, M)
        rows.append(-np.cumsum(n[1:] - n[:-1], axis=-1))
    return np.concatenate(rows, axis=-1)


def channel_stats(snaps, dims, M: int) -> dict:
    """Spreads from the trajectories (host, subsampled nodes): of every field,
    of its change over one interval, of the change of each molar density n_s (per
    interval, for the loss weights) and of the implied x fluxes of n_s."""
    x = snaps.cpu().numpy().astype(np.float64)
    C = channels(M)
    segs = list(_tube_views(x, dims, C))
    allf = np.concatenate([s for s in segs], axis=2)
    d = allf[1:] - allf[:-1]
    n = np.concatenate([molar_densities(s, M) for s in segs], axis=2)
    dn = n[1:] - n[:-1]
    F = x_flux_targets(x, dims, C, M)
    return {"mean": allf.mean(axis=(0, 2)), "std": allf.std(axis=(0, 2)), "dstd": d.std(axis=(0, 2)),
            "dn_std": dn.std(axis=(0, 2)), "dn_ms_pair": (dn ** 2).mean(axis=2),
            "Fx_std": np.sqrt((F ** 2).mean(axis=(0, 2))), "Fx_ms_pair": (F ** 2).mean(axis=2)}


IN_FLOOR = 1e-3      # smallest input spread used for scaling (T and u vary by ~1e-3)
OUT_FLOOR = 1e-4     # smallest output unit (a channel that never changes, e.g. u_y in a 1-D tube)


def norm_from_stats(st: dict, M: int) -> dict:
    """Inputs to zero mean and unit spread; outputs (conservative form): the x
    fluxes of n_s in units of their typical size, the y and z fluxes in units of
    the typical change of n_s, T and u in units of their typical change; floors
    keep channels that (almost) never vary from being blown up to round-off."""
    in_scale = 1.0 / np.maximum(st["std"], IN_FLOOR)
    flux = np.repeat(np.maximum(st["dn_std"], 1e-7), 3)
    flux[0::3] = np.maximum(st["Fx_std"], 1e-7)
    tu = np.maximum(st["dstd"][M:M + 4], OUT_FLOOR)
    return {"in_shift": st["mean"].astype(np.float32), "in_scale": in_scale.astype(np.float32),
            "out_scale": np.concatenate([flux, tu]).astype(np.float32)}


def he_init(C: int, S: int, depth: int, seed: int, out: int) -> np.ndarray:
    """He-normal weights for the ReLU layers, a small last layer, zero biases
    (host order of include/mclbm_nn.h)."""
    rng = np.random.default_rng(seed)
    width = 64
    ins = [C + S] + [width] * (depth - 1)
    outs = [width] * (depth - 1) + [out]
    parts = []
    for k, (o, i) in enumerate(zip(outs, ins)):
        std = np.sqrt(2.0 / (27 * i)) * (1.0 if k < depth - 1 else 0.1)
        parts += [rng.normal(0.0, std, 27 * o * i), np.zeros(o)]
    return np.concatenate(parts).astype(np.float32)


def build_net(dims, tubes_params, norm, M: int, depth: int = DEPTH, params=None, seed: int = 0):
    """The surrogate over these tubes: conservative output form (species moles
    kept exactly), the M mole fractions also as second BF16 terms, the tube
    constants as conditioning channels."""
    C = channels(M)
    cond = np.stack([conditioning(p) for p in tubes_params])
    net = mc.Net(C, depth, dims, conditioning=cond.shape[1], two_term=M, species=M)
    net.set_conditioning(cond)
    net.set_norm(norm["in_shift"], norm["in_scale"], norm["out_scale"])
    net.set_params(he_init(C, cond.shape[1], depth, seed, 3 * M + 4) if params is None else params)
    return net


def pair_weights(st: dict, M: int, floor_frac: float = 1e-2, flux_weight: float = 0.1) -> np.ndarray:
    """Loss weights per snapshot pair in physical units: the molar densities by
    the pair's own mean squared change (a relative error, so late, slow
    intervals count as much as early ones), T and u by their typical change at
    weights 0.2 and 0.1, and the x fluxes (the p slot) by flux_weight over the
    pair's mean squared x flux (also relative). Returns [nsnap][C]."""
    C = channels(M)
    ms = st["dn_ms_pair"]
    floor = floor_frac * ms.mean(axis=0)
    out = np.zeros((ms.shape[0], C), dtype=np.float64)
    out[:, :M] = 1.0 / np.maximum(ms, floor)
    msF = st["Fx_ms_pair"].mean(axis=1)
    out[:, M + 4] = flux_weight / np.maximum(msF, floor_frac * msF.mean())
    out[:, M] = 0.2 / np.maximum(st["dstd"][M], OUT_FLOOR) ** 2
    out[:, M + 1:M + 4] = 0.1 / np.maximum(st["dstd"][M + 1:M + 4], OUT_FLOOR) ** 2
    return out.astype(np.float32)


def train(net, snaps, iters: int, weights, lr: float = LR, seed: int = 0, log_every: int = 0,
          warmup: int = 500, clip: float = 0.0):
    """Adam on random (t, t + K) snapshot pairs of all tubes at once, with a
    linear learning-rate warm-up over the first `warmup` iterations and a cosine
    decay after; weights: per-pair channel weights [nsnap][C]. clip > 0 clips
    the gradient by its global norm at clip times a running mean of the recent
    (clipped) norms, so that a single outlying pair cannot throw the weights far.
    Returns the loss history."""
    rng = np.random.default_rng(seed)
    losses = []
    nsnap = snaps.shape[0] - 1
    norm_mean = None
    for it in range(iters):
        j = int(rng.integers(0, nsnap))
        net.fields_in.copy_(snaps[j])
        net.forward()
        losses.append(net.loss(snaps[j + 1], weights[j]))
        net.backward()
        if clip > 0.0:
            limit = 0.0 if norm_mean is None or it < 50 else clip * norm_mean
            nrm = net.clip_grad_norm(limit)
            if np.isfinite(nrm):
                kept = min(nrm, limit) if limit > 0.0 else nrm
                norm_mean = kept if norm_mean is None else 0.98 * norm_mean + 0.02 * kept
        lr_it = (lr * 0.5 * (1.0 + np.cos(np.pi * it / iters)) + 0.02 * lr) * min(1.0, (it + 1) / max(warmup, 1))
        net.adam_step(lr_it)
        if log_every and (it + 1) % log_every == 0:
            print(f"  iter {it + 1}: loss {np.mean(losses[-log_every:]):.4g}", flush=True)
    return losses


def evaluate(params, norm, eval_tubes, K: int = K_DEFAULT, starts=(0, 500, 2000), depth: int = DEPTH,
             resid_tol: float = 1e-4, change_tol: float = float("inf")):
    """Judge the surrogate by the lattice: from the same state at each start
    time, K lattice steps against one network hop. Reports the mole-fraction
    error (L-infinity over all tubes), that of the persistence prediction (no
    change), the mole residual, the two quantities the advance entry point
    gates on (the residual, the largest relative change of a species' mass or
    of the energy per tube, for the network and for the K lattice steps; the
    change, the largest mole-fraction change the hop predicts), whether the hop
    was accepted, and the times of the hop (read, forward, residual and
    re-initialisation through mclbm_nn_advance) and of the K lattice steps."""
    import torch

    b = mc.Batch([p for p, _ in eval_tubes], mc.MCLBM_FP32)
    ref = mc.Batch([p for p, _ in eval_tubes], mc.MCLBM_FP32)
    dims = [(s[2], s[1], s[0]) for s in b.shapes]
    M = b.M
    C = channels(M)
    net = build_net(dims, [p for p, _ in eval_tubes], norm, M, depth, params)
    fields = [f for _, f in eval_tubes]
    # one accepted hop, untimed, so that the timed ones do not carry the first
    # use of the re-initialisation path (every start re-initialises b anyway)
    b.init_fields(fields)
    net.advance(b, K, float("inf"), float("inf"))
    out = []
    for t0 in starts:
        for x in (b, ref):
            x.init_fields(fields)
            x.step(t0)
        # lattice reference: K steps, timed on the stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start = ref.read_fields_f32().clone()
        c0 = ref.conservation()
        e0.record(ref.stream)
        ref.step(K)
        e1.record(ref.stream)
        e1.synchronize()
        t_lbm = e0.elapsed_time(e1)
        want = ref.read_fields_f32().clone()
        c1 = ref.conservation()
        keep = np.concatenate([np.arange(M), [M + 4]])         # species masses and the energy
        lat_res = float(np.max(np.abs(c1[:, keep] - c0[:, keep]) / np.abs(c0[:, keep])))
        # network prediction from the same state (forward only, for the error)
        net.fields_in.copy_(start)
        net.forward()
        torch.cuda.synchronize()
        pred = net.fields_out.clone()
        res = net.mole_residual(M, start, pred)
        res_lattice = net.mole_residual(M, start, want)
        # the advance entry point end to end (timed on the stream)
        e0.record(b.stream)
        used, res_adv, chg_adv = net.advance(b, K, resid_tol, change_tol)
        e1.record(b.stream)
        e1.synchronize()
        t_adv = e0.elapsed_time(e1)
        # forward pass alone
        e0.record(net.stream)
        net.forward()
        e1.record(net.stream)
        e1.synchronize()
        t_fwd = e0.elapsed_time(e1)

        def xerr(a):
            """(L-infinity, RMS) of the mole-fraction error over all tubes."""
            ea, eb = a.cpu().numpy(), want.cpu().numpy()
            linf, sq, cnt = 0.0, 0.0, 0
            off = 0
            for nx, ny, nz in dims:
                n = nx * ny * nz
                d = ea[C * off:C * (off + n)].reshape(C, n)[:M] - eb[C * off:C * (off + n)].reshape(C, n)[:M]
                linf = max(linf, float(np.abs(d).max()))
                sq += float(np.sum(d.astype(np.float64) ** 2))
                cnt += d.size
                off += n
            return linf, (sq / cnt) ** 0.5

        (e_inf, e_rms), (p_inf, p_rms) = xerr(pred), xerr(start)
        out.append({"t0": int(t0), "K": int(K), "X_linf": e_inf, "X_linf_persistence": p_inf,
                    "X_rms": e_rms, "X_rms_persistence": p_rms,
                    "mole_residual_max": float(np.max(res)),
                    "lattice_mole_residual_max": float(np.max(res_lattice)),
                    "state_residual": float(res_adv), "lattice_state_residual": lat_res,
                    "state_change": float(chg_adv), "resid_tol": float(resid_tol),
                    "change_tol": float(change_tol), "accepted": not used,
                     "ms_lattice": t_lbm, "ms_advance": t_adv, "ms_forward": t_fwd})
    net.close()
    b.close()
    ref.close()
    return out


def calibrate_change_tol(hops, bar: float = 1e-3) -> float:
    """The advance gate's change threshold from calibration hops judged by the
    lattice (dicts with "X_linf", the hop's mole-fraction error, and
    "state_change", the largest change it predicts): the largest change among
    hops within `bar` that lies strictly below the change of every hop outside
    it, so that every calibration hop with a change at most the threshold is
    within the bar; 0 when no hop qualifies."""
    bad_min = min((h["state_change"] for h in hops if h["X_linf"] > bar), default=float("inf"))
    below = [h["state_change"] for h in hops if h["X_linf"] <= bar and h["state_change"] < bad_min]
    return max(below) if below else 0.0


def conv_flops_per_node(C: int, S: int, out: int, depth: int = DEPTH, width: int = 64) -> float:
    """Multiply-adds x 2 of one forward pass per node over the real channels
    (layer 0: fields, second terms and conditioning, C + S inputs; last layer:
    out outputs)."""
    ins = [C + S] + [width] * (depth - 1)
    outs = [width] * (depth - 1) + [out]
    return float(sum(2 * 27 * o * i for o, i in zip(outs, ins)))


def timed_train_step(net, snaps, weights, reps: int = 20):
    """Milliseconds of one forward + loss + backward + Adam step (mean of reps)."""
    import torch

    w = weights[0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    net.fields_in.copy_(snaps[0])
    t0 = time.perf_counter()
    e0.record(net.stream)
    for _ in range(reps):
        net.forward()
        net.loss(snaps[1], w)
        net.backward()
        net.adam_step(1e-6)
    e1.record(net.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps, (time.perf_counter() - t0) * 1e3 / reps

"""Learned warm start of the pressure solve: training data from the solver,
training of the U-Net on the GPU, and its use as the initial guess.

Orchestration only: the snapshots are written by the solver library's kernels
(ibm_set_snapshot), training steps and inference run in the network's BF16
matrix-core kernels (ibm_unet_*), and the solve with the learned guess is the
library's own time step (IBM_INIT_LEARNED).  PyTorch holds the snapshot
tensors and cuts the training crops out of them.

The network predicts phi^{n+1} - phi^n from the maps of the step's Poisson
problem (residual of phi^n, phi^n, body mask), in units of out_scale times the
RMS of that residual; out_scale is the RMS of the targets over the training
set, so the network's targets have unit RMS.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import ibm
from . import unet as U


def solver_for(wl: dict, **over):
    prm = dict(wl["params"])
    prm.update(over)
    return ibm.Solver(wl["nx"], wl["ny"], wl["xf"], wl["yf"], wl["u0"], wl["v0"], wl["p0"], **prm)


def _net_options(s, factor, options=None):
    if s.set_option(ibm.OPT_NET_FACTOR, factor) != ibm.OK:
        raise ValueError(f"coarsening factor {factor} does not divide the grid")
    for opt, val in (options or {}).items():
        if s.set_option(opt, val) != ibm.OK:
            raise ValueError(f"option {opt} = {val}")


def collect(wl: dict, cases, steps: int, keep_from: int = 1, factor: int = 1, snap_iters=(0,), policy=None,
            options=None):
    """Snapshots of the network's maps and targets on the grid coarsened by
    `factor`.  Each case (a dict of parameter overrides of the workload) is
    advanced `steps` steps by PCG; for every step >= keep_from (1-based) and
    every k in snap_iters one snapshot is taken: k = 0 at the start of the
    solve (phi_s = phi^n), k > 0 after k red-black SOR iterations from phi^n
    (PCG finishes that solve).  With a policy (dict: params, out_scale,
    every, options, guess) the k > 0 snapshots follow the solve that network
    guides: a correction every `every` iterations (and its guess at the start
    when guess is true), so that the snapshots show the states the network
    meets in use.  options: solver options of the network (e.g. its maps) for
    every solver.  Returns float32 device tensors feats
    (N, 3, ny/F, nx/F) and targets (N, 1, ny/F, nx/F), targets in units of
    s_r, the k of each snapshot, and the seconds spent."""
    import torch
    ny, nx = wl["ny"] // factor, wl["nx"] // factor
    feats, targets, ks = [], [], []
    t0 = time.perf_counter()
    for case in cases:
        drv = solver_for(wl, p_method=ibm.PCG, p_init_prev=ibm.INIT_PREVIOUS, **case)
        _net_options(drv, factor, options)
        mid = solver_for(wl, p_method=ibm.RBSOR,
                         p_init_prev=ibm.INIT_LEARNED if policy and policy.get("guess") else ibm.INIT_PREVIOUS,
                         **case) \
            if any(k > 0 for k in snap_iters) else None
        if mid is not None:
            _net_options(mid, factor, options)
            if policy:
                pnet = U.UNet(1, ny, nx, device=mid.device, stream=mid.stream)
                pnet.set_params(policy["params"])
                opts = dict(policy.get("options") or {})
                opts[ibm.OPT_NET_EVERY] = policy["every"]
                for opt, val in opts.items():
                    if mid.set_option(opt, val) != ibm.OK:
                        raise ValueError(f"option {opt} = {val}")
                mid.set_warm_start(pnet, policy["out_scale"])
        f = torch.empty((3, ny, nx), dtype=torch.float32, device=drv.device)
        t = torch.empty((ny, nx), dtype=torch.float32, device=drv.device)
        for step in range(1, steps + 1):
            keep = step >= keep_from
            blob = drv.get_state() if keep and mid is not None else None
            drv.set_snapshot(f, t, 1.0) if keep and 0 in snap_iters else drv.set_snapshot(None, None)
            st = drv.step(1)
            if st["rc"] < 0:
                raise ibm.IbmError(f"snapshot run failed at step {step}: {ibm.status_string(st['rc'])}")
            if keep and 0 in snap_iters:
                feats.append(f.clone())
                targets.append(t.clone().unsqueeze(0))
                ks.append(0)
            for k in snap_iters:
                if k <= 0 or not keep:
                    continue
                mid.set_state(blob)
                if mid.set_option(ibm.OPT_SNAPSHOT_ITER, k) != ibm.OK:
                    raise ValueError(f"snapshot iteration {k}: not a multiple of the check interval")
                mid.set_snapshot(f, t, 1.0)
                st = mid.step(1)
                if st["rc"] < 0:
                    raise ibm.IbmError(f"snapshot run failed at step {step}, k {k}")
                feats.append(f.clone())
                targets.append(t.clone().unsqueeze(0))
                ks.append(k)
        drv.close()
        if mid is not None:
            mid.close()
    torch.cuda.synchronize()
    return torch.stack(feats), torch.stack(targets), np.array(ks), time.perf_counter() - t0


def plunge_cases(n: int, seed: int):
    """n plunge settings drawn from a seeded generator: amplitude in [0.3, 0.7]
    (chords), frequency in [0.3, 0.5], phase in [0.5, 2 pi - 0.5] (clear of the
    evaluation case's phase), Reynolds number in {300, 500, 1000}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ph = rng.uniform(0.5, 2.0 * math.pi - 0.5)
        out.append(dict(amp=float(rng.uniform(0.3, 0.7)), freq=float(rng.uniform(0.3, 0.5)),
                        phase=float(ph), re=float(rng.choice([300.0, 500.0, 1000.0]))))
    return out


def crops(feats, targets, batch: int, size_y: int, size_x: int, rng):
    """A batch of random crops, offsets multiples of 8 (the network's pooling
    grid stays aligned with the full image's)."""
    import torch
    n, _, ny, nx = feats.shape
    idx = rng.integers(0, n, size=batch)
    ys = rng.integers(0, (ny - size_y) // 8 + 1, size=batch) * 8
    xs = rng.integers(0, (nx - size_x) // 8 + 1, size=batch) * 8
    x = torch.stack([feats[i, :, y:y + size_y, xx:xx + size_x] for i, y, xx in zip(idx, ys, xs)]).contiguous()
    t = torch.stack([targets[i, :, y:y + size_y, xx:xx + size_x] for i, y, xx in zip(idx, ys, xs)]).contiguous()
    return x, t


def train(net: U.UNet, feats, targets, iters: int, lr: float = 1e-3, lr_end: float = 1e-4, seed: int = 0,
          log_every: int = 0, relative: bool = False):
    """Adam on random crops of the snapshots (crop shape = the network's
    shape); cosine learning-rate decay from lr to lr_end.  relative: each
    image's squared error is divided by its target's mean square (a relative
    error per image, for targets whose sizes span decades; targets are
    expected near unit RMS, and weights are capped at 1e6).  Returns the loss
    history (every log_every iterations, and the last)."""
    rng = np.random.default_rng(seed)
    hist = []
    for k in range(iters):
        x, t = crops(feats, targets, net.max_batch, net.h, net.w, rng)
        w = 1.0 / t.pow(2).mean(dim=(1, 2, 3)).clamp_min(1e-6) if relative else None
        a = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * k / max(iters - 1, 1)))
        want = (log_every and k % log_every == 0) or k == iters - 1
        loss = net.train_step(x, t, a, want_loss=bool(want), weight=w)
        if want:
            hist.append((k, loss))
    return hist


def evaluate(wl: dict, params: np.ndarray, out_scale: float, warm_steps: int, method=ibm.RBSOR,
             warm_method=ibm.PCG, eval_steps: int = 1, modes=(ibm.INIT_ZERO, ibm.INIT_PREVIOUS, ibm.INIT_LEARNED),
             factor: int = 1, every: int = 0, options=None, guess: bool = True):
    """Advance the workload warm_steps steps (warm_method), then run
    eval_steps steps from that same state with each initial guess of `modes`
    (the learned mode also corrects every `every` SOR iterations when every >
    0, with the extra solver options given; guess=False keeps phi^n as its
    initial guess and uses the network for the corrections only); returns {mode: [step statistics]} (iterations, initial and final
    relative residuals, seconds of the whole step including the network)."""
    base = solver_for(wl, p_method=warm_method, p_init_prev=ibm.INIT_PREVIOUS)
    for _ in range(warm_steps):
        base.step(1)
    blob = base.get_state()
    base.close()
    out = {}
    net = None
    for mode in modes:
        s = solver_for(wl, p_method=method,
                       p_init_prev=ibm.INIT_PREVIOUS if mode == ibm.INIT_LEARNED and not guess else mode)
        s.set_state(blob)
        if mode == ibm.INIT_LEARNED:
            _net_options(s, factor)
            if every and s.set_option(ibm.OPT_NET_EVERY, every) != ibm.OK:
                raise ValueError(f"correction interval {every}")
            for opt, val in (options or {}).items():
                if s.set_option(opt, val) != ibm.OK:
                    raise ValueError(f"option {opt} = {val}")
            net = U.UNet(1, wl["ny"] // factor, wl["nx"] // factor, device=s.device, stream=s.stream)
            net.set_params(params)
            s.set_warm_start(net, out_scale)
        out[mode] = [s.step(1) for _ in range(eval_steps)]
        s.close()
    return out


MODE_NAMES = {ibm.INIT_ZERO: "zero", ibm.INIT_PREVIOUS: "previous", ibm.INIT_LEARNED: "learned"}


RECIPE_OPTIONS = {ibm.OPT_NET_MAPS: 5}  # residual and mask maps: no phi (see train_default)


def train_default(wl: dict, factor: int = 8, every: int = 4000, cases: int = 16, seed: int = 1,
                  iters: int = 3000, batch: int = 16, snap_iters=(200, 1000, 4000, 16000),
                  policy_iters=(4000, 8000, 16000, 32000, 64000), rounds: int = 4, options=None, log=None):
    """The training recipe of the learned correction, all on the GPU:
    a first training round on snapshots of plain SOR solves (3 steps of `cases` seeded plunge
    settings, snapshots at snap_iters); each later round on snapshots along
    the solve the current network corrects every `every` iterations (one step
    of `cases` other settings, snapshots at policy_iters), fine-tuning on all
    snapshots so far.  The start of a solve (k = 0, the raw residual of
    phi^n) is left out by default: its targets hold detail the coarse grid
    cannot carry, and with it the relative loss can stall at the zero
    prediction.  options: the network's solver options for every snapshot and
    for use (default RECIPE_OPTIONS: without the phi map, whose shape the
    network otherwise learns to copy on plain SOR iterates, a shortcut that
    fails on the iterates its own corrections produce).  Returns (parameters,
    out_scale, info)."""
    import torch
    say = log or (lambda *_: None)
    options = RECIPE_OPTIONS if options is None else options
    info = {"options": {int(k): int(v) for k, v in options.items()}}
    ny, nx = wl["ny"] // factor, wl["nx"] // factor
    f, t, ks, sec = collect(wl, plunge_cases(cases, seed), steps=3, factor=factor, snap_iters=snap_iters,
                            options=options)
    rms = t.pow(2).mean(dim=(1, 2, 3)).sqrt().cpu().numpy()
    out_scale = float(np.median(rms))
    t /= out_scale
    net = U.UNet(batch, ny, nx)
    net.set_params(he_uniform(seed))
    rounds_info = []
    for r in range(rounds):
        if r > 0:
            policy = dict(params=net.get_params(), out_scale=out_scale, every=every, guess=False,
                          options=options)
            f2, t2, _, sec = collect(wl, plunge_cases(cases, seed + r), steps=2, keep_from=2, factor=factor,
                                     snap_iters=policy_iters, policy=policy, options=options)
            t2 /= out_scale
            keep = t2.pow(2).mean(dim=(1, 2, 3)).sqrt() > 1e-3  # a solve done before its snapshot: no target
            f, t = torch.cat([f, f2[keep]]), torch.cat([t, t2[keep]])
            del f2, t2
        t0 = time.perf_counter()
        hist = train(net, f, t, iters, lr=1e-3 if r == 0 else 3e-4, lr_end=1e-5, log_every=max(iters // 3, 1),
                     relative=True, seed=seed + r)
        torch.cuda.synchronize()
        rounds_info.append({"snapshots": int(f.shape[0]), "collect_s": round(sec, 2),
                            "train_s": round(time.perf_counter() - t0, 2),
                            "loss": [(k, round(l, 5)) for k, l in hist]})
        say(f"round {r + 1}: {rounds_info[-1]}")
    info["rounds"] = rounds_info
    params = net.get_params()
    net.close()
    return params, out_scale, info


def he_uniform(seed: int) -> np.ndarray:
    """Initial parameters: He-uniform weights (bound sqrt(6 / fan_in)) and
    zero biases from a seeded generator, in the parameter-vector layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, _ in U.LAYERS:
        bound = math.sqrt(6.0 / (ci * 9))
        parts.append(rng.uniform(-bound, bound, size=co * ci * 9).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    return np.concatenate(parts)


def main(argv=None):
    """Train the learned correction for the plunging 1024x768 workload on the
    GPU and time the solve it guides against plain SOR from the previous
    step's phi; prints one JSON line."""
    import argparse
    import json

    from . import workloads

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--cases", type=int, default=16, help="plunge settings per training round")
    ap.add_argument("--iters", type=int, default=3000, help="Adam iterations per round")
    ap.add_argument("--rounds", type=int, default=4)
    ap.add_argument("--every", type=int, default=4000, help="SOR iterations between corrections")
    ap.add_argument("--factor", type=int, default=8, help="coarsening factor of the network's grid")
    ap.add_argument("--warm-steps", type=int, default=1, help="steps before the timed one")
    ap.add_argument("--baseline", type=int, default=1, help="1: also time plain SOR from the previous phi")
    a = ap.parse_args(argv)
    wl = workloads.plunging_1024x768()
    t0 = time.perf_counter()
    params, scale, info = train_default(wl, factor=a.factor, every=a.every, cases=a.cases, iters=a.iters,
                                        rounds=a.rounds)
    info["total_s"] = round(time.perf_counter() - t0, 2)
    modes = (ibm.INIT_PREVIOUS, ibm.INIT_LEARNED) if a.baseline else (ibm.INIT_LEARNED,)
    res = evaluate(wl, params, scale, warm_steps=a.warm_steps, method=ibm.RBSOR, modes=modes, factor=a.factor,
                   every=a.every, guess=False, options=RECIPE_OPTIONS)
    out = {"workload": wl["name"], "training": info,
           "steps": {("previous_guess" if m == ibm.INIT_PREVIOUS else "learned_correction"):
                     {k: v[0][k] for k in ("p_iters", "p_rel", "seconds", "n_net", "net_step")}
                     for m, v in res.items()}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python
"""Benchmark of the plain FP64 hot path on one MI355X.

Workload: plunging ellipse (chord 1, thickness 0.12, y = 0.5 sin(2 pi 0.4 t)),
Re 500, dt 5e-4, on the 1024x768 grid that is uniform (0.01c) around the body's
path and stretched geometrically outward on a 16c x 12c channel; u = 1, v = 0,
p = 0 at t = 0.  A step is one whole time step on the GPU: classification,
momentum predictor, forcing, implicit viscous solves, the pressure Poisson
solve to a relative residual of 1e-8, projection and forces.

Reported: Poisson cell-updates/s over the timed steps (nx*ny*iterations /
wall time; `value`), seconds per time step, the dominant kernel against the
HBM roofline (HIP events on the solver stream), a Jacobi-PCG leg, the
mixed-precision SOR leg, the learned warm start and correction (network
trained on the GPU in the run, then the same steps timed with it), and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s per time step + Poisson cell-updates/s at 1024x768; learned/FP32 vs plain FP64"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 compute units x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6
# algorithmic FLOPs of one red-black SOR cell update: the four neighbour
# products and their sum (7), minus V b (1), times 1/d (1), the relaxation
# (1 - omega) x + omega g (3)
SOR_FLOP_PER_UPDATE = 12.0
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak of the MI355X
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2402_17337_amd", "csrc", f)
                  for f in ("ibm_kernels.hpp", "ibm_device.hpp")]
# the library's default interior tile of the blocked sweep (10 iterations per launch)
DEFAULT_TILE = (76, 44)


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(kernel: str, workload_tag: str):
    """key = value lines of the committed rocprofv3 counter summary of a
    kernel (HBM bytes per launch, VALU busy fraction, ...), if it was taken
    with the current kernel sources; else None."""
    path = os.path.join(PROFILES, f"{kernel}_{workload_tag}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return vals


def _counter(vals, key):
    try:
        return float(vals[key]) if vals is not None else None
    except (KeyError, ValueError):
        return None


def _round_phases(ph):
    return None if ph is None else {k: round(v, 4) for k, v in ph.items()}


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def build_if_missing():
    from paper_2402_17337_amd import ibm
    from oracle import oracle as O
    if not os.path.exists(ibm.LIB_PATH) or not os.path.exists(O._LIB):
        import __graft_entry__
        __graft_entry__.build()


def gpu_leg(case, method, steps, warmup, profile_every, max_iters=0, p_init=None, net=None, keep_fields=False,
            check=None, repeats=1):
    """Time `steps` steps after `warmup` untimed ones.  p_init overrides the
    initial guess; net = (params, out_scale, factor, every, options) attaches
    a trained warm-start network; check overrides the stop-test interval.
    repeats > 1: the timed steps run that many times from the state after the
    warm-up (restored from a checkpoint; the same iterates each time) and the
    median run is reported (`wall`), with every run's time in `walls`."""
    import torch
    from paper_2402_17337_amd import ibm

    prm = dict(case["params"], p_method=method)
    if check is not None:
        prm["p_check"] = check
    if max_iters > 0:
        prm["p_max_iter"] = max_iters
    if p_init is not None:
        prm["p_init_prev"] = p_init
    g = ibm.Solver(case["nx"], case["ny"], case["xf"], case["yf"], case["u0"], case["v0"], case["p0"],
                   device="cuda:0", **prm)
    if net is not None:
        from paper_2402_17337_amd import unet as U
        params, out_scale, factor, every, opts = net
        for opt, val in [(ibm.OPT_NET_FACTOR, factor), (ibm.OPT_NET_EVERY, every)] + list(opts.items()):
            if g.set_option(opt, val) != ibm.OK:
                raise RuntimeError(f"solver option {opt} = {val} rejected")
        unet = U.UNet(1, case["ny"] // factor, case["nx"] // factor, stream=g.stream)
        unet.set_params(params)
        g.set_warm_start(unet, out_scale)
    for _ in range(warmup):
        st = g.step(1)
        if st["rc"] < 0:
            raise RuntimeError(f"warmup step failed: {st}")
    blob = g.get_state() if repeats > 1 else None
    runs = []
    for rep in range(repeats):
        if rep > 0:
            g.set_state(blob)
        g.profile(profile_every)
        iters, stats = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = g.step(1)
            if st["rc"] < 0:
                raise RuntimeError(f"timed step failed: {st}")
            iters.append(st["p_iters"])
            stats.append(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        log(f"{case['nx']}x{case['ny']} method {method} p_init {prm.get('p_init_prev')} "
            f"check {prm.get('p_check', 10)} net {'yes' if net is not None else 'no'} run {rep + 1}/{repeats}: "
            f"{steps} steps in {wall:.2f} s, iterations {iters}")
        phases, nph = g.profile_phases() if profile_every > 0 else ({}, 0)
        runs.append(dict(wall=wall, iters=iters, stats=stats, prof={k: g.profile_query(k) for k in ibm.KERNEL_NAMES},
                         phases={k: v / nph for k, v in phases.items()} if nph else None))
    med = sorted(runs, key=lambda r: r["wall"])[len(runs) // 2]
    fields = g.fields() if keep_fields else None
    g.close()
    cells = case["nx"] * case["ny"]
    wall = med["wall"]
    return dict(wall=wall, walls=[r["wall"] for r in runs], iters=med["iters"], stats=med["stats"],
                prof=med["prof"], phases_ms=med["phases"], fields=fields,
                cell_updates_per_s=cells * sum(med["iters"]) / wall if wall > 0 else 0.0)


def network_roofline(params, case, factor, reps=20):
    """The network's matrix-core rate: forward passes at the solve's coarse
    size and at the full grid, and a training step at the training shape,
    timed with events on the stream the kernels run on, against the dense
    BF16 peak.  FLOPs count 2 per multiply-add of the convolutions (the
    backward pass: twice the forward)."""
    import torch
    from paper_2402_17337_amd import unet as U
    out = {"bound": "mfma", "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s"}
    shapes = (("forward_coarse", 1, case["ny"] // factor, case["nx"] // factor, False),
              ("forward_full_grid", 1, case["ny"], case["nx"], False),
              ("train_step", 16, case["ny"] // factor, case["nx"] // factor, True))
    for name, b, h, w, train in shapes:
        net = U.UNet(b, h, w)
        net.set_params(params)
        x = torch.randn(b, 3, h, w, device="cuda:0")
        t = torch.randn(b, 1, h, w, device="cuda:0")
        y = torch.empty(b, 1, h, w, device="cuda:0")
        for _ in range(3):
            net.train_step(x, t, 0.0, want_loss=False) if train else net.forward(x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
        for _ in range(reps):
            net.train_step(x, t, 0.0, want_loss=False) if train else net.forward(x, y)
        e1.record(net.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        flops = U.forward_flops(b, h, w) * (3.0 if train else 1.0)
        tf = flops / (ms * 1e-3) / 1e12
        out[name] = {"shape": f"{b}x3x{h}x{w}", "ms": round(ms, 4), "gflop": round(flops / 1e9, 3),
                     "achieved": round(tf, 2), "frac": round(tf / BF16_PEAK_TFLOPS, 5)}
        net.close()
    return out


def c3_learned_leg(params, scale, steps, mp_check=10):
    """Full 2048x1536 steps to the 1e-8 stop test: SOR with the learned
    correction (the network trained on the 1024x768 workload, on the grid
    coarsened 16x: again 128x96), with FP64 sweeps (stop test every 10
    iterations, and every mp_check) and with FP32 sweeps + FP64 refinement
    every mp_check iterations, from one common state (one PCG step); errors
    of the mixed form in u, v, p and the force coefficients against the FP64
    form with the 10-iteration test."""
    import numpy as np
    import torch
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import unet as U
    from paper_2402_17337_amd import workloads as W

    wl = W.plunging_2048x1536()
    base = ibm.Solver(wl["nx"], wl["ny"], wl["xf"], wl["yf"], wl["u0"], wl["v0"], wl["p0"], device="cuda:0",
                      **dict(wl["params"], p_method=ibm.PCG))
    base.step(1)
    blob = base.get_state()
    base.close()
    res = {}
    forms = [("f64", ibm.RBSOR, 10), ("mixed", ibm.RBSOR_MP, mp_check)]
    if mp_check != 10:
        forms.insert(1, ("f64_same_interval", ibm.RBSOR, mp_check))
    for name, method, check in forms:
        s = ibm.Solver(wl["nx"], wl["ny"], wl["xf"], wl["yf"], device="cuda:0",
                       **dict(wl["params"], p_method=method, p_check=check))
        s.set_state(blob)
        for opt, val in ((ibm.OPT_NET_FACTOR, 16), (ibm.OPT_NET_EVERY, 4000), (ibm.OPT_NET_MAPS, 5)):
            if s.set_option(opt, val) != ibm.OK:
                raise RuntimeError(f"option {opt} = {val} rejected")
        net = U.UNet(1, wl["ny"] // 16, wl["nx"] // 16, stream=s.stream)
        net.set_params(params)
        s.set_warm_start(net, scale)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [s.step(1) for _ in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        log(f"2048x1536 learned {name}: {steps} steps in {wall:.2f} s, iterations {[x['p_iters'] for x in sts]}")
        res[name] = dict(s_per_step=round(wall / steps, 4), check_interval=check,
                         poisson_iters=[x["p_iters"] for x in sts],
                         final_rel_residual=[x["p_rel"] for x in sts], fields=s.fields()[:3], forces=s.forces())
        s.close()
    f, m = res["f64"], res["mixed"]
    err = {k: float(np.linalg.norm(a - b) / np.linalg.norm(b)) for k, a, b in zip("uvp", m["fields"], f["fields"])}
    err["cd"] = abs(m["forces"][0] - f["forces"][0]) / abs(f["forces"][0])
    err["cl"] = abs(m["forces"][1] - f["forces"][1]) / abs(f["forces"][1])
    for r in res.values():
        del r["fields"], r["forces"]
    return {"workload": "plunging ellipse 2048x1536, Re 1000, h 0.6, f 0.5; steps 2.. after one common PCG step, "
                        "pressure solves to 1e-8 with the learned correction (network trained on 1024x768, "
                        "coarse grid 128x96)",
            **res,
            "mixed_speedup": round(res["f64"]["s_per_step"] / res["mixed"]["s_per_step"], 3),
            "mixed_speedup_same_interval": round(res["f64_same_interval"]["s_per_step"] / res["mixed"]["s_per_step"], 3)
            if "f64_same_interval" in res else None,
            "mixed_rel_error_vs_f64": err}


def learned_legs(case, args, sor_leg):
    """Train the warm-start network on the GPU (the recipe of
    paper_2402_17337_amd.warmstart.train_default), then time the same steps as
    the headline leg with the learned correction every args.learned_every SOR
    iterations from the previous step's phi (FP64 and FP32 sweeps), and with
    args.learned_guess_legs also the zero guess and the learned guess alone;
    PCG with the learned guess beside PCG's own legs."""
    import numpy as np
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import warmstart as WS

    F, every = args.learned_factor, args.learned_every
    t0 = time.perf_counter()
    params, scale, info = WS.train_default(case, factor=F, every=every, iters=args.learned_train_iters, log=log)
    opts = WS.RECIPE_OPTIONS
    info["total_s"] = round(time.perf_counter() - t0, 2)
    base_s = sor_leg["wall"] / args.steps
    out = {"network": f"4-level U-Net 16/32/64/128, BF16 matrix cores, on the grid coarsened {F}x "
                      f"({case['nx'] // F}x{case['ny'] // F})",
           "training": info, "out_scale": scale,
           "reference": {"initial_guess": "previous phi", "s_per_time_step": round(base_s, 6),
                         "poisson_iters_per_step": sor_leg["iters"]}}
    legs = [("zero_guess", ibm.INIT_ZERO, None, ibm.RBSOR, None),
            ("learned_guess", ibm.INIT_LEARNED, (params, scale, F, 0, opts), ibm.RBSOR, None)] \
        if args.learned_guess_legs else []
    legs.append(("learned_correction", ibm.INIT_PREVIOUS, (params, scale, F, every, opts), ibm.RBSOR, None))
    if every % args.mp_check == 0:
        # the learned correction with FP32 sweeps and FP64 refinement (the
        # refinement interval divides the correction interval)
        legs.append(("learned_correction_mixed", ibm.INIT_PREVIOUS, (params, scale, F, every, opts), ibm.RBSOR_MP,
                     args.mp_check))
    ref = sor_leg["fields"]
    for name, p_init, net, meth, check in legs:
        leg = gpu_leg(case, meth, args.steps, args.warmup, 0, p_init=p_init, net=net,
                      keep_fields=ref is not None, check=check)
        s_step = leg["wall"] / args.steps
        d = {"s_per_time_step": round(s_step, 6), "poisson_iters_per_step": leg["iters"],
             "final_rel_residual": [st["p_rel"] for st in leg["stats"]],
             "speedup_vs_previous_guess": round(base_s / s_step, 3) if s_step > 0 else None}
        if net is not None:
            d["network_steps_per_time_step"] = [st["n_net"] for st in leg["stats"]]
            d["mean_step_length"] = [round(st["net_step"], 4) for st in leg["stats"]]
            if net[3]:
                d["correction_every"] = net[3]
        if check is not None:
            d["check_interval"] = check
        if ref is not None and leg["fields"] is not None:
            d["rel_l2_vs_previous_guess_run"] = {
                k: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
                for k, a, b in zip(("u", "v", "p"), leg["fields"][:3], ref[:3])}
        out[name] = d
    out["network_roofline"] = network_roofline(params, case, F)
    if args.c3_learned_steps > 0:
        out["c3_full_steps"] = c3_learned_leg(params, scale, args.c3_learned_steps,
                                              args.mp_check if 4000 % args.mp_check == 0 else 10)
    if args.pcg_steps > 0:
        leg = gpu_leg(case, ibm.PCG, args.pcg_steps, args.warmup, 0, p_init=ibm.INIT_LEARNED,
                      net=(params, scale, F, 0, opts))
        out["pcg_learned_guess"] = {"s_per_time_step": round(leg["wall"] / args.pcg_steps, 6),
                                    "poisson_iters_per_step": leg["iters"]}
    return out


def batch_leg(args):
    """The many-case workload (64 plunging cases, grids 256x192 to 1024x768):
    one time step of every case with the pressure solves batched (one blocked
    launch per 10 iterations over all cases' tiles), against the same cases
    stepped one after another.  Each pressure solve is capped at
    args.c4_iters iterations (the cases' full solves take up to 1.4 M
    iterations).  Tile shapes: the one-by-one run uses the shape tuned for each
    grid size alone (small grids want small tiles to fill the GPU); the batch
    is timed with those and with the library's default shape (DEFAULT_TILE)
    for every case, since a batch has parallelism to spare and small tiles
    cost halo work; the faster of the two is reported as the batched time.
    The default-shape batch is also timed replaying stretches of
    args.c4_graph check intervals from a HIP graph."""
    import torch
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W

    cases = W.batched_plunging(args.c4_cases, 0)
    cap = args.c4_iters

    def make(tiles, **over):
        out = []
        for c in cases:
            s = ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], device="cuda:0",
                           **dict(c["params"], p_max_iter=cap, **over))
            tx, ty = tiles.get((c["nx"], c["ny"]), DEFAULT_TILE)
            s.set_option(ibm.OPT_TB_TILE_X, tx)
            s.set_option(ibm.OPT_TB_TILE_Y, ty)
            out.append(s)
        return out

    tuned = {}
    if args.c4_autotune:
        for c in cases:
            key = (c["nx"], c["ny"])
            if key not in tuned:
                s = ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], device="cuda:0", **c["params"])
                tuned[key] = s.autotune_tiles()[0]
                s.close()

    def timed_batch(solvers, graph=0):
        batch = ibm.Batch(solvers)
        if graph:
            batch.set_graph(graph)
        batch.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = batch.step(1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        batch.close()
        return dt, st

    t_uniform, st_b = timed_batch(make({}))
    log(f"batched step of {len(cases)} cases, default tiles: {t_uniform:.3f} s")
    # one tile shape for the whole batch, tuned on the batch itself
    probe = ibm.Batch(make({}))
    probe.step(1)
    batch_shape, batch_times = probe.autotune_tiles()
    probe.close()
    log(f"batch-wide tile autotune: {batch_shape} from {batch_times}")
    t_bt, st_bt = timed_batch(make({(c["nx"], c["ny"]): batch_shape for c in cases}))
    log(f"batched step of {len(cases)} cases, batch-tuned tiles {batch_shape}: {t_bt:.3f} s")
    t_graph = None
    if args.c4_graph:
        t_graph, st_g = timed_batch(make({}), args.c4_graph)
        log(f"batched step of {len(cases)} cases, default tiles, graph of {args.c4_graph} intervals: {t_graph:.3f} s")
    t_tuned = None
    if tuned:
        t_tuned, st_t = timed_batch(make(tuned))
        log(f"batched step of {len(cases)} cases, per-size tiles: {t_tuned:.3f} s")
    solo = make(tuned)
    for s in solo:
        s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_s = [s.step(1) for s in solo]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    log(f"the same step case by case: {t_s:.3f} s")
    # same tiles: bitwise the same solves; other tiles: the same iterates, with
    # the stop-test sums taken over other tile partials (last bits of p_rel)
    same = None if t_tuned is None else all(a["p_iters"] == b["p_iters"] and a["p_rel"] == b["p_rel"]
                                             for a, b in zip(st_t, st_s))
    same_iters = all(a["p_iters"] == b["p_iters"] and abs(a["p_rel"] - b["p_rel"]) <= 1e-12 * b["p_rel"]
                     for a, b in zip(st_b, st_s))
    mixed = None
    if args.c4_mixed:
        # FP32 sweeps with FP64 refinement every args.mp_check iterations:
        # batched (default tiles) and case by case (per-size tiles; the tile
        # shape does not change the float iterates, nor the refinement's sums)
        over = dict(p_method=ibm.RBSOR_MP, p_check=args.mp_check)
        bt = {(c["nx"], c["ny"]): batch_shape for c in cases}
        t_mb, st_mb = timed_batch(make(bt, **over))
        log(f"mixed-precision batched step of {len(cases)} cases: {t_mb:.3f} s")
        t_mbg, st_mbg = (timed_batch(make(bt, **over), args.c4_graph) if args.c4_graph else (None, None))
        if t_mbg is not None:
            log(f"mixed-precision batched step, graph of {args.c4_graph} intervals: {t_mbg:.3f} s")
        solo_mp = make(tuned, **over)
        for s in solo_mp:
            s.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_ms = [s.step(1) for s in solo_mp]
        torch.cuda.synchronize()
        t_ms = time.perf_counter() - t0
        for s in solo_mp:
            s.close()
        log(f"the same mixed-precision step case by case: {t_ms:.3f} s")
        mixed = {"check_interval": args.mp_check, "batched_s": round(t_mb, 4), "sequential_s": round(t_ms, 4),
                 "speedup": round(t_ms / t_mb, 3), "tile": f"{batch_shape[0]}x{batch_shape[1]}",
                 "batched_s_graph": round(t_mbg, 4) if t_mbg is not None else None,
                 "graph_bitwise_equal_to_launched": None if t_mbg is None else all(
                     a["p_iters"] == b["p_iters"] and a["p_rel"] == b["p_rel"] and a["cd"] == b["cd"]
                     for a, b in zip(st_mbg, st_mb)),
                 "bitwise_equal_to_sequential": all(a["p_iters"] == b["p_iters"] and a["p_rel"] == b["p_rel"]
                                                    and a["cd"] == b["cd"] for a, b in zip(st_mb, st_ms))}
    t_b = min(t for t in (t_uniform, t_tuned, t_graph, t_bt) if t is not None)
    if mixed is not None:
        mixed["speedup_vs_f64_batch"] = round(t_b / mixed["batched_s"], 3)
    graph_same = None if t_graph is None else all(
        a["p_iters"] == b["p_iters"] and a["p_rel"] == b["p_rel"] and a["cd"] == b["cd"] for a, b in zip(st_g, st_b))
    cells = [c["nx"] * c["ny"] for c in cases]
    upd = sum(n * st["p_iters"] for n, st in zip(cells, st_b))
    return {"workload": f"{len(cases)} plunging cases, grids 256x192..1024x768 (seed 0), one time step, "
                        f"pressure solves capped at {cap} iterations",
            "cells": sum(cells), "batched_s": round(t_b, 4), "sequential_s": round(t_s, 4),
            "speedup": round(t_s / t_b, 3) if t_b > 0 else None,
            "batched_s_default_tiles": round(t_uniform, 4),
            "batched_s_per_size_tiles": round(t_tuned, 4) if t_tuned is not None else None,
            "batched_s_default_tiles_graph": round(t_graph, 4) if t_graph is not None else None,
            "batched_s_batch_tuned": round(t_bt, 4), "batch_tuned_tile": f"{batch_shape[0]}x{batch_shape[1]}",
            "batch_autotune_s": {f"{k[0]}x{k[1]}": round(v, 4) for k, v in batch_times.items()},
            "graph_intervals": args.c4_graph or None,
            "graph_batch_bitwise_equal_to_launched": graph_same,
            "batched_cell_updates_per_s": round(upd / t_b, 1), "sequential_cell_updates_per_s": round(upd / t_s, 1),
            "poisson_iters": sorted(set(st["p_iters"] for st in st_b)),
            "per_size_batch_bitwise_equal_to_sequential": same,
            "uniform_batch_same_iterations_as_sequential": same_iters,
            "per_size_tiles": {f"{k[0]}x{k[1]}": f"{v[0]}x{v[1]}" for k, v in tuned.items()},
            "mixed_precision": mixed,
            "uncapped": uncapped_batch(args, cases, tuned, batch_shape) if args.c4_uncapped else None}


def uncapped_batch(args, cases, tuned, batch_shape):
    """The many-case workload to the 1e-8 stop test, no iteration cap: every
    case advanced two steps with Jacobi-PCG (per case), then one step with
    FP32 sweeps and FP64 refinement every args.mp_check iterations, batched
    (one tile shape tuned for the batch, the solve replayed from a HIP graph of
    args.c4_graph intervals) and case by case (tiles tuned per grid size),
    from the same states."""
    import torch
    from paper_2402_17337_amd import ibm

    blobs = []
    for c in cases:
        s = ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], device="cuda:0",
                       **dict(c["params"], p_method=ibm.PCG))
        s.step(2)
        blobs.append(s.get_state())
        s.close()
    over = dict(p_method=ibm.RBSOR_MP, p_check=args.mp_check, p_max_iter=20_000_000)

    def make(shape_of):
        out = []
        for c, blob in zip(cases, blobs):
            s = ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], device="cuda:0", **dict(c["params"], **over))
            tx, ty = shape_of(c)
            s.set_option(ibm.OPT_TB_TILE_X, tx)
            s.set_option(ibm.OPT_TB_TILE_Y, ty)
            s.set_state(blob)
            out.append(s)
        return out

    batch = ibm.Batch(make(lambda c: batch_shape))
    if args.c4_graph:
        batch.set_graph(args.c4_graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_b = batch.step(1)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    batch.close()
    log(f"uncapped mixed-precision batched step of {len(cases)} cases: {t_b:.2f} s, "
        f"iterations {min(s['p_iters'] for s in st_b)}..{max(s['p_iters'] for s in st_b)}")
    solo = make(lambda c: tuned.get((c["nx"], c["ny"]), DEFAULT_TILE))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_s = [s.step(1) for s in solo]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    for s in solo:
        s.close()
    log(f"the same uncapped step case by case: {t_s:.2f} s")
    ok = all(b["rc"] >= 0 and b["p_rel"] <= 1e-8 for b in st_b)
    cells = [c["nx"] * c["ny"] for c in cases]
    upd = sum(n * st["p_iters"] for n, st in zip(cells, st_b))
    return {"workload": f"{len(cases)} plunging cases, step 3 (after two PCG steps per case), pressure solves to "
                        f"1e-8 with no cap; FP32 sweeps + FP64 refinement every {args.mp_check} iterations",
            "poisson_iteration_cap": None, "batched_s": round(t_b, 3), "sequential_s": round(t_s, 3),
            "speedup": round(t_s / t_b, 3), "graph_intervals": args.c4_graph or None,
            "tile": f"{batch_shape[0]}x{batch_shape[1]}",
            "poisson_iters_min_max": [min(s["p_iters"] for s in st_b), max(s["p_iters"] for s in st_b)],
            "all_converged_to_1e-8": ok,
            "bitwise_equal_to_sequential": all(a["p_iters"] == b["p_iters"] and a["p_rel"] == b["p_rel"]
                                               and a["cd"] == b["cd"] for a, b in zip(st_b, st_s)),
            "batched_cell_updates_per_s": round(upd / t_b, 1)}


def stress_leg(nx=8192, ny=6144, iters=60):
    """The Poisson sweep kernels on a grid whose phi and V b (805 MB) exceed
    the last-level cache, so that their traffic is HBM traffic: 60 fixed
    iterations of each SOR kernel on a uniform grid, kernel durations from HIP
    events."""
    import torch
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W

    g = ibm.Solver(nx, ny, W.uniform_faces(nx, 16.0), W.uniform_faces(ny, 12.0), device="cuda:0", body=0)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(0)
    b = torch.rand((ny, nx), dtype=torch.float64, device="cuda:0", generator=gen) - 0.5
    out = {"grid": f"{nx}x{ny}", "iterations": iters}
    for kern, kid in ((ibm.SOR_TEMPORAL, ibm.KERNEL_SOR_TB), (ibm.SOR_PER_COLOUR, ibm.KERNEL_SOR_SWEEP)):
        if g.set_option(ibm.OPT_SOR_KERNEL, kern) != ibm.OK:
            raise RuntimeError("kernel option rejected")
        x = torch.zeros_like(b)
        g.profile(1)
        g.poisson_solve(b, x, method=ibm.RBSOR, fixed_iters=iters, check_every=10)
        q = g.profile_query(kid)
        gbs = q["bytes_per_launch"] / (q["avg_ms"] * 1e-3) / 1e9 if q["avg_ms"] > 0 else 0.0
        out[ibm.KERNEL_NAMES[kid]] = {"avg_us": round(q["avg_ms"] * 1e3, 2), "achieved_GBps": round(gbs, 1),
                                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
    g.close()
    return out


def c1_leg(cpu=True):
    """The stationary 128x96 workload, all 100 steps (RB-SOR to 1e-8 every 10
    iterations): GPU seconds for the whole run, and the oracle's (one thread:
    a grid this small runs its loops serially) for the same run."""
    import torch
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W

    c = W.stationary_128x96()
    g = ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], device="cuda:0", **c["params"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [g.step(1) for _ in range(c["steps"])]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    iters = sum(s["p_iters"] for s in sts)
    out = {"workload": c["name"] + ", all 100 steps", "gpu_s": round(wall, 4), "poisson_iters_total": iters,
           "gpu_s_per_step": round(wall / c["steps"], 6)}
    log(f"128x96, 100 steps on the GPU: {wall:.2f} s ({iters} Poisson iterations)")
    if cpu:
        from oracle import oracle as O
        o = O.Oracle(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], **c["params"])
        t0 = time.perf_counter()
        rc, so = o.step(c["steps"])
        cw = time.perf_counter() - t0
        out.update(oracle_s=round(cw, 3), oracle_threads=1, speedup=round(cw / wall, 2),
                   oracle_poisson_iters_total=sum(x["p_iters"] for x in so))
        log(f"128x96, 100 steps on the oracle: {cw:.2f} s")
    return out


def pcg_long_leg(case, steps, method, late_sor_steps=0, capture=()):
    """Jacobi-PCG over a long stretch of the 1024x768 workload from t = 0
    (the workload's full length is 2000 steps): seconds per step over the
    run and over its last tenth; then, from the state it reached, a window of
    late_sor_steps red-black SOR steps (the late-window SOR timing).  For
    each step number in `capture`, the pressure system of that step (V b,
    the previous phi, the step's iterations) is kept in `captured` (host
    copies, taken between steps; not part of the returned line)."""
    import torch
    from paper_2402_17337_amd import ibm

    g = ibm.Solver(case["nx"], case["ny"], case["xf"], case["yf"], case["u0"], case["v0"], case["p0"],
                   device="cuda:0", **dict(case["params"], p_method=method))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks, iters, captured = [], [], []
    for k in range(steps):
        phi_prev = g.fields()[3] if k + 1 in capture else None
        st = g.step(1)
        if st["rc"] < 0:
            raise RuntimeError(f"PCG step {k} failed: {st}")
        iters.append(st["p_iters"])
        if phi_prev is not None:
            captured.append({"step": k + 1, "vb": g.poisson_rhs(), "phi_prev": phi_prev,
                             "step_iters": st["p_iters"]})
        if (k + 1) % max(1, steps // 10) == 0:
            torch.cuda.synchronize()
            marks.append(time.perf_counter() - t0)
            log(f"1024x768 PCG from t = 0: step {k + 1} of {steps}, {marks[-1]:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cd, cl = g.forces()
    blob = g.get_state() if late_sor_steps > 0 else None
    g.close()
    log(f"1024x768 PCG, {steps} steps from t = 0: {wall:.2f} s")
    last = (marks[-1] - marks[-2]) / max(1, steps // 10) if len(marks) >= 2 else wall / steps
    out = {"steps": steps, "solver": "one-reduction Jacobi-PCG" if method == ibm.CG1 else "Jacobi-PCG",
           "s_per_time_step": round(wall / steps, 6),
           "s_per_time_step_last_tenth": round(last, 6), "poisson_iters_mean": round(sum(iters) / steps, 1),
           "poisson_iters_last": iters[-1], "cd_last": cd, "cl_last": cl}
    if late_sor_steps > 0:
        s = ibm.Solver(case["nx"], case["ny"], case["xf"], case["yf"], device="cuda:0",
                       **dict(case["params"], p_method=ibm.RBSOR))
        s.set_state(blob)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [s.step(1) for _ in range(late_sor_steps)]
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        s.close()
        if any(x["rc"] < 0 for x in sts):
            raise RuntimeError(f"late SOR step failed: {sts}")
        it = [x["p_iters"] for x in sts]
        log(f"1024x768 SOR, steps {steps + 1}..{steps + late_sor_steps}: {w:.2f} s, iterations {it}")
        out["sor_late_window"] = {
            "steps": f"{steps + 1}..{steps + late_sor_steps}", "initial_guess": "previous phi (from the PCG run)",
            "s_per_time_step": round(w / late_sor_steps, 6), "poisson_iters_per_step": it,
            "cell_updates_per_s": round(case["nx"] * case["ny"] * sum(it) / w, 1)}
    return out, captured


def poisson_bench_leg(case, fixed=10000, captured=()):
    """Stand-alone Poisson solves on the 1024x768 grid with a manufactured
    right-hand side: the Laplacian of p = cos(pi x / 2 Lx) cos(pi y / Ly),
    which meets the channel conditions (Neumann, p = 0 on the outlet face).
    Red-black SOR and the one-reduction CG for `fixed` iterations (rate), and
    each to 1e-8 from zero (iterations, seconds, error against p).  Then the
    pressure systems captured from time steps of the workload (V b, from the
    previous step's phi): the same rate and to-tolerance runs."""
    import numpy as np
    import torch
    from paper_2402_17337_amd import ibm

    xf, yf = np.asarray(case["xf"]), np.asarray(case["yf"])
    Lx, Ly = xf[-1] - xf[0], yf[-1] - yf[0]
    xc, yc = 0.5 * (xf[1:] + xf[:-1]) - xf[0], 0.5 * (yf[1:] + yf[:-1]) - yf[0]
    X, Y = np.meshgrid(xc, yc)
    pe = np.cos(np.pi * X / (2 * Lx)) * np.cos(np.pi * Y / Ly)
    b = -((np.pi / (2 * Lx)) ** 2 + (np.pi / Ly) ** 2) * pe
    g = ibm.Solver(case["nx"], case["ny"], case["xf"], case["yf"], device="cuda:0", body=0)
    rhs = torch.from_numpy(b).to("cuda:0")
    cells = case["nx"] * case["ny"]
    out = {"rhs": "Laplacian of cos(pi x / 2 Lx) cos(pi y / Ly) on the stretched grid", "fixed_iterations": fixed}
    for name, m in (("sor", ibm.RBSOR), ("cg1", ibm.CG1)):
        x = torch.zeros_like(rhs)
        g.poisson_solve(rhs, x, method=m, fixed_iters=100)  # warm-up
        x.zero_()
        st = g.poisson_solve(rhs, x, method=m, fixed_iters=fixed)
        x.zero_()
        st2 = g.poisson_solve(rhs, x, method=m, tol=1e-8, max_iter=20_000_000)
        err = float(np.max(np.abs(x.cpu().numpy() - pe)))
        out[name] = {"fixed_s": round(st["seconds"], 6), "cell_updates_per_s": round(cells * fixed / st["seconds"], 1),
                     "to_1e-8_iters": st2["iters"], "to_1e-8_s": round(st2["seconds"], 4), "rc": st2["rc"],
                     "max_error_vs_p": err}
        log(f"Poisson bench {name}: {fixed} iterations in {st['seconds'] * 1e3:.2f} ms; to 1e-8: "
            f"{st2['iters']} iterations in {st2['seconds']:.3f} s, max |x - p| {err:.2e}")
    area = np.diff(yf)[:, None] * np.diff(xf)[None, :]
    rows = []
    for cap in captured:
        b = torch.from_numpy(cap["vb"] / area).to("cuda:0")
        x0 = torch.from_numpy(cap["phi_prev"]).to("cuda:0")
        row = {"step": cap["step"], "step_iters_cg1": cap["step_iters"]}
        for name, m in (("sor", ibm.RBSOR), ("cg1", ibm.CG1)):
            x = x0.clone()
            st = g.poisson_solve(b, x, method=m, fixed_iters=fixed)
            x.copy_(x0)
            st2 = g.poisson_solve(b, x, method=m, tol=1e-8, max_iter=20_000_000)
            row[name] = {"fixed_s": round(st["seconds"], 6),
                         "cell_updates_per_s": round(cells * fixed / st["seconds"], 1),
                         "to_1e-8_iters": st2["iters"], "to_1e-8_s": round(st2["seconds"], 4), "rc": st2["rc"]}
        log(f"Poisson bench, step {cap['step']}'s system from the previous phi: SOR {row['sor']['to_1e-8_iters']} "
            f"iterations in {row['sor']['to_1e-8_s']:.3f} s, CG1 {row['cg1']['to_1e-8_iters']} in "
            f"{row['cg1']['to_1e-8_s']:.4f} s (the step took {cap['step_iters']} CG1 iterations)")
        rows.append(row)
    if rows:
        out["captured_systems"] = {"rhs": "V b of time steps of the 1024x768 workload (one-reduction CG run from "
                                          "t = 0), solved from the previous step's phi", "rows": rows}
    g.close()
    return out


def scaling_leg(steps=3, warmup=2, sor_iters=2000):
    """Input scaling at the paper's three mesh sizes (0.6, 1.2 and 1.8 M
    cells): the plunging construction at 896x672, 1280x960 and 1536x1152,
    seconds per step with Jacobi-PCG to 1e-8 after `warmup` steps, and the
    red-black SOR rate (fixed iteration counts) on each grid."""
    import torch
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W

    rows = []
    for nx, ny in ((896, 672), (1280, 960), (1536, 1152)):
        c = W.plunging_scaled(nx, ny)
        g = ibm.Solver(nx, ny, c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], device="cuda:0",
                       **dict(c["params"], p_method=ibm.PCG))
        for _ in range(warmup):
            g.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [g.step(1) for _ in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gen = torch.Generator(device="cpu").manual_seed(0)
        rhs = (torch.rand(ny, nx, generator=gen, dtype=torch.float64) - 0.5).to("cuda:0")
        x = torch.zeros_like(rhs)
        g.poisson_solve(rhs, x, fixed_iters=200)
        x.zero_()
        sor = g.poisson_solve(rhs, x, fixed_iters=sor_iters)
        g.close()
        cells = nx * ny
        it = sum(s["p_iters"] for s in sts)
        rows.append({"grid": f"{nx}x{ny}", "cells": cells, "pcg_s_per_time_step": round(wall / steps, 6),
                     "pcg_iters_per_step": [s["p_iters"] for s in sts],
                     "pcg_cell_updates_per_s": round(cells * it / wall, 1),
                     "sor_cell_updates_per_s": round(cells * sor_iters / sor["seconds"], 1)})
        log(f"scaling {nx}x{ny}: PCG {wall / steps:.4f} s per step, SOR {rows[-1]['sor_cell_updates_per_s']:.3e} "
            f"cell-updates/s")
    return {"workload": "plunging construction (core spacing 0.01 * 1024 / nx), Re 500, h 0.5, f 0.4; "
                        f"steps {warmup + 1}..{warmup + steps}", "rows": rows}


# The paper's own speedups (whole solver, 1000 steps of its plunging-ellipse
# case on 0.6/1.2/1.8 M cells): OpenACC on one V100 against its serial C++ on
# one Xeon Gold 6248 thread, and against OpenMP on 16 threads of that CPU.
PAPER_SPEEDUPS = {
    "hardware": "NVIDIA Tesla V100 32 GB (OpenACC) vs Intel Xeon Gold 6248 (20 cores, 2.6 GHz)",
    "vs_serial": {"0.6M": 53.8, "1.2M": 65.2, "1.8M": 108.6},
    "vs_openmp_16_threads": {"0.6M": 17.3, "1.2M": 21.6, "1.8M": 32.5},
    "claim": "O(10) over OpenMP, O(10^2) over serial",
}


def cpu_leg(case, target_seconds, gpu_iters_per_step, threads=0):
    """Oracle on a bounded sample: one time step of the same workload with the
    pressure solve capped at M red-black SOR iterations (tolerance unreachable),
    at two values of M; per-iteration and per-step costs from the difference.
    threads > 0 runs the oracle on that many OpenMP threads (else all)."""
    from oracle import oracle as O

    prm = dict(case["params"], p_tol=1e-300)
    if threads > 0:
        O.set_num_threads(threads)

    def one(m):
        o = O.Oracle(case["nx"], case["ny"], case["xf"], case["yf"], case["u0"], case["v0"], case["p0"],
                     **dict(prm, p_max_iter=m))
        t0 = time.perf_counter()
        o.step(1)
        return time.perf_counter() - t0

    m1 = 10
    t1 = one(m1)
    probe = one(m1 + 40)
    per_it = max((probe - t1) / 40.0, 1e-9)
    m2 = int(max(100, min(20000, (target_seconds - t1) / per_it)))
    t2 = one(m2)
    per_it = (t2 - t1) / (m2 - m1)
    overhead = max(t1 - m1 * per_it, 0.0)
    cells = case["nx"] * case["ny"]
    est_step = overhead + per_it * gpu_iters_per_step
    used = O.num_threads()
    if threads > 0:
        O.set_num_threads(os.cpu_count() or 1)
    return dict(value=cells / per_it, unit="cell-updates/s", cores=used, kind="oracle",
                sample=(f"one {case['nx']}x{case['ny']} time step of the same workload with the "
                        f"pressure solve capped at {m1} and at {m2} red-black SOR iterations; "
                        f"rate from the difference"),
                seconds=round(t1 + probe + t2, 2),
                s_per_time_step_est=est_step,
                step_overhead_s=overhead)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--solver", choices=("sor", "pcg"), default="sor",
                    help="pressure solver of the headline leg")
    ap.add_argument("--pcg-steps", type=int, default=4, help="timed steps of the PCG leg (0: skip)")
    ap.add_argument("--mp-steps", type=int, default=2,
                    help="timed steps of the mixed-precision SOR leg (float sweeps, double refinement; 0: skip)")
    ap.add_argument("--c3-iters", type=int, default=20000,
                    help="Poisson iterations per solve of the capped 2048x1536 comparison of double and "
                         "mixed-precision SOR (0: skip)")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="bracket every n-th launch of each timed kernel with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample (0: skip the CPU baseline)")
    ap.add_argument("--max-poisson-iters", type=int, default=0,
                    help="profiling aid: cap each pressure solve at this many iterations "
                         "(same kernels and launch shapes; the line is then marked capped)")
    ap.add_argument("--stress", type=int, default=1,
                    help="1: also time the SOR kernels on the HBM-resident 8192x6144 grid")
    ap.add_argument("--learned", type=int, default=1,
                    help="1: train the warm-start network on the GPU and time the learned guess and correction")
    ap.add_argument("--learned-guess-legs", type=int, default=1,
                    help="1: also time the zero guess and the learned guess alone (the warm start proper, "
                         "about 50 s)")
    ap.add_argument("--mp-check", type=int, default=100,
                    help="stop-test (= refinement) interval of the FP32-sweep legs; the FP64 legs test every 10")
    ap.add_argument("--c3-learned-steps", type=int, default=2,
                    help="full 2048x1536 steps with the learned correction, FP64 and mixed sweeps (0: skip)")
    ap.add_argument("--learned-every", type=int, default=4000,
                    help="SOR iterations between learned corrections")
    ap.add_argument("--learned-factor", type=int, default=8, help="coarsening factor of the network's grid")
    ap.add_argument("--learned-train-iters", type=int, default=3000, help="Adam iterations per training round")
    ap.add_argument("--c4-cases", type=int, default=64,
                    help="cases of the batched many-grid leg (0: skip)")
    ap.add_argument("--c4-iters", type=int, default=2000, help="Poisson iteration cap of the batched leg")
    ap.add_argument("--c4-autotune", type=int, default=1,
                    help="1: tune the tile shape per grid size (for the case-by-case run, and as a batch variant)")
    ap.add_argument("--c4-mixed", type=int, default=1,
                    help="1: also time the batched leg with FP32 sweeps and FP64 refinement (--mp-check)")
    ap.add_argument("--c4-graph", type=int, default=10,
                    help="check intervals per HIP-graph stretch of the batched variant replayed from a graph "
                         "(even; 0: skip that variant)")
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed runs of the headline, PCG and mixed-precision legs (the same steps from the same "
                         "checkpoint); the median is reported")
    ap.add_argument("--c1", type=int, default=1, help="1: time all 100 steps of the 128x96 workload (GPU and oracle)")
    ap.add_argument("--late-sor-steps", type=int, default=5,
                    help="SOR steps timed after the long PCG run, from its state (0: skip)")
    ap.add_argument("--poisson-bench", type=int, default=1,
                    help="1: stand-alone Poisson solves with a manufactured right-hand side, and with the "
                         "systems of steps 1, 10, 100 and the last of the long PCG run")
    ap.add_argument("--pcg-long-steps", type=int, default=400,
                    help="steps of the long Jacobi-PCG run of the 1024x768 workload from t = 0 (0: skip)")
    ap.add_argument("--scaling", type=int, default=1,
                    help="1: input-scaling rows at 0.6, 1.2 and 1.8 M cells (PCG steps, SOR rate)")
    ap.add_argument("--c4-uncapped", type=int, default=1,
                    help="1: also one uncapped batched step to 1e-8 (mixed precision, graph, batch-tuned tiles) "
                         "against the same step case by case")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run only a plain device-to-device copy of this many MiB, 20 times "
                         "(reference kernel for scaling the HBM byte counters)")
    args = ap.parse_args()

    if args.calibrate_copy > 0:
        import torch
        n = args.calibrate_copy * 2 ** 20 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 8, "bytes_written": n * 8, "launches": 20}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the solver is single-device "
                                   "(grid sharding is described but not implemented); use --gpus 1"}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be >= 1 and --warmup >= 0")

    build_if_missing()
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W

    case = W.plunging_1024x768()
    tag = "plunging1024x768"
    method = ibm.RBSOR if args.solver == "sor" else ibm.PCG
    learned = args.learned and args.solver == "sor" and not args.max_poisson_iters
    reps = max(1, args.repeats)
    main_leg = gpu_leg(case, method, args.steps, args.warmup, args.profile_every, args.max_poisson_iters,
                       keep_fields=learned, repeats=reps)
    pcg_leg = cg1_leg = None
    if args.solver == "sor" and args.pcg_steps > 0:
        pcg_leg = gpu_leg(case, ibm.PCG, args.pcg_steps, args.warmup, args.profile_every,
                          args.max_poisson_iters, repeats=reps)
        cg1_leg = gpu_leg(case, ibm.CG1, args.pcg_steps, args.warmup, args.profile_every,
                          args.max_poisson_iters, repeats=reps)

    mp_leg = None
    if args.solver == "sor" and args.mp_steps > 0:
        mp_leg = gpu_leg(case, ibm.RBSOR_MP, args.mp_steps, args.warmup, args.profile_every,
                         args.max_poisson_iters, check=args.mp_check, repeats=reps)
    f64_same = f64_k10 = None
    if mp_leg is not None and args.mp_check != 10:
        f64_same = gpu_leg(case, ibm.RBSOR, args.mp_steps, args.warmup, 0, args.max_poisson_iters,
                           check=args.mp_check)
    if mp_leg is not None:
        # the plain FP64 solve (stop test every 10 iterations) over the same steps
        f64_k10 = gpu_leg(case, ibm.RBSOR, args.mp_steps, args.warmup, 0, args.max_poisson_iters)
    c3 = None
    if args.solver == "sor" and args.c3_iters > 0:
        case3 = W.plunging_2048x1536()
        c3 = {}
        for name, m in (("f64", ibm.RBSOR), ("mixed", ibm.RBSOR_MP)):
            leg = gpu_leg(case3, m, 1, 0, args.profile_every, args.c3_iters,
                          check=args.mp_check if m == ibm.RBSOR_MP else None)
            c3[name] = {"s_per_step": round(leg["wall"], 4), "poisson_iters": leg["iters"][0],
                        "us_per_iteration": round(1e6 * leg["wall"] / max(leg["iters"][0], 1), 3)}

    # dominant kernel of the headline leg: the most total sampled time
    cands = ((ibm.KERNEL_SOR_TB, ibm.KERNEL_SOR_SWEEP) if method == ibm.RBSOR
             else (ibm.KERNEL_PCG_DIR_SPMV, ibm.KERNEL_PCG_UPDATE))
    kid = max(cands, key=lambda k: main_leg["prof"][k]["avg_ms"] * main_leg["prof"][k]["launches"])
    q = main_leg["prof"][kid]
    kname = ibm.KERNEL_NAMES[kid]
    dur = q["avg_ms"] * 1e-3
    eff = q["bytes_per_launch"] / dur / 1e9 if dur > 0 else 0.0
    cnt = read_counters(kname, tag)
    traffic = _counter(cnt, "hbm_bytes_per_launch")
    # The sweep's data (phi and V b, 12.6 MB) stays in L2 and the Infinity
    # Cache: the counters show HBM-side traffic far below the algorithmic
    # 24 B per update and the VALU busy about half the time, so the kernel is
    # placed against the FP64 vector roofline with its algorithmic FLOPs.
    if method == ibm.RBSOR:
        flops = SOR_FLOP_PER_UPDATE * q["bytes_per_launch"] / 24.0
        tf = flops / dur / 1e12 if dur > 0 else 0.0
        head = {"bound": "alu", "achieved": round(tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP64_PEAK_TFLOPS, 4)}
    else:  # the PCG kernels stream their vectors
        flops = None
        head = {"bound": "hbm", "achieved": round(eff, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(eff / HBM_PEAK_GBS, 4)}
    roofline = {**head, "traffic": traffic,
                "kernel": kname, "avg_us": round(q["avg_ms"] * 1e3, 3), "samples": q["samples"],
                "launches": q["launches"], "alg_flops_per_launch": flops,
                "alg_bytes_per_launch": q["bytes_per_launch"],
                "effective_GBps_algorithmic": round(eff, 1),
                "effective_frac_of_hbm_peak": round(eff / HBM_PEAK_GBS, 4),
                "hbm_GBps_counters": round(traffic / dur / 1e9, 1) if traffic and dur > 0 else None,
                "hbm_frac_counters": round(traffic / dur / 1e9 / HBM_PEAK_GBS, 4) if traffic and dur > 0 else None,
                "valu_busy_counters": _counter(cnt, "valu_busy"),
                "wait_frac_counters": _counter(cnt, "wait_frac")}

    steps = args.steps
    ms_per_step = 1e3 * main_leg["wall"] / steps
    iters_per_step = sum(main_leg["iters"]) / steps
    out = {
        "metric": METRIC,
        "value": round(main_leg["cell_updates_per_s"], 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case["name"] + ", dt 5e-4, h 0.5, f 0.4, stretched 16c x 12c grid",
                   "nx": case["nx"], "ny": case["ny"],
                   "solver": ("red-black SOR omega 1.8, tol 1e-8 every 10 iterations"
                              if method == ibm.RBSOR else "Jacobi-PCG, tol 1e-8"),
                   "initial_guess": "previous phi", "first_timed_step": args.warmup + 1,
                   "poisson_iteration_cap": args.max_poisson_iters or None},
        "s_per_time_step": round(main_leg["wall"] / steps, 6),
        "s_per_time_step_runs": [round(w / steps, 6) for w in main_leg["walls"]],
        "phases_ms_per_step": _round_phases(main_leg["phases_ms"]),
        "poisson_iters_per_step": main_leg["iters"],
        "poisson_iters_mean": iters_per_step,
        "roofline": roofline,
    }
    if pcg_leg is not None:
        out["pcg"] = {"s_per_time_step": round(pcg_leg["wall"] / args.pcg_steps, 6),
                      "s_per_time_step_runs": [round(w / args.pcg_steps, 6) for w in pcg_leg["walls"]],
                      "phases_ms_per_step": _round_phases(pcg_leg["phases_ms"]),
                      "poisson_iters_per_step": pcg_leg["iters"],
                      "cell_updates_per_s": round(pcg_leg["cell_updates_per_s"], 1),
                      "kernels_avg_us": {ibm.KERNEL_NAMES[k]: round(pcg_leg["prof"][k]["avg_ms"] * 1e3, 3)
                                         for k in (ibm.KERNEL_PCG_DIR_SPMV, ibm.KERNEL_PCG_UPDATE)}}
    if cg1_leg is not None:
        q = cg1_leg["prof"][ibm.KERNEL_CG1_ITER]
        out["pcg_one_reduction"] = {
            "solver": "Jacobi-PCG with one reduction per iteration (one kernel per iteration), tol 1e-8",
            "s_per_time_step": round(cg1_leg["wall"] / args.pcg_steps, 6),
            "s_per_time_step_runs": [round(w / args.pcg_steps, 6) for w in cg1_leg["walls"]],
            "phases_ms_per_step": _round_phases(cg1_leg["phases_ms"]),
            "poisson_iters_per_step": cg1_leg["iters"],
            "cell_updates_per_s": round(cg1_leg["cell_updates_per_s"], 1),
            "speedup_vs_pcg": round(pcg_leg["wall"] / cg1_leg["wall"], 3) if cg1_leg["wall"] > 0 else None,
            "k_cg1_iter": {"avg_us": round(q["avg_ms"] * 1e3, 3),
                           "effective_GBps": round(q["bytes_per_launch"] / (q["avg_ms"] * 1e-3) / 1e9, 1)
                           if q["avg_ms"] > 0 else None}}
    if mp_leg is not None:
        mp_steps = args.mp_steps
        kern = {}
        for k in (ibm.KERNEL_SOR_MP, ibm.KERNEL_SOR_MP_REFINE):
            q = mp_leg["prof"][k]
            if q["avg_ms"] > 0:
                kern[ibm.KERNEL_NAMES[k]] = {
                    "avg_us": round(q["avg_ms"] * 1e3, 3),
                    "achieved_GBps": round(q["bytes_per_launch"] / (q["avg_ms"] * 1e-3) / 1e9, 1)}
        mp_s = mp_leg["wall"] / mp_steps
        f64_same_s = f64_same["wall"] / mp_steps if f64_same is not None else main_leg["wall"] / steps
        out["mixed_precision"] = {
            "solver": "red-black SOR omega 1.8, float sweeps on the correction, double residual, update and "
                      f"stop test every {args.mp_check} iterations, tol 1e-8",
            "check_interval": args.mp_check,
            "s_per_time_step": round(mp_s, 6),
            "s_per_time_step_runs": [round(w / mp_steps, 6) for w in mp_leg["walls"]],
            "phases_ms_per_step": _round_phases(mp_leg["phases_ms"]),
            "poisson_iters_per_step": mp_leg["iters"],
            "f64_sor_same_steps": {"s_per_time_step": round(f64_k10["wall"] / mp_steps, 6),
                                   "poisson_iters_per_step": f64_k10["iters"]},
            "speedup_vs_f64_sor": round((f64_k10["wall"] / mp_steps) / mp_s, 3) if mp_s > 0 else None,
            "f64_same_interval": {"s_per_time_step": round(f64_same_s, 6),
                                  "poisson_iters_per_step": (f64_same or main_leg)["iters"]},
            "speedup_vs_f64_same_interval": round(f64_same_s / mp_s, 3) if mp_s > 0 else None,
            "kernels": kern}
    if c3 is not None:
        out["c3_capped"] = dict(c3, workload="plunging ellipse 2048x1536, Re 1000, h 0.6, f 0.5; first step, "
                                             f"Poisson solve capped at {args.c3_iters} iterations",
                                speedup_per_iteration=round(c3["f64"]["us_per_iteration"] /
                                                            max(c3["mixed"]["us_per_iteration"], 1e-9), 3))
    if learned:
        out["learned"] = learned_legs(case, args, main_leg)
    if args.solver == "sor" and args.c4_cases > 0:
        out["batched_cases"] = batch_leg(args)
    if args.stress:
        out["stress_hbm"] = stress_leg()
    if args.c1:
        out["c1_full_run"] = c1_leg(cpu=args.cpu_seconds > 0)
    captured = []
    if args.solver == "sor" and args.pcg_long_steps > 0:
        marks = tuple(k for k in (1, 10, 100, args.pcg_long_steps) if k <= args.pcg_long_steps) \
            if args.poisson_bench else ()
        out["pcg_long"], captured = pcg_long_leg(case, args.pcg_long_steps, ibm.CG1, args.late_sor_steps,
                                                 capture=marks)
    if args.poisson_bench:
        out["poisson_bench"] = poisson_bench_leg(case, captured=captured)
    if args.scaling:
        out["input_scaling"] = scaling_leg()
    if args.cpu_seconds > 0:
        # the oracle on all host threads (the paper's OpenMP SOL1 analogue)
        # and on one (its serial SOL0 analogue); speedups as the paper forms
        # them: S = T_reference / T_gpu per time step
        gpu_step = main_leg["wall"] / steps
        cb = cpu_leg(case, args.cpu_seconds, iters_per_step)
        cb1 = cpu_leg(case, args.cpu_seconds, iters_per_step, threads=1)
        cb["speedup_s_per_step"] = round(cb["s_per_time_step_est"] / gpu_step, 2)
        cb["one_thread"] = {k: cb1[k] for k in ("value", "cores", "sample", "seconds", "s_per_time_step_est")}
        cb["one_thread"]["speedup_s_per_step"] = round(cb1["s_per_time_step_est"] / gpu_step, 2)
        cb["threads_over_one_thread"] = round(cb1["s_per_time_step_est"] / cb["s_per_time_step_est"], 3)
        out["cpu_baseline"] = cb
        out["paper_speedups"] = PAPER_SPEEDUPS
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the fused coupled lattice-Boltzmann ice-growth step on one MI355X.

Headline: coupled MLUPS (cells x steps / s / 1e6) of the ventilated 2048 x 2048 workload (D2Q9 flow
with the crystal as a solid, D2Q5 vapour, phase field with 6-fold anisotropy; inlet u = 0.01, seed
R = 8 at (300, 1024)) in FP32 storage, with all state resident in HBM.  One timed "step" is one
coupled time step (the fused kernel, replayed from captured HIP graphs); exactly --steps steps are
timed, five times over, and the median is reported; the FP64 conservation diagnostics follow the timed
runs and are timed on their own.  Also reported: the HBM roofline of the step kernel (algorithmic
bytes per launch over its measured average duration), the practical copy-kernel ceiling, 16-bit
storage variants, and the FP64 CPU oracle timed on the host cores on a bounded sample.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E published peak


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def bytes_per_update(flow: bool, storage: str) -> int:
    """Algorithmic HBM bytes per cell update of the method: every population read once and written
    once (4 B in FP32 storage, 2 B in 16-bit storage), plus phi_prev (FP32) read and written."""
    npop = 23 if flow else 14
    e = 4 if storage == "fp32" else 2
    return npop * e * 2 + 4 * 2


def impl_bytes_per_update(flow: bool, storage: str) -> int:
    """Bytes per cell update this implementation moves: the algorithmic bytes, plus in 16-bit storage
    the cell's 16-bit reference values (U, and rho, jx, jy with flow) read and written."""
    refs = 0 if storage == "fp32" else (4 if flow else 1) * 2 * 2
    return bytes_per_update(flow, storage) + refs


def launch_name(grid_mode: int) -> str:
    """The launch a grid mode selects: bit 0 persistent grid, grid_mode >> 1 the tile order."""
    return "%s, %s" % ("persistent grid" if grid_mode & 1 else "one workgroup per tile",
                       ("row order", "512-cell strips", "four strips")[grid_mode >> 1])


def kernel_source_sha() -> str:
    """Hash of the step kernel's code (its source and the two headers it is built from), comments and
    blank space removed, so that only a change of that code marks counters as stale."""
    h = hashlib.sha256()
    for name in ("snowlb_kernels.hip", "snowlb_device.h", "snowlb_internal.h"):
        for line in open(os.path.join(ROOT, "paper_2101_07163_amd", "csrc", name)):
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


ORDER_SUFFIX = {0: "", 1: "_strips", 2: "_four_strips"}  # tile order (grid_mode >> 1) -> summary name


def kernel3_source_sha() -> str:
    """The same hash for the 3D step kernel (its source and its descriptor header)."""
    h = hashlib.sha256()
    for name in ("snowlb3d_kernels.hip", "snowlb3d_internal.h"):
        for line in open(os.path.join(ROOT, "paper_2101_07163_amd", "csrc", name)):
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(workload: str, storage: str, tile: str = "64x4", grid_mode: int = 0):
    """Measured HBM bytes per launch from the committed rocprofv3 counter summary of this launch (tile
    shape and grid mode), if it was taken on the current kernel source; None otherwise."""
    p = os.path.join(ROOT, "profiles", "k_step_%s_%s%s_traffic.txt" % (
        workload, storage, ORDER_SUFFIX.get(grid_mode >> 1, "_unknown")))
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    if kv.get("tile", tile) != tile or kv.get("grid_mode", str(grid_mode)) != str(grid_mode):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


REPEATS = 5  # timed repeats of the K steps; the median is reported


def time_steps(S, torch, cfg, storage, steps, warmup, tile, repeats=REPEATS, grid_mode=-1):
    """W untimed warm-up steps, then `repeats` timed runs of exactly `steps` steps, each bracketed by
    device synchronisation, replayed from captured graphs on the current stream; the kernel time per
    step comes from events on that stream.  Returns the median wall time, the median event time per
    step, the timings of every repeat, and the FP64 diagnostics taken after the timed runs (their
    synchronisation is timed on its own)."""
    sim = S.Sim(cfg, storage=storage, tile=tile)
    if grid_mode >= 0:
        sim.set_grid_mode(grid_mode)
    sim.init()
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()  # the kernels are launched on this stream
    walls, kms = [], []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kms.append(e0.elapsed_time(e1) / steps)
    t0 = time.perf_counter()
    diag = sim.diag()  # FP64 conservation sums; synchronises the stream
    diag_ms = (time.perf_counter() - t0) * 1e3
    return sim, float(np.median(walls)), float(np.median(kms)), diag, {
        "wall_s": [round(w, 6) for w in walls], "kernel_ms": [round(k, 5) for k in kms],
        "diag_ms": round(diag_ms, 3)}


def bw_probe(S, torch, nbytes=2 << 30, reps=10):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    S.snowlb_bw_probe(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.snowlb_bw_probe(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def stencil_family(S, torch, W, cfg, storage, steps, tile):
    """The gradient-stencil family of Sec. 3.1.1 on the headline workload (same bytes per update;
    E6 and E8 stage a two-cell halo) and on the stencil-study workload (800^2, thermal model), MLUPS."""
    cells = cfg["nx"] * cfg["ny"]
    bpu = bytes_per_update(bool(cfg.get("flow", 0)), storage)
    res = {"workload": cfg["name"], "storage": storage}
    for st in (2, 4, 6, 8):
        sim, wall, k_ms, _, _ = time_steps(S, torch, dict(cfg, stencil=st), storage, steps, 50, tile)
        res["E%d" % st] = {"MLUPS": round(cells * steps / wall / 1e6, 1), "kernel_avg_ms": round(k_ms, 5),
                           "GBps_algorithmic": round(cells * bpu / (k_ms * 1e-3) / 1e9, 1)}
        del sim
    study = {"workload": W.F1["name"], "steps": 20000}
    for st in (2, 4, 6, 8):
        c = dict(W.F1, stencil=st)
        sim, wall, k_ms, _, _ = time_steps(S, torch, c, "fp32", 20000, 200, tile, repeats=1)
        study["E%d_MLUPS" % st] = round(c["nx"] * c["ny"] * 20000 / wall / 1e6, 1)
        del sim
    res["study"] = study
    res["fourfold"] = fourfold_setup(S, torch, W, tile)
    return res


def axis_tip(phi, cx, cy):
    """Distance from the seed centre to the phi = 0 crossing along the +x lattice axis (linear
    interpolation between the last ice node and the next one)."""
    row = phi[int(cy), int(cx):]
    i = int(np.nonzero(row >= 0)[0][-1])
    return i + float(row[i] / (row[i] - row[i + 1]))


def fourfold_setup(S, torch, W, tile):
    """The four-fold validation set-up of Sec. 3.1.2 at its own sizes and lengths: tip distance at
    the end and the dimensionless tip velocity V d0 / D over the last fifth of the run."""
    a1 = 5.0 * math.sqrt(2.0) / 8.0
    out = {}
    for c in (W.FOURFOLD, W.FOURFOLD_055):
        sim = S.Sim(c, tile=tile).init()
        n = c["steps"]
        t_a = (4 * n) // 5
        sim.step(t_a)
        r_a = axis_tip(sim.read("phi").cpu().numpy(), *c["seed"][:2])
        sim.step(n - t_a)
        r_b = axis_tip(sim.read("phi").cpu().numpy(), *c["seed"][:2])
        d0 = a1 * c["W0"] / c["lam"]
        D = (c["tau_vap"] - 0.5) / 3.0
        out[c["name"]] = {"U0": c["U0"], "steps": n, "tip_cells": round(r_b, 2),
                          "V_d0_over_D": round((r_b - r_a) / (n - t_a) * d0 / D, 5)}
        del sim
    return out


def habit_sweep(S, torch, W, steps=20000, warmup=200):
    """The seven Table 2 morphologies (Sec. 3.2.1) on 400^2 through the physical-unit front end, as
    one batch: aggregate MLUPS."""
    from paper_2101_07163_amd import units
    cfgs = [units.plate_regime(U0, L) for (_, _, U0, L) in W.TABLE2]
    b = S.Batch(cfgs, tile=-1).init()
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = {"domains": len(cfgs), "cells": b.cells, "steps": steps, "tile": S.snowlb_tile_name(b.tile),
           "batched_MLUPS": round(b.cells * steps / wall / 1e6, 1)}
    del b
    return res


def batch_sweep(S, torch, W, steps=200, warmup=20, solo_steps=64):
    """The 64-crystal sweep as one batch (one launch per step over all tiles) against the same work
    done crystal by crystal (solo contexts, graph-replayed), both in aggregate MLUPS."""
    cfgs = W.c4_domains()
    b = S.Batch(cfgs, tile=-1).init()
    b.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = b.cells
    tile = S.snowlb_tile_name(b.tile)
    del b
    torch.cuda.empty_cache()
    solo_ms = 0.0
    for c in cfgs:
        sim = S.Sim(c).init()
        sim.step(8)
        torch.cuda.synchronize()
        e0.record()
        sim.step(solo_steps)
        e1.record()
        torch.cuda.synchronize()
        solo_ms += e0.elapsed_time(e1)
        del sim
    return {"domains": len(cfgs), "cells": cells, "steps": steps, "tile": tile,
            "batched_MLUPS": round(cells * steps / (ms * 1e-3) / 1e6, 1),
            "solo_sum_MLUPS": round(cells * solo_steps / (solo_ms * 1e-3) / 1e6, 1)}


def adjoint_ratio(S, torch, W):
    """The adjoint workload (512^2, no flow, 5000 steps, sqrt(N) checkpoints): time of the forward pass
    with checkpoints, of the backward pass (recompute + reverse steps), their ratio, and the plain
    forward for reference."""
    cfg = dict(W.C5)
    n = cfg["steps"]
    sim = S.Sim(cfg)
    U = torch.from_numpy(W.c5_U_init(cfg)).float().cuda()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    sim.init(U).step(n)  # warm-up (code objects, graph)
    torch.cuda.synchronize()
    sim.init(U)
    e0.record(stream)
    sim.step(n)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    sim.init(U)
    e0.record(stream)
    S.snowlb_adj_forward(sim.ctx, n, 0, stream.cuda_stream)
    e1.record(stream)
    phi = sim.read("phi")
    seed = (2 * phi).contiguous()
    dU = torch.empty_like(seed)
    torch.cuda.synchronize()
    e1b = torch.cuda.Event(enable_timing=True)
    e1b.record(stream)
    S.snowlb_adj_backward(sim.ctx, seed.data_ptr(), dU.data_ptr(), stream.cuda_stream)
    e2.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    bwd_ms = e1b.elapsed_time(e2)
    cells = cfg["nx"] * cfg["ny"]
    return {"workload": cfg["name"], "steps": n, "ckpt_stride": int(-(-n ** 0.5 // 1)),
            "forward_ms": round(fwd_ms, 2), "backward_ms": round(bwd_ms, 2),
            "adjoint_forward_ratio": round(bwd_ms / fwd_ms, 3),
            "plain_forward_ms": round(plain_ms, 2),
            "plain_forward_MLUPS": round(cells * n / (plain_ms * 1e-3) / 1e6, 1)}


def three_d(S, torch, W, steps=200, warmup=20):
    """The 3D extension on its workload (256 x 128 x 128 ventilated crystal, FP32): MLUPS and the
    step kernel's algorithmic bandwidth, (19 + 7 + 7) populations x 4 B read and written plus phi_prev
    read and written = 272 B per cell update."""
    cfg = W.F4_3D
    sim = S.Sim3D(cfg).init()
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    walls, kms = [], []
    for _ in range(REPEATS):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kms.append(e0.elapsed_time(e1) / steps)
    cells = cfg["nx"] * cfg["ny"] * cfg["nz"]
    bpu = (19 + 7 + 7) * 4 * 2 + 8
    k_ms = float(np.median(kms))
    gbs = cells * bpu / (k_ms * 1e-3) / 1e9
    d = sim.diag()
    del sim
    return {"workload": cfg["name"], "steps": steps, "MLUPS": round(cells * steps / float(np.median(walls)) / 1e6, 1),
            "kernel_avg_ms": round(k_ms, 5), "bytes_per_update": bpu, "GBps_algorithmic": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "finite": d["status"] == S.OK}


def cpu_baseline(cfg, seconds, threads=0):
    """The FP64 oracle timed on a bounded sample of the workload (whole steps of the full lattice from
    the seeded initial state), on all host threads or on `threads` of them."""
    import oracle
    all_threads = oracle.threads()
    if threads:
        oracle.set_threads(threads)
    try:
        o = oracle.Oracle(oracle.Params.from_dict(cfg)).init_seed(*cfg["seed"], cfg["w_init"], cfg["U0"])
        o.step(1)  # first-touch of the buffers outside the timed sample
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            o.step(1)
            n += 1
        dt = time.perf_counter() - t0
        used = oracle.threads()
    finally:
        oracle.set_threads(all_threads)
    cells = cfg["nx"] * cfg["ny"]
    return {"value": round(cells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": used,
            "kind": "oracle",
            "sample": "%s, FP64 oracle, %d steps of the full %dx%d lattice from the seeded initial "
                      "state (%.1f s)" % (cfg["name"], n, cfg["nx"], cfg["ny"], dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--tile", type=int, default=-1, help="-1: autotune")
    ap.add_argument("--grid-mode", type=int, default=-1,
                    help="with --tile >= 0: launch mode (bit 0 persistent grid; mode >> 1: 0 row order, "
                         "1 512-cell strips, 2 four strips)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="copy,fp16,bf16,c4,c5,stencils,table2,f4",
                    help="comma list of extra measurements: copy (copy-kernel ceiling), fp16, bf16, "
                         "c4 (64-crystal batch), c5 (adjoint/forward time ratio), stencils, table2 (habit "
                         "sweep), f4 (the 3D extension)")
    args = ap.parse_args()
    if args.grid_mode >= 0 and args.tile < 0:
        ap.error("--grid-mode needs an explicit --tile (with --tile -1 the autotuner picks both)")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the lattice would "
              "shard by spatial domain decomposition, with one exchange of boundary populations per step). "
              "Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2101_07163_amd import snowlb as S
    from paper_2101_07163_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = {"c1": W.C1, "c2": W.C2, "c3": W.C3}[args.workload]
    cells = cfg["nx"] * cfg["ny"]
    flow = bool(cfg["flow"])

    log("workload %s %dx%d storage %s: warmup %d, timed %d steps" % (
        cfg["name"], cfg["nx"], cfg["ny"], args.storage, args.warmup, args.steps))
    sim, wall, kernel_ms, diag, reps = time_steps(S, torch, cfg, args.storage, args.steps, args.warmup, args.tile,
                                                   grid_mode=args.grid_mode)
    mlups = cells * args.steps / wall / 1e6
    bpu = bytes_per_update(flow, args.storage)
    achieved = cells * bpu / (kernel_ms * 1e-3) / 1e9
    log("MLUPS %.1f (median of %d), step kernel %.4f ms, %.0f GB/s algorithmic, tile %s, %s; repeats %s" % (
        mlups, REPEATS, kernel_ms, achieved, S.snowlb_tile_name(sim.tile), launch_name(sim.grid_mode), reps))
    if diag["status"] != S.OK:
        raise SystemExit("non-finite state after the timed steps")

    traffic = load_traffic(cfg["name"], args.storage, S.snowlb_tile_name(sim.tile), sim.grid_mode)
    out = {
        "metric": "coupled MLUPS and % HBM roofline at 2048^2; adjoint/forward time ratio",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "f32 (%s storage)" % args.storage,
        "data": "synthetic: circular ice seed in uniform supersaturation with uniform inflow",
        "config": {"workload": cfg["name"], "nx": cfg["nx"], "ny": cfg["ny"], "storage": args.storage,
                   "flow": "D2Q9 inlet/outlet" if cfg.get("inout") else ("D2Q9 periodic" if flow else "off"),
                   "u_in": cfg.get("u_in"), "eps": cfg["eps"], "tile": S.snowlb_tile_name(sim.tile),
                   "launch": launch_name(sim.grid_mode)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": "k_step", "bytes_per_update": bpu,
                     "impl_bytes_per_update": impl_bytes_per_update(flow, args.storage),
                     "kernel_avg_ms": round(kernel_ms, 5)},
        "timing": {"repeats": REPEATS, "statistic": "median", "path": "captured HIP graphs",
                   "wall_s": reps["wall_s"], "kernel_ms_per_step": reps["kernel_ms"],
                   "diag_sync_ms": reps["diag_ms"]},
    }
    del sim
    torch.cuda.empty_cache()

    if not args.no_extras:
        extras = {}
        wanted = set(x for x in args.extras.split(",") if x)
        if "copy" in wanted:
            extras["copy_ceiling_GBps"] = round(bw_probe(S, torch), 1)
            extras["copy_probe_bytes"] = 2 << 30
            log("copy-kernel ceiling %.0f GB/s" % extras["copy_ceiling_GBps"])
        for st in ("fp16", "bf16"):
            if st == args.storage or st not in wanted:
                continue
            s2, w2, k2, _, _ = time_steps(S, torch, cfg, st, min(args.steps, 1000), 100, args.tile,
                                          grid_mode=args.grid_mode)
            launch2 = "%s, %s" % (S.snowlb_tile_name(s2.tile), launch_name(s2.grid_mode))
            b2 = bytes_per_update(flow, st)
            i2 = impl_bytes_per_update(flow, st)
            extras["%s_storage" % st] = {"MLUPS": round(cells * min(args.steps, 1000) / w2 / 1e6, 1),
                                         "kernel_avg_ms": round(k2, 5),
                                         "GBps_algorithmic": round(cells * b2 / (k2 * 1e-3) / 1e9, 1),
                                         "frac_algorithmic": round(cells * b2 / (k2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                         "bytes_per_update": b2,
                                         "impl_bytes_per_update": i2,
                                         "GBps_impl": round(cells * i2 / (k2 * 1e-3) / 1e9, 1),
                                         "launch": launch2}
            log("%s storage: %s" % (st, extras["%s_storage" % st]))
            del s2
        if "stencils" in wanted:
            extras["stencils"] = stencil_family(S, torch, W, cfg, args.storage, min(args.steps, 1000), args.tile)
            log("gradient stencils: %s" % extras["stencils"])
        if "table2" in wanted:
            extras["table2_habits"] = habit_sweep(S, torch, W)
            log("Table 2 habit sweep: %s" % extras["table2_habits"])
        if "c4" in wanted:
            extras["c4_batch"] = batch_sweep(S, torch, W)
            log("64-crystal batch: %s" % extras["c4_batch"])
        if "c5" in wanted:
            extras["c5_adjoint"] = adjoint_ratio(S, torch, W)
            log("adjoint: %s" % extras["c5_adjoint"])
        if "f4" in wanted:
            extras["f4_3d"] = three_d(S, torch, W)
            log("3D extension: %s" % extras["f4_3d"])
        out["extras"] = extras

    if not args.no_cpu_baseline:
        log("CPU baseline: FP64 oracle for %.0f s" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
        log("CPU baseline %s" % out["cpu_baseline"])
        if "extras" in out:  # the same oracle on one thread, for a per-core figure
            out["extras"]["cpu_baseline_1thread"] = cpu_baseline(cfg, min(5.0, args.cpu_seconds), threads=1)
            log("CPU baseline, one thread %s" % out["extras"]["cpu_baseline_1thread"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

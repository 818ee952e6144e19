#!/usr/bin/env python3
"""Throughput benchmark of the pCT reconstruction hot path on one MI355X.

Workload (default, config 3): 2e8 seeded synthetic proton histories made on
the device, through a 200 x 200 x 40 grid of 1 mm voxels (elliptic head
phantom with 8 inserts), 180 gantry angles, 8 DROP sweeps in blocks of 2e5
histories, every row rebuilt from the histories in every block (A is never
stored).  --config 2 / 4: 1e7 histories with rows cached in HBM (FP32 / FP16
lengths) and swept through the tiled plan.

One step = one whole reconstruction through the C ABI (pct_reconstruct)
from device-resident histories: rebuilt rows: per-proton path set-up, then
the 8 sweeps (most-likely path + voxel walk + projection + scatter + block
update in every block; the first sweep also counts s_j, the later ones read
the kept counts); cached rows: trace, plan build, 6 sweeps and the FP64
residual after every sweep.  value = histories x sweeps / step time
(histories per second per sweep).

Also reported: per-kernel device times (HIP events on the launching stream),
the roofline of the dominant kernel (for rebuilt rows: the largest of its
path-arithmetic, cache-gather and atomic times against measured peaks of
the same access patterns), the FP64 residual of the final image, the time to
reach <= 1% RSP error in the insert ROIs, and the FP64 CPU oracle timed on a
bounded sample of the same workload on this job's host threads.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X vector FP64
# FP64 operations per most-likely-path sample in the path kernel (an FMA counts
# as 2): three antiderivative moments F_p(d1) (8-term Horner + powers, 54),
# I_m and J_m from them (17), Highland scaling (6), the 2x2 gain and the two
# lateral offsets (36), world and grid coordinates (15), the segment to the
# next sample (length, floor, local frame: 17) and its voxel walk (3 axes of
# crossing set-up plus ~2 steps: 15)
PATH_FLOPS_PER_POINT = 160
CALIB_BYTES = 1 << 30      # plain copy used to scale the FETCH/WRITE counters
KERNEL_SOURCES = ("path_device.h", "trace.hip", "sweep.hip", "plan.hip", "abi.hip", "pct_internal.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3,
                    help="workload: 3 (2e8 histories, rows rebuilt in every sweep), 2 (1e7, FP32 rows cached) "
                         "or 4 (1e7, FP16 rows cached)")
    ap.add_argument("--n", type=int, default=None, help="override the history count")
    ap.add_argument("--fused", action="store_true", help="recompute rows in every sweep (config 3 always does)")
    ap.add_argument("--no-plan", action="store_true", help="cached rows swept with atomics (no tiled plan)")
    ap.add_argument("--path-fp32", action="store_true", help="FP32 path positions (reduced precision)")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-accuracy", action="store_true")
    ap.add_argument("--skip-variants", action="store_true", help="rebuilt rows: do not also time the FP32-path form")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="histories the CPU oracle runs on (default: 2e6 with rows rebuilt, 3e6 with cached rows, "
                         "10-20 s of host time)")
    ap.add_argument("--max-sweeps-acc", type=int, default=30)
    ap.add_argument("--warmstart", action="store_true",
                    help="learned warm start: train the 3D U-Net on solver pairs of seeded phantoms, then compare "
                         "the time to <= 1%% RSP error from the hull start and from the network's x0")
    ap.add_argument("--block-study", action="store_true",
                    help="RSP error per sweep and time per sweep for several DROP block sizes (config 2 data) and exit")
    ap.add_argument("--block-sizes", type=str, default="20000,50000,200000,1000000,10000000")
    ap.add_argument("--tvs-study", action="store_true",
                    help="TV superiorization before every block against plain DROP (config 2) and exit")
    ap.add_argument("--tvs-beta0", type=float, default=1.0)
    ap.add_argument("--tvs-a", type=float, default=0.995)
    ap.add_argument("--cnn-timing", action="store_true",
                    help="time the warm-start network's kernels on one 200x200x40 volume and exit")
    ap.add_argument("--ws-train", type=int, default=24, help="training phantoms (seeds 1000, 1001, ...)")
    ap.add_argument("--ws-n", type=int, default=10_000_000, help="histories per phantom (training and evaluation)")
    ap.add_argument("--ws-steps", type=int, default=3000, help="Adam steps (one phantom per step)")
    ap.add_argument("--ws-lr", type=float, default=5e-4)
    ap.add_argument("--ws-variants", type=str, default="1:0:truth,1:0:clean,2:0:out",
                    help="networks to compare, comma separated: '<input sweeps joined by ->:<coarse-loss weight>"
                         "[:out|truth|clean]' (target: the image after --ws-out sweeps, the phantom itself, or "
                         "the image after --ws-out sweeps of the same protons without WEPL noise)")
    ap.add_argument("--ws-out", type=int, default=20, help="sweeps of the training target")
    ap.add_argument("--ws-ensemble", type=int, default=3,
                    help="networks per variant, trained from different seeds; the warm start is their mean")
    ap.add_argument("--ws-channels", type=str, default="16,32,64,64")
    ap.add_argument("--ws-precision", choices=("f32", "bf16"), default="bf16",
                    help="the network's convolutions: FP32, or bfloat16 on the matrix cores where the shape allows")
    ap.add_argument("--ws-eval-2e8", action="store_true",
                    help="also compare the starts on the 2e8-history workload (needs a network on the 1-sweep image)")
    ap.add_argument("--ws-eval-seeds", type=str, default="3,2,5000,5001",
                    help="held-out phantoms (3: the 2e8 workload's phantom, 2: the 1e7 workload's)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this benchmark and exit")
    return ap.parse_args()


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1707_05014_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_dir, write_dir, out_json):
    """Per-kernel FETCH_SIZE / WRITE_SIZE (KiB per dispatch) from rocprofv3
    counter CSVs, with the scale factor read off the 1 GiB calibration copy."""
    import collections
    import csv
    import glob

    def load(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                agg[r["Kernel_Name"].split("(")[0].replace("void ", "")].append(float(r["Counter_Value"]))
        return agg

    fetch = load(fetch_dir, "FETCH_SIZE")
    write = load(write_dir, "WRITE_SIZE")
    # the calibration is a 1 GiB device-to-device torch copy, which the runtime
    # runs as its blit kernel: the largest copyBuffer dispatch of the run
    copy = [k for k in fetch if "copyBuffer" in k]
    calib_kib = CALIB_BYTES / 1024
    f_cal = max(v for k in copy for v in fetch[k])
    w_cal = max(v for k in copy for v in write.get(k, [0.0]))
    out = {"source_hash": source_hash(), "fetch_scale": f_cal / calib_kib, "write_scale": w_cal / calib_kib,
           "kernels": {}}
    for k in fetch:
        if not k.startswith("pct::"):
            continue
        fv, wv = fetch[k], write.get(k, [])
        out["kernels"][k] = {"dispatches": len(fv), "fetch_kib_per_dispatch": sum(fv) / len(fv),
                             "write_kib_per_dispatch": (sum(wv) / len(wv)) if wv else None}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


def path_points(h, cfg) -> int:
    """Number of most-likely-path samples over all histories (sum of K + 1 over
    histories whose entry and exit lines meet the hull): the work count of
    the path kernels, from the hull geometry alone (float64, on the device
    that holds the histories, in chunks)."""
    import torch
    b = cfg.phantom.body
    a2, b2 = b.ax[0] ** 2, b.ax[1] ** 2
    step = min(cfg.grid.dx, cfg.grid.dy, cfg.grid.dz)
    n = h["phi"].numel()
    total = 0
    for i0 in range(0, n, 1 << 24):
        f64 = lambda k: h[k][i0:i0 + (1 << 24)].to(torch.float64)  # noqa: E731
        phi = f64("phi")
        c, s = torch.cos(phi), torch.sin(phi)

        def interval(u_ref, t, v, st, sv):
            T = t - st * u_ref
            V = v - sv * u_ref
            px, qx = c - st * s, -T * s
            py, qy = s + st * c, T * c
            A = px * px / a2 + py * py / b2
            B = 2 * (px * qx / a2 + py * qy / b2)
            C = qx * qx / a2 + qy * qy / b2 - 1
            disc = B * B - 4 * A * C
            ok = disc > 0
            sq = torch.sqrt(torch.where(ok, disc, torch.zeros_like(disc)))
            lo, hi = (-B - sq) / (2 * A), (-B + sq) / (2 * A)
            nz = sv != 0
            svs = torch.where(nz, sv, torch.ones_like(sv))
            z0 = torch.where(nz, (b.z0 - V) / svs, torch.full_like(sv, -float("inf")))
            z1 = torch.where(nz, (b.z1 - V) / svs, torch.full_like(sv, float("inf")))
            lo = torch.maximum(lo, torch.minimum(z0, z1))
            hi = torch.minimum(hi, torch.maximum(z0, z1))
            ok &= nz | ((V >= b.z0) & (V <= b.z1))
            return lo, hi, ok & (hi > lo)

        lo0, _, ok0 = interval(cfg.beam.u_in, f64("t_in"), f64("v_in"), f64("dt_in"), f64("dv_in"))
        _, hi2, ok2 = interval(cfg.beam.u_out, f64("t_out"), f64("v_out"), f64("dt_out"), f64("dv_out"))
        L = hi2 - lo0
        ok = ok0 & ok2 & (L > 0)
        K = torch.clamp(torch.ceil(L[ok] / step - 1e-9), min=1)
        total += int(torch.sum(K + 1).item())
    return total


def host_info() -> dict:
    """Cores and CPU model of the host (for the oracle baseline)."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    info["omp_num_threads"] = os.environ.get("OMP_NUM_THREADS")
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def probe_peaks(dev) -> dict:
    """Measured peaks of the memory paths (pct_probe): HBM copy, path-like
    4-byte gathers inside the image (6.4 MB: last-level cache), path-like
    global FP32 atomic adds into it, LDS atomic adds."""
    from paper_1707_05014_amd import api
    M = 1_600_000
    out = {}
    ms, _ = api.probe("copy", 1 << 28, reps=5)
    out["hbm_copy_GBps"] = round(8 * (1 << 28) / ms / 1e6, 1)
    n = 1 << 28
    ms, _ = api.probe("gather", M, n, reps=5)
    out["llc_gather_per_s"] = round(n / ms * 1e3)
    n = 1 << 26
    ms, _ = api.probe("atomic", M, n, reps=5)
    out["global_atomic_per_s"] = round(n / ms * 1e3)
    n = 1 << 28
    ms, _ = api.probe("lds_atomic", 0, n, reps=5)
    out["lds_atomic_per_s"] = round(n / ms * 1e3)
    torch_sync(dev)
    return out


def torch_sync(dev):
    import torch
    torch.cuda.synchronize(dev)


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    if args.warmstart:
        warmstart_experiment(args)
        return
    if args.cnn_timing:
        cnn_timing(args)
        return
    if args.block_study:
        block_study(args)
        return
    if args.tvs_study:
        tvs_study(args)
        return
    import numpy as np
    import torch

    import synth
    from paper_1707_05014_amd import _lib, api

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    _lib.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    cfg = synth.config(args.config, n=args.n)
    fused = args.fused or cfg.rows == "fused"
    N = cfg.n
    S = cfg.sweeps
    g = cfg.grid
    M = g.M
    # inputs resident in HBM: histories made by the device generator
    torch.cuda.synchronize()
    t0 = time.time()
    H = api.Histories(synth.generate_gpu(cfg, device=dev))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    log(f"generated {N} histories on the device in {gen_s:.1f} s")
    points = path_points(H.t, cfg)
    order_np = synth.block_order(N, cfg.perm_seed)
    mask_np = synth.hull_mask(cfg)
    labels_np = synth.roi_labels(cfg)
    true_rsp = synth.insert_rsp(cfg)

    b = cfg.phantom.body
    poly = synth.prior_poly(cfg.beam.E_kin)
    grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz), poly,
                         path_fp32=args.path_fp32)
    order = torch.from_numpy(order_np).to(dev)
    del order_np
    mask = torch.from_numpy(mask_np).to(dev)
    labels = torch.from_numpy(labels_np).to(dev)
    x0 = mask.to(torch.float32)
    x = x0.clone()
    len_dtype = 1 if cfg.rows == "f16" else 0
    params = api.sweep_params("drop", cfg.block, cfg.lam, S, order=order, hull_mask=mask)

    rows = None
    plan = None
    nnz_est = None
    if fused:
        # entries per history, from a traced sample (the fused sweep never stores rows)
        ns = min(N, 1_000_000)
        Hs = api.Histories({k: v[:ns] for k, v in H.t.items()})
        rs = api.mlp_trace(grid, geom, Hs)
        torch.cuda.synchronize()
        nnz_est = rs.nnz / ns * N
        log(f"fused: ~{rs.nnz / ns:.1f} row entries per history (first {ns} histories)")
        del Hs, rs
        api._ws_cache.clear()
    else:
        rows = api.mlp_trace(grid, geom, H, len_dtype=len_dtype)  # sizing + allocation
        torch.cuda.synchronize()
        log(f"rows: nnz {rows.nnz} ({rows.nnz / N:.1f} per history), "
            f"{(rows.idx.numel() * 4 + rows.len.numel() * rows.len.element_size()) / 1e9:.2f} GB")
        if not args.no_plan:
            plan = api.plan_build(grid, H, rows, params)  # sizing + allocation
            torch.cuda.synchronize()
            ps = plan.struct
            log(f"plan: {ps.entries} entries, {ps.chunks} chunks, {ps.refs} reference slots reserved, "
                f"{ps.bytes / 1e9:.2f} GB")

    # One step = one whole reconstruction from device-resident histories:
    # rebuilt rows: path set-up + S sweeps (the first one counting, the later
    # ones reading the kept counts); cached rows: trace, plan build, S sweeps
    # and the FP64 residual after every sweep.
    def step():
        x.copy_(x0)
        return api.reconstruct(grid, geom, H, params, x, rows=rows, plan=plan, want_residuals=not fused)

    # a plain copy of known size: the reference for the FETCH/WRITE counters
    src = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for k in range(args.steps):
        res = step()
        if fused:
            log(f"step {k + 1} of {args.steps} done")
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    value = N * S / (ms_per_step / 1e3)
    log(f"step {ms_per_step:.1f} ms -> {value:.3e} histories/s per sweep; residuals {res}")

    # per-kernel device times of one step (events on the launching stream)
    api.profile_enable(True)
    step()
    torch.cuda.synchronize()
    prof = api.profile_read()
    api.profile_enable(False)
    log("kernel classes (launches, ms): " + json.dumps(prof))
    residual_ms = None
    if fused:
        # the FP64 residual ||Ax - b|| of the final image (one more path pass)
        api.profile_enable(True)
        resid_final = api.residual(grid, geom, H, None, x)
        torch.cuda.synchronize()
        residual_ms = api.profile_read()["residual"][1]
        api.profile_enable(False)
        log(f"residual after {S} sweeps: {resid_final:.6g} ({residual_ms:.1f} ms)")

    variants = None
    if fused and not args.path_fp32 and not args.skip_variants:
        # the reduced-precision form (FP32 path positions and walk, the
        # the benchmark spec's MLP precision): one warm-up and one timed step
        geom32 = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz),
                               poly, path_fp32=True)

        def step32():
            x.copy_(x0)
            api.reconstruct(grid, geom32, H, params, x, want_residuals=False)

        step32()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step32()
        torch.cuda.synchronize()
        ms32 = (time.perf_counter() - t0) * 1e3
        variants = {"path_fp32": {"ms_per_step": round(ms32, 3), "value": round(N * S / (ms32 / 1e3), 1)}}
        log(f"FP32 path positions: step {ms32:.1f} ms -> {N * S / (ms32 / 1e3):.3e} histories/s per sweep")

    peaks = probe_peaks(dev)
    log(f"probes: {peaks}")

    nnz = rows.nnz if rows is not None else None
    n_blocks = (N + cfg.block - 1) // cfg.block
    lb = 4 if len_dtype == 0 else 2
    kpath = "float" if args.path_fp32 else "double"
    # work models per launch (stated in the design doc): HBM bytes or FP64 flops
    models = {"trace": ("alu", PATH_FLOPS_PER_POINT * points, FP64_PEAK_TFLOPS, "TFLOP/s",
                        f"pct::k_trace_stage<{kpath}>")}
    if plan is not None:
        ps = plan.struct
        lbp = 4 if ps.len_dtype == 0 else 2
        # algorithmic bytes per launch (one block): the dot streams the block's
        # list entries (2 B code + length), 8 B per chunk (first piece-end
        # ordinal), reads each piece end's row slot and writes its partial
        # (4 + 4 B) and reads x once (4 B/voxel); the scatter streams the same
        # entries, 16 B per chunk (piece-end mask + first ordinal), reads the
        # row of each piece end (4 B) and r of each row (4 B), and reads and
        # writes x (8 B/voxel)
        ends_pb = ps.ends / n_blocks
        models["plan_dot"] = ("hbm", ((2 + lbp) * ps.entries + 8 * ps.chunks) / n_blocks + 8 * ends_pb + 4 * M,
                              HBM_PEAK_GBS, "GB/s", "pct::k_plan_dot<1, false>" if lbp == 2 else "pct::k_plan_dot<0, false>")
        models["plan_scatter"] = ("hbm", ((2 + lbp) * ps.entries + 16 * ps.chunks) / n_blocks + 4 * ends_pb
                                  + 4 * cfg.block + 8 * M, HBM_PEAK_GBS, "GB/s",
                                  "pct::k_plan_scatter<1>" if lbp == 2 else "pct::k_plan_scatter<0>")
    if rows is not None and plan is None:
        models["project"] = ("hbm", ((4 + lb) * nnz + (16 + 8 + 8 + 4) * N) / n_blocks + 20 * M, HBM_PEAK_GBS,
                             "GB/s", "pct::k_project_cached<0>")
    fused_bounds = None
    if fused:
        # rows rebuilt in every block: the path work of the block's histories.
        # The project class holds the sweeps that read the kept block counts
        # (one atomic per entry), project_counting the first sweep (two).
        models["project"] = ("alu", PATH_FLOPS_PER_POINT * points / n_blocks, FP64_PEAK_TFLOPS, "TFLOP/s",
                             f"pct::k_project_fused<{kpath}, 0>")
        # the three resources the rebuilt-row projection can be bound by (per
        # launch, one block): FP64 path arithmetic against the vector peak,
        # x gathered from the last-level cache (4 B per entry) and one global
        # FP32 atomic per entry, each against the measured path-like rate of
        # the same access pattern (pct_probe)
        e_blk = nnz_est / n_blocks
        launches_p, ms_p = prof["project"]
        t_launch = ms_p / max(launches_p, 1) / 1e3
        t_alu = PATH_FLOPS_PER_POINT * points / n_blocks / (FP64_PEAK_TFLOPS * 1e12)
        t_llc = e_blk / peaks["llc_gather_per_s"]
        t_atom = e_blk / peaks["global_atomic_per_s"]
        fused_bounds = {"alu_ms": round(t_alu * 1e3, 4), "llc_gather_ms": round(t_llc * 1e3, 4),
                        "atomic_ms": round(t_atom * 1e3, 4), "achieved_ms": round(t_launch * 1e3, 4),
                        "entries_per_launch": round(e_blk)}
    timing = dict(prof)
    timing["trace"] = prof["trace_path"]
    dom = max((k for k in models if timing.get(k, (0, 0.0))[0]), key=lambda k: timing[k][1])
    launches, tot_ms = timing[dom]
    bound, work, peak, unit, kname = models[dom]
    if dom == "trace":
        work = work / launches  # the path pass runs in chunks of rows: work per launch
    avg_ms = tot_ms / launches
    achieved = work / (avg_ms / 1e3) / (1e9 if unit == "GB/s" else 1e12)
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_fused_head2e8.json" if fused else "traffic_plan_head10M.json")
    if os.path.exists(tpath):
        tj = json.load(open(tpath))
        kk = tj.get("kernels", {}).get(kname)
        if tj.get("source_hash") == source_hash() and kk and kk.get("write_kib_per_dispatch") is not None:
            traffic = round((kk["fetch_kib_per_dispatch"] / tj["fetch_scale"]
                             + kk["write_kib_per_dispatch"] / tj["write_scale"]) * 1024)
    roofline = {"kernel": kname, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic, "avg_launch_ms": round(avg_ms, 4),
                "work_per_launch": int(work), "work_unit": "bytes" if unit == "GB/s" else "FP64 flops"}
    if fused_bounds is not None:
        # The rebuilt-row projection's bound is the largest of its three
        # resource times (path arithmetic, cache gathers, atomics); the
        # roofline is reported against that resource, its peak measured on
        # this device with the same access pattern (pct_probe), the FP64 flop
        # model kept under "resources".
        tb = max(fused_bounds["alu_ms"], fused_bounds["llc_gather_ms"], fused_bounds["atomic_ms"])
        binding = max(("alu", "llc_gather", "atomic"), key=lambda k: fused_bounds[k + "_ms"])
        fused_bounds["binding"] = binding
        fused_bounds["frac_of_bound"] = round(tb / fused_bounds["achieved_ms"], 4)
        fused_bounds["alu_tflops"] = roofline["achieved"]
        e_s = fused_bounds["entries_per_launch"] / (avg_ms / 1e3)
        if binding == "atomic":
            roofline.update({"bound": "atomic", "achieved": round(e_s), "peak": peaks["global_atomic_per_s"],
                             "unit": "FP32 atomic adds/s", "frac": round(e_s / peaks["global_atomic_per_s"], 4),
                             "work_per_launch": fused_bounds["entries_per_launch"], "work_unit": "atomic adds",
                             "peak_source": "pct_probe atomic (brick-order path-like runs), this device"})
        elif binding == "llc_gather":
            roofline.update({"bound": "llc", "achieved": round(e_s), "peak": peaks["llc_gather_per_s"],
                             "unit": "4-byte gathers/s", "frac": round(e_s / peaks["llc_gather_per_s"], 4),
                             "work_per_launch": fused_bounds["entries_per_launch"], "work_unit": "gathers",
                             "peak_source": "pct_probe gather (brick-order path-like runs), this device"})
        roofline["resources"] = fused_bounds
    # the plan_dot class holds the sweeps' dot launches (one block each); the
    # residual's dot pass over every block is counted in the residual class
    dot_sweep_ms = prof["plan_dot"][1]
    # the per-proton path set-up (hull, end states) runs once per call: with
    # cached rows before the trace, in the fused form before the first sweep
    # (one record per history, read by every later path pass)
    setup_ms = prof["path_setup"][1]
    sweep_ms = (prof["project"][1] + prof["project_counting"][1] + prof["apply"][1] + dot_sweep_ms
                + prof["plan_rows"][1] + prof["plan_scatter"][1] + prof["other"][1]) / S
    if residual_ms is None:
        residual_ms = prof["residual"][1] / max(S, 1)
    trace_ms = prof["trace_path"][1] + prof["trace_compact"][1] + setup_ms
    plan_ms = prof["plan_build"][1]
    others = {k: {"achieved": round(models[k][1] / (timing[k][0] if k == "trace" else 1)
                                    / (timing[k][1] / timing[k][0] / 1e3)
                                    / (1e9 if models[k][3] == "GB/s" else 1e12), 3),
                  "unit": models[k][3], "avg_launch_ms": round(timing[k][1] / timing[k][0], 4)}
              for k in models if timing.get(k, (0, 0.0))[0]}

    # time to <= 1% RSP error (plain sweeps from the hull start); rebuilt
    # rows: checked after every tenth of a sweep
    acc = None
    if not args.skip_accuracy:
        x.copy_(x0)
        errs = []
        hit = None
        if fused:
            t_setup = setup_ms / 1e3
            t_block = sweep_ms / 1e3 / n_blocks
            chunk = max(1, n_blocks // 10)
            # the block order made contiguous, so that a stretch of it is a
            # plain slice swept in blocks of the same size
            Hp = H.permuted(order)
            p1 = api.sweep_params("drop", cfg.block, cfg.lam, 1, hull_mask=mask)
            done = 0
            for s_ in range(args.max_sweeps_acc):
                for b0 in range(0, n_blocks, chunk):
                    nb = min(chunk, n_blocks - b0)
                    sub = api.Histories({k: v[b0 * cfg.block:min(N, (b0 + nb) * cfg.block)] for k, v in Hp.t.items()})
                    api.project_sweep(grid, geom, sub, None, x, p1)
                    done += nb
                    sums, cnts = api.roi_stats(x, labels, len(true_rsp))
                    means = (sums / cnts.clamp(min=1)).cpu().numpy()
                    err = float(np.max(np.abs(means - true_rsp) / true_rsp))
                    errs.append(err)
                    if err <= 0.01:
                        hit = done / n_blocks
                        break
                if hit is not None:
                    break
            del Hp, sub
            acc = {"sweeps_to_1pct": round(hit, 2) if hit else None,
                   "time_to_1pct_s": round(t_setup + hit * n_blocks * t_block, 4) if hit else None,
                   "rsp_err_per_tenth_sweep": [round(e, 5) for e in errs[:12]],
                   "checked": "after every tenth of a sweep; time = path set-up + that share of a sweep at the "
                              "timed step's average rate"}
        else:
            p1 = api.sweep_params("drop", cfg.block, cfg.lam, 1, order=order, hull_mask=mask)
            for s_ in range(1, args.max_sweeps_acc + 1):
                if plan is not None:
                    api.plan_sweep(grid, plan, x, p1)
                else:
                    api.project_sweep(grid, geom, H, rows, x, p1)
                sums, cnts = api.roi_stats(x, labels, len(true_rsp))
                means = (sums / cnts.clamp(min=1)).cpu().numpy()
                err = float(np.max(np.abs(means - true_rsp) / true_rsp))
                errs.append(err)
                if err <= 0.01 and hit is None:
                    hit = s_
                    break
            # trace + plan build + the sweeps needed (device time of the timed step's kernels)
            acc = {"sweeps_to_1pct": hit,
                   "time_to_1pct_s": round((trace_ms + plan_ms + hit * sweep_ms) / 1e3, 4) if hit else None,
                   "rsp_err_after_sweeps": [round(e, 5) for e in errs[: min(len(errs), 12)]],
                   "rsp_err_after_config_sweeps": round(errs[S - 1], 5) if len(errs) >= S else None}
        log(f"accuracy: {acc}")

    cpu = None
    if not args.skip_cpu:
        n_cpu = args.cpu_sample if args.cpu_sample else (2_000_000 if fused else 3_000_000)
        cpu = cpu_baseline(cfg, n_cpu, fused)
        log(f"cpu baseline: {cpu}")

    rows_kind = "fused" if fused else cfg.rows
    out = {
        "metric": "proton histories/s per sweep",
        "value": round(value, 1),
        "unit": "histories/s/sweep",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if rows_kind == "f16" else "f32",
        "data": "synthetic (seeded phantom + Fermi-Eyges transport, made on the device)",
        "config": {
            "workload": f"config {cfg.key}: {N} histories, {g.nx}x{g.ny}x{g.nz} voxels of {g.dx} mm, "
                        f"{cfg.beam.n_angles} angles, {S} DROP sweeps, blocks of {cfg.block}, lambda {cfg.lam}, "
                        + ("rows recomputed every sweep" if fused else f"rows cached ({cfg.rows})")
                        + ("" if (fused or args.no_plan) else ", tiled sweep plan"),
            "histories": N, "voxels": M, "sweeps": S, "block": cfg.block,
            "rows": rows_kind, "path_positions": "f32" if args.path_fp32 else "f64",
            "step": "one whole reconstruction: " + (
                f"path set-up + {S} sweeps (rows rebuilt in every block), no residual" if fused else
                f"trace + plan build + {S} sweeps + FP64 residual after each"),
            "nnz_per_history": round((nnz if nnz else nnz_est) / N, 2),
            "time_to_image_s": round(ms_per_step / 1e3, 3),
            "trace_ms": round(trace_ms, 3), "plan_ms": round(plan_ms, 3), "sweep_ms": round(sweep_ms, 3),
            "rows_bytes": (int(rows.nnz) * (4 + (4 if rows.len_dtype == 0 else 2)) + 16 * N) if rows is not None else None,
            "plan_bytes": int(plan.struct.bytes) if plan is not None else None,
            "sweep_only_hist_per_s": round(N / (sweep_ms / 1e3), 1) if sweep_ms > 0 else None,
            "residual_ms": round(residual_ms, 3),
            "kernel_ms": {k: [v[0], round(v[1], 3)] for k, v in prof.items()},
            "kernel_rates": others, "path_points": points, "probes": peaks, "variants": variants,
            "accuracy": acc, "gen_s": round(gen_s, 1),
            "paper_context": "2e9 histories in under 10 min on the authors' earlier cluster (Sec. 1); "
                             "Table 1: 2.107e9 histories in 3:32 on 120 x (CPU core + Tesla GPU)",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _roi_errors(x, labels, true_rsp, api):
    """(max relative error of the ROI means, mean of the ROI standard
    deviations / true RSP): the ROI analysis of Sec. 3.2 / 4.2; the means
    from pct_roi_stats, the spread (noise) as a torch reduction for the
    report."""
    import numpy as np
    import torch
    sums, cnts = api.roi_stats(x, labels, len(true_rsp))
    means = (sums / cnts.clamp(min=1)).cpu().numpy()
    err = float(np.max(np.abs(means - true_rsp) / true_rsp))
    lab = labels.to(torch.int64)
    xd = x.to(torch.float64)
    sq = torch.zeros(len(true_rsp) + 1, dtype=torch.float64, device=x.device).index_add_(0, lab, xd * xd)[1:]
    var = (sq.cpu().numpy() / np.maximum(cnts.cpu().numpy(), 1)) - means ** 2
    noise = float(np.mean(np.sqrt(np.maximum(var, 0.0)) / true_rsp))
    return err, noise


def block_study(args):
    """Sec. 2.1 leaves the number of blocks to the user: RSP error after each
    sweep and device time per sweep for several block sizes, on the 1e7-
    history workload (config 2 data, rows rebuilt in every block so that
    every block size runs the same kernels; the counts are formed with
    atomics in every sweep).  Prints one JSON line."""
    import torch

    import synth
    from paper_1707_05014_amd import _lib, api

    _lib.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = synth.config(2, n=args.n)
    N, g, b = cfg.n, cfg.grid, cfg.phantom.body
    H = api.Histories(synth.generate_gpu(cfg, device=dev))
    grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz),
                         synth.prior_poly(cfg.beam.E_kin))
    order = torch.from_numpy(synth.block_order(N, cfg.perm_seed)).to(dev)
    mask = torch.from_numpy(synth.hull_mask(cfg)).to(dev)
    labels = torch.from_numpy(synth.roi_labels(cfg)).to(dev)
    true_rsp = synth.insert_rsp(cfg)
    out = {"metric": "RSP error per sweep by block size", "n_gpus": 1,
           "config": {"workload": f"config 2 data: {N} histories, {g.nx}x{g.ny}x{g.nz} voxels, lambda {cfg.lam}, "
                                  "rows rebuilt in every block"}, "blocks": []}
    for bs in (int(v) for v in args.block_sizes.split(",")):
        p1 = api.sweep_params("drop", bs, cfg.lam, 1, order=order, hull_mask=mask)
        x = mask.to(torch.float32)
        errs, noise, hit = [], [], None
        api.project_sweep(grid, geom, H, None, x.clone(), p1)  # warm-up (workspace, code)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_sweeps = 0.0
        for s_ in range(1, args.max_sweeps_acc + 1):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            api.project_sweep(grid, geom, H, None, x, p1)
            torch.cuda.synchronize()
            t_sweeps += time.perf_counter() - t1
            e, nz = _roi_errors(x, labels, true_rsp, api)
            errs.append(round(e, 5))
            noise.append(round(nz, 5))
            if e <= 0.01 and hit is None:
                hit = s_
            if hit is not None and s_ >= hit + 2:
                break
        ms = t_sweeps / len(errs) * 1e3
        row = {"block": bs, "blocks_per_sweep": -(-N // bs), "ms_per_sweep": round(ms, 2),
               "sweeps_to_1pct": hit, "time_to_1pct_s": round(hit * ms / 1e3, 4) if hit else None,
               "rsp_err_after_sweeps": errs, "roi_noise_after_sweeps": noise}
        log(f"block study: {row}")
        out["blocks"].append(row)
    print(json.dumps(out), flush=True)


def tvs_study(args):
    """TV superiorization before every DROP block (Sec. 4.2) against the
    plain sweeps, on the 1e7-history workload with its tiled plan: RSP
    error, ROI noise (standard deviation in the insert ROIs relative to the
    true RSP) and relative L2 to the phantom inside the hull after each
    sweep.  Prints one JSON line."""
    import numpy as np
    import torch

    import synth
    from paper_1707_05014_amd import _lib, api

    _lib.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = synth.config(2, n=args.n)
    N, g, b = cfg.n, cfg.grid, cfg.phantom.body
    H = api.Histories(synth.generate_gpu(cfg, device=dev))
    grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz),
                         synth.prior_poly(cfg.beam.E_kin))
    order = torch.from_numpy(synth.block_order(N, cfg.perm_seed)).to(dev)
    mask = torch.from_numpy(synth.hull_mask(cfg)).to(dev)
    inside = mask.bool()
    labels = torch.from_numpy(synth.roi_labels(cfg)).to(dev)
    true_rsp = synth.insert_rsp(cfg)
    truth = torch.from_numpy(synth.truth_image(cfg)).to(dev)
    rows = api.mlp_trace(grid, geom, H)
    p0 = api.sweep_params("drop", cfg.block, cfg.lam, 1, order=order, hull_mask=mask)
    plan = api.plan_build(grid, H, rows, p0)
    out = {"metric": "TV superiorization vs plain DROP", "n_gpus": 1,
           "config": {"workload": f"config 2: {N} histories, blocks of {cfg.block}, lambda {cfg.lam}, tiled plan",
                      "tvs": {"beta0": args.tvs_beta0, "n_steps": 1, "max_trials": 3, "a": args.tvs_a,
                              "eps": 1e-3}}, "forms": {}}
    for form in ("plain", "tvs"):
        tv = api.Tvs(beta0=args.tvs_beta0, n_steps=1, max_trials=3, a=args.tvs_a, eps=1e-3) if form == "tvs" else None
        p1 = api.sweep_params("drop", cfg.block, cfg.lam, 1, order=order, hull_mask=mask, tvs=tv)
        x = mask.to(torch.float32)
        errs, noise, l2, ms = [], [], [], 0.0
        for s_ in range(args.max_sweeps_acc):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            api.plan_sweep(grid, plan, x, p1)
            torch.cuda.synchronize()
            ms += (time.perf_counter() - t1) * 1e3
            e, nz = _roi_errors(x, labels, true_rsp, api)
            errs.append(round(e, 5))
            noise.append(round(nz, 5))
            l2.append(round(float(torch.linalg.vector_norm((x - truth)[inside]) /
                                  torch.linalg.vector_norm(truth[inside])), 5))
        hit = next((k + 1 for k, e in enumerate(errs) if e <= 0.01), None)
        out["forms"][form] = {"ms_per_sweep": round(ms / len(errs), 2), "sweeps_to_1pct": hit,
                              "rsp_err_after_sweeps": errs, "roi_noise_after_sweeps": noise,
                              "rel_l2_after_sweeps": l2, "beta_after": tv.beta if tv else None}
        log(f"tvs study {form}: {out['forms'][form]}")
    print(json.dumps(out), flush=True)


def cnn_timing(args):
    """Device time of the warm-start network on one 200 x 200 x 40 volume
    (channels --ws-channels): inference and one training step in FP32 and
    with the bfloat16 matrix-core convolutions, and each convolution shape of
    the network's first three levels (forward, input gradient, weight
    gradient; the first two also on the matrix cores) with its throughput (2
    flops per multiply-add of the 3x3x3 contraction).  Prints one JSON line."""
    import numpy as np
    import torch

    from paper_1707_05014_amd import _lib, cnn

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    _lib.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    D, H, W = 40, 200, 200
    channels = tuple(int(c) for c in args.ws_channels.split(","))
    net = cnn.UNet3D(channels, device=dev, seed=0)
    net16 = cnn.UNet3D(channels, device=dev, seed=0, precision="bf16")
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.uniform(0, 1.8, size=(1, D, H, W)).astype(np.float32)).to(dev)
    t = torch.from_numpy(rng.uniform(0, 1.8, size=(1, D, H, W)).astype(np.float32)).to(dev)

    def ms(fn, n):
        # median over 5 repetitions of n calls, timed with events on the
        # stream: a host-side stall in one repetition does not count
        fn()
        torch.cuda.synchronize()
        reps = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(n):
                fn()
            b.record()
            b.synchronize()
            reps.append(a.elapsed_time(b) / n)
        return sorted(reps)[2]

    out = {"metric": "warm-start network device time", "unit": "ms", "n_gpus": 1, "dtype": "f32",
           "config": {"workload": f"one {W}x{H}x{D} volume, channels {list(channels)}"},
           "inference_ms": round(ms(lambda: net.predict(x), args.steps * 3), 3),
           "train_step_ms": round(ms(lambda: net.train_step(x, t, 1e-4), args.steps * 3), 3),
           "bf16_inference_ms": round(ms(lambda: net16.predict(x), args.steps * 3), 3),
           "bf16_train_step_ms": round(ms(lambda: net16.train_step(x, t, 1e-4), args.steps * 3), 3), "conv": []}
    dims = (D, H, W)
    for lvl, c in enumerate(channels[:3]):
        a = torch.from_numpy(rng.normal(size=(c,) + dims).astype(np.float32)).to(dev)
        w = torch.from_numpy(rng.normal(size=(c, c, 3, 3, 3)).astype(np.float32)).to(dev)
        b = torch.zeros(c, dtype=torch.float32, device=dev)
        y = torch.empty_like(a)
        dx = torch.empty_like(a)
        wt = torch.empty(c * c * 27, dtype=torch.float32, device=dev)
        sc = torch.empty(cnn.wgrad_scratch(c, c, *dims), dtype=torch.float32, device=dev)
        dw, db = torch.empty_like(w), torch.empty_like(b)
        flops = 2.0 * dims[0] * dims[1] * dims[2] * c * c * 27
        f = ms(lambda: cnn.conv3d(a, w, b, y), args.steps * 5)
        bd = ms(lambda: cnn.conv3d_bwd_data(y, w, dx, wt), args.steps * 5)
        bw = ms(lambda: cnn.conv3d_bwd_weight(a, y, dw, db, sc), args.steps * 5)
        wp = torch.empty(max(cnn.bf16_scratch(c, c), 1), dtype=torch.uint8, device=dev)
        rec = {"level": lvl, "shape": f"{c}->{c} on {dims[2]}x{dims[1]}x{dims[0]}",
               "fwd_ms": round(f, 4), "bwd_data_ms": round(bd, 4), "bwd_weight_ms": round(bw, 4),
               "fwd_tflops": round(flops / f / 1e9, 2), "bwd_data_tflops": round(flops / bd / 1e9, 2),
               "bwd_weight_tflops": round(flops / bw / 1e9, 2)}
        if cnn.bf16_scratch(c, c):
            f16 = ms(lambda: cnn.conv3d(a, w, b, y, wpack=wp), args.steps * 5)
            bd16 = ms(lambda: cnn.conv3d_bwd_data(y, w, dx, wt, wpack=wp), args.steps * 5)
            # per launch: x read once (4 B/value) and y written once (4 B/value)
            hbm = 8.0 * c * dims[0] * dims[1] * dims[2]
            rec.update({"bf16_fwd_ms": round(f16, 4), "bf16_bwd_data_ms": round(bd16, 4),
                        "bf16_fwd_tflops": round(flops / f16 / 1e9, 2),
                        "bf16_fwd_frac_of_mfma_peak": round(flops / f16 / 1e9 / 2500.0, 4),
                        "bf16_fwd_hbm_GBps": round(hbm / f16 / 1e6, 1)})
        if cnn.bf16_wgrad_ok(c, c):
            bw16 = ms(lambda: cnn.conv3d_bwd_weight(a, y, dw, db, sc, bf16=True), args.steps * 5)
            rec.update({"bf16_bwd_weight_ms": round(bw16, 4), "bf16_bwd_weight_tflops": round(flops / bw16 / 1e9, 2),
                        "bf16_bwd_weight_frac_of_mfma_peak": round(flops / bw16 / 1e9 / 2500.0, 4)})
        out["conv"].append(rec)
        dims = tuple(d // 2 for d in dims)
    print(json.dumps(out), flush=True)


def warmstart_experiment(args):
    """Time to <= 1% RSP error from the hull start and from the learned warm
    start, on the held-out phantom of the 2e8-history workload (seed 3)
    with --ws-n histories.  The network is trained first on pairs (images
    after the input sweeps, image after --ws-out sweeps) of --ws-train seeded
    phantoms reconstructed the same way (same history count, block size and
    relaxation).  --ws-variants lists networks to train and compare, each as
    "<input sweeps joined by '-'>:<coarse-loss weight>".  Prints one JSON line
    (value: the first variant's time to <= 1%)."""
    import numpy as np
    import torch

    import synth
    from paper_1707_05014_amd import _lib, api, cnn
    from paper_1707_05014_amd import warmstart as wsm

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    _lib.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    N = args.ws_n
    variants = []
    for v in args.ws_variants.split(","):
        f = v.split(":")
        variants.append((tuple(int(q) for q in f[0].split("-")), float(f[1]), f[2] if len(f) > 2 else "out"))
    snaps_needed = sorted({q for ins, _, _ in variants for q in ins} | {args.ws_out})
    last_in = max(q for ins, _, _ in variants for q in ins)
    want_truth = any(tg == "truth" for _, _, tg in variants)
    want_clean = any(tg == "clean" for _, _, tg in variants)
    if any(tg not in ("out", "truth", "clean") for _, _, tg in variants):
        raise SystemExit("--ws-variants: the target is out, truth or clean")

    def setup(cfg):
        g = cfg.grid
        b = cfg.phantom.body
        t0 = time.time()
        H = api.Histories(synth.generate_gpu(cfg, device=dev))
        torch.cuda.synchronize()
        gen_s = time.time() - t0
        grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
        geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz),
                             synth.prior_poly(cfg.beam.E_kin))
        order = torch.from_numpy(synth.block_order(cfg.n, cfg.perm_seed)).to(dev)
        mask = torch.from_numpy(synth.hull_mask(cfg)).to(dev)
        params = api.sweep_params("drop", cfg.block, cfg.lam, 1, order=order, hull_mask=mask)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = api.mlp_trace(grid, geom, H)
        plan = api.plan_build(grid, H, rows, params)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        return dict(grid=grid, H=H, rows=rows, plan=plan, params=params, mask=mask, gen_s=gen_s, setup_s=setup_s)

    # ---- training pairs from the solver on seeded phantoms
    train_snaps = []
    t_data = time.time()
    for i in range(args.ws_train):
        cfg = synth.training_config(1000 + i, N)
        S = setup(cfg)
        x = S["mask"].to(torch.float32)
        train_snaps.append(wsm.sweep_snapshots(S["grid"], S["plan"], x, S["params"], snaps_needed))
        if want_truth:
            train_snaps[-1]["truth"] = torch.from_numpy(synth.truth_image(cfg)).to(dev)
        if want_clean:
            # the solver's own image after --ws-out sweeps of the same protons
            # with the WEPL noise left out: converged, and without noise that
            # no network could predict from its input
            cc = dataclasses.replace(cfg, beam=dataclasses.replace(cfg.beam, wepl_sigma=0.0))
            Sc = setup(cc)
            xc = Sc["mask"].to(torch.float32)
            train_snaps[-1]["clean"] = wsm.sweep_snapshots(Sc["grid"], Sc["plan"], xc, Sc["params"],
                                                           [args.ws_out])[args.ws_out]
            del Sc, xc
        log(f"training phantom {i + 1}/{args.ws_train} (seed {1000 + i}): generated in {S['gen_s']:.1f} s")
        grid_t = S["grid"]
        del S, x
    data_s = time.time() - t_data

    channels = tuple(int(c) for c in args.ws_channels.split(","))
    def mean_loss(net, pairs):
        return float(np.mean([float(net.loss_and_grad(a, b).item()) for a, b in pairs]))

    nets = []
    for ins, wc, tg in variants:
        pairs = [(wsm.net_input(sn, ins, grid_t), wsm.volume(sn[args.ws_out if tg == "out" else tg], grid_t))
                 for sn in train_snaps]
        members, train_s = [], 0.0
        for e in range(max(args.ws_ensemble, 1)):
            net = cnn.UNet3D(channels, device=dev, seed=7 + e, in_channels=len(ins), precision=args.ws_precision)
            loss0 = mean_loss(net, pairs)  # the untrained network is the identity on its last input
            losses, t_e = wsm.train(net, pairs, args.ws_steps, args.ws_lr, seed=11 + e, coarse_weight=wc, log=log)
            loss1 = mean_loss(net, pairs)
            train_s += t_e
            log(f"variant {ins}:{wc}:{tg} (network {e + 1}/{max(args.ws_ensemble, 1)}): trained {args.ws_steps} "
                f"steps in {t_e:.1f} s; mean training loss {loss0:.4e} (identity) -> {loss1:.4e}")
            members.append((loss1, net))
        # a member whose training failed (loss near the identity's) would pull
        # the mean back toward its input: keep the members within 3x of the best
        best = min(l for l, _ in members)
        kept = [m for l, m in members if l <= 3.0 * best]
        if len(kept) < len(members):
            log(f"variant {ins}:{wc}:{tg}: {len(members) - len(kept)} of {len(members)} networks left out "
                f"(training loss above 3x the best)")
        loss1 = best
        nets.append((ins, wc, tg, kept if len(kept) > 1 else kept[0], (loss0, loss1), train_s))
        del pairs
    del train_snaps

    # ---- evaluation on held-out phantoms (the first one: the 2e8 workload's phantom, seed 3)
    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def evaluate(cfg):
        S = setup(cfg)
        grid, plan, params, mask = S["grid"], S["plan"], S["params"], S["mask"]
        labels = torch.from_numpy(synth.roi_labels(cfg)).to(dev)
        true_rsp = synth.insert_rsp(cfg)
        truth = torch.from_numpy(synth.truth_image(cfg)).to(dev)
        inside = mask.bool()

        def rsp_err(x):
            sums, cnts = api.roi_stats(x, labels, len(true_rsp))
            means = (sums / cnts.clamp(min=1)).cpu().numpy()
            return float(np.max(np.abs(means - true_rsp) / true_rsp))

        def rel_l2(x):
            return float(torch.linalg.vector_norm((x - truth)[inside]) / torch.linalg.vector_norm(truth[inside]))

        def sweeps_until(x, max_sweeps, t_start, errs):
            t = t_start
            for s in range(1, max_sweeps + 1):
                _, dt = timed(lambda: api.plan_sweep(grid, plan, x, params))
                t += dt
                errs.append(rsp_err(x))
                if errs[-1] <= 0.01:
                    return s, t
            return None, None

        # hull start, keeping the snapshots the networks read
        x = mask.to(torch.float32)
        e_h = []
        snaps = {}
        t = S["setup_s"]
        hit_h = t_h = None
        t_at = {}
        for s_ in range(1, max(args.max_sweeps_acc, args.ws_out) + 1):
            _, dt = timed(lambda: api.plan_sweep(grid, plan, x, params))
            t += dt
            t_at[s_] = t
            e_h.append(rsp_err(x))
            if s_ in snaps_needed:
                snaps[s_] = x.clone()
            if e_h[-1] <= 0.01 and hit_h is None:
                hit_h, t_h = s_, t
            if hit_h is not None and s_ >= max(last_in, args.ws_out):
                break
        hull = {"sweeps_to_1pct": hit_h, "time_to_1pct_s": round(t_h, 4) if t_h else None,
                "rsp_err_per_sweep": [round(e, 5) for e in e_h],
                "rel_l2_after_sweeps": {k: round(rel_l2(v), 5) for k, v in snaps.items()}}
        res = []
        for ins, wc, tg, net, _, _ in nets:
            inp = wsm.net_input(snaps, ins, grid)
            x0, t_net = timed(lambda: wsm.warm_start(net, inp, mask))
            err_net = rsp_err(x0)
            l2_net = rel_l2(x0)
            t0 = t_at[max(ins)] + t_net
            e_c = []
            if err_net <= 0.01:
                hit_c, t_c = 0, t0
            else:
                hit_c, t_c = sweeps_until(x0, args.max_sweeps_acc, t0, e_c)
            res.append({"net_ms": round(t_net * 1e3, 3), "rsp_err_of_net_output": round(err_net, 5),
                        "rel_l2_of_net_output": round(l2_net, 5), "sweeps_after_net_to_1pct": hit_c,
                        "total_sweeps": (max(ins) + hit_c) if hit_c is not None else None,
                        "time_to_1pct_s": round(t_c, 4) if t_c else None,
                        "rsp_err_per_sweep_after_net": [round(e, 5) for e in e_c]})
        del S
        return hull, res

    eval_seeds = [int(q) for q in args.ws_eval_seeds.split(",")]
    per_phantom = []
    for k, seed in enumerate(eval_seeds):
        cfg = synth.config(5, n=N) if seed == 3 else synth.training_config(seed, N)
        hull, res = evaluate(cfg)
        per_phantom.append({"phantom_seed": seed, "hull_start": hull, "warm_start": res})
        log(f"held-out phantom {seed}: hull {hull['sweeps_to_1pct']} sweeps; networks "
            f"{[r['total_sweeps'] for r in res]} sweeps, output RSP errors {[r['rsp_err_of_net_output'] for r in res]}")

    def tot(xs):
        return None if any(v is None for v in xs) else round(sum(xs), 4)

    hull_t = tot([p["hull_start"]["time_to_1pct_s"] for p in per_phantom])
    summary = []
    for j, (ins, wc, tg, net, (loss0, loss1), train_s) in enumerate(nets):
        tj = tot([p["warm_start"][j]["time_to_1pct_s"] for p in per_phantom])
        summary.append({"inputs_after_sweeps": list(ins), "coarse_loss_weight": wc, "target": tg,
                        "total_sweeps_per_phantom": [p["warm_start"][j]["total_sweeps"] for p in per_phantom],
                        "time_to_1pct_s_total": tj,
                        "speedup_vs_hull_start": round(hull_t / tj, 3) if (hull_t and tj) else None,
                        "rel_l2_of_net_output_per_phantom": [p["warm_start"][j]["rel_l2_of_net_output"]
                                                             for p in per_phantom],
                        "ensemble_members_kept": len(net) if isinstance(net, list) else 1,
                        "train_s": round(train_s, 1),
                        "train_ms_per_step": round(train_s * 1e3 / max(args.ws_steps * max(args.ws_ensemble, 1), 1), 2),
                        "train_loss_identity": loss0, "train_loss_trained": loss1})
    out = {
        "metric": "time to <= 1% RSP error (learned warm start vs hull start)",
        "value": per_phantom[0]["warm_start"][0]["time_to_1pct_s"], "unit": "s", "n_gpus": 1,
        "higher_is_better": False,
        "hull_start_value": per_phantom[0]["hull_start"]["time_to_1pct_s"],
        "dtype": "f32", "data": "synthetic (seeded phantoms + Fermi-Eyges transport)",
        "config": {"workload": f"held-out head phantoms (seeds {eval_seeds}; value: seed 3), {N} histories each, "
                               f"200x200x40 voxels of 1 mm, DROP blocks of 200000, lambda 0.5, rows cached (f32), "
                               f"tiled sweep plan",
                   "network": {"channels": list(channels), "train_phantoms": args.ws_train,
                               "train_steps": args.ws_steps, "lr": args.ws_lr, "target_sweeps": args.ws_out,
                               "ensemble": max(args.ws_ensemble, 1),
                               "precision": args.ws_precision}},
        "training_data_s": round(data_s, 1),
        "hull_start_sweeps_per_phantom": [p["hull_start"]["sweeps_to_1pct"] for p in per_phantom],
        "hull_start_time_to_1pct_s_total": hull_t,
        "variants": summary, "per_phantom": per_phantom,
    }
    if args.ws_eval_2e8:
        out["config3"] = warmstart_at_scale(args, nets, N)
    print(json.dumps(out), flush=True)


def warmstart_at_scale(args, nets, n_train):
    """The 2e8-history workload (phantom seed 3, rows rebuilt in every block)
    from the hull start and from the warm start.  The first n_train histories
    of the block order form the same number of blocks of the same size as one
    whole sweep of a training phantom, so the network that reads the image
    after one sweep reads the image after that first stretch here.  RSP error
    checked after every tenth of a sweep (and at the network's output); time
    = device time of the sweeps, the path set-up and the network."""
    import numpy as np
    import torch

    import synth
    from paper_1707_05014_amd import api
    from paper_1707_05014_amd import warmstart as wsm

    pick = [k for k, nt in enumerate(nets) if tuple(nt[0]) == (1,)]
    if not pick:
        return {"skipped": "no network reads the image after one sweep"}
    net = nets[pick[0]][3]
    dev = torch.device("cuda", 0)
    cfg = synth.config(3)
    N = cfg.n
    g = cfg.grid
    b = cfg.phantom.body
    t0 = time.time()
    H = api.Histories(synth.generate_gpu(cfg, device=dev))
    torch.cuda.synchronize()
    log(f"config 3: generated {N} histories on the device in {time.time() - t0:.1f} s")
    grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz),
                         synth.prior_poly(cfg.beam.E_kin))
    order = torch.from_numpy(synth.block_order(N, cfg.perm_seed)).to(dev)
    Hp = H.permuted(order)  # block order made contiguous: stretches of it are plain slices
    del H, order
    mask = torch.from_numpy(synth.hull_mask(cfg)).to(dev)
    labels = torch.from_numpy(synth.roi_labels(cfg)).to(dev)
    true_rsp = synth.insert_rsp(cfg)
    params = api.sweep_params("drop", cfg.block, cfg.lam, 1, hull_mask=mask)
    tenth = N // 10

    def rsp_err(x):
        sums, cnts = api.roi_stats(x, labels, len(true_rsp))
        means = (sums / cnts.clamp(min=1)).cpu().numpy()
        return float(np.max(np.abs(means - true_rsp) / true_rsp))

    def stretch(x, a, b_):
        sub = api.Histories({k: v[a:b_] for k, v in Hp.t.items()})
        torch.cuda.synchronize()
        t = time.perf_counter()
        api.project_sweep(grid, geom, sub, None, x, params)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def run(x, start, t_start, errs, max_tenths=20):
        t = t_start
        pos = start
        for k in range(max_tenths):
            a = pos % N
            b_ = min(a + tenth - (a % tenth), N)  # to the next tenth of the sweep
            t += stretch(x, a, b_)
            pos += b_ - a
            errs.append([round(pos / N, 3), round(rsp_err(x), 5)])
            if errs[-1][1] <= 0.01:
                return pos / N, t
        return None, None

    x = mask.to(torch.float32)
    e_h = []
    f_h, t_h = run(x, 0, 0.0, e_h)
    x = mask.to(torch.float32)
    t_in = stretch(x, 0, n_train)
    e_in = rsp_err(x)
    snaps = {1: x}
    inp = wsm.net_input(snaps, (1,), grid)
    torch.cuda.synchronize()
    t = time.perf_counter()
    x0 = wsm.warm_start(net, inp, mask)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t
    e_net = rsp_err(x0)
    e_w = []
    if e_net <= 0.01:
        f_w, t_w = n_train / N, t_in + t_net
    else:
        f_w, t_w = run(x0, n_train, t_in + t_net, e_w)
    res = {"workload": f"config 3: {N} histories, phantom seed 3, blocks of {cfg.block}, rows rebuilt in every block",
           "hull_start": {"sweeps_to_1pct": f_h, "time_to_1pct_s": round(t_h, 4) if t_h else None,
                          "rsp_err_by_sweep_fraction": e_h},
           "warm_start": {"histories_before_net": n_train, "rsp_err_before_net": round(e_in, 5),
                          "net_ms": round(t_net * 1e3, 3), "rsp_err_of_net_output": round(e_net, 5),
                          "sweeps_to_1pct": f_w, "time_to_1pct_s": round(t_w, 4) if t_w else None,
                          "rsp_err_by_sweep_fraction": e_w},
           "speedup_vs_hull_start": round(t_h / t_w, 3) if (t_h and t_w) else None}
    log(f"config 3 warm start: {res}")
    return res


def cpu_baseline(cfg, n_sample, fused=False):
    """The FP64 oracle on the first n_sample histories of the same workload,
    on the host threads this job may use: rows traced once and the
    configured number of DROP sweeps in the same block size (cached rows),
    or every block's rows traced afresh in every sweep (rows rebuilt)."""
    import numpy as np

    import oracle
    import synth
    n_sample = min(n_sample, cfg.n)
    threads = oracle._threads(None)
    h = synth.generate(cfg, n=n_sample)
    g = cfg.grid
    b = cfg.phantom.body
    G = oracle.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geo = oracle.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1, min(g.dx, g.dy, g.dz),
                           synth.prior_poly(cfg.beam.E_kin))
    order = synth.block_order(n_sample, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    info = host_info()
    if fused:
        sweeps = 2
        t0 = time.perf_counter()
        oracle.drop_recompute(G, geo, h, mask.astype(np.float64), order, cfg.block, cfg.lam, sweeps, mask=mask,
                              threads=threads)
        t2 = time.perf_counter()
        sample = (f"first {n_sample} histories of the workload: FP64 DROP with every block's rows traced afresh, "
                  f"{sweeps} sweeps with per-sweep residual ({t2 - t0:.1f} s)")
        value = n_sample * sweeps / (t2 - t0)
    else:
        t0 = time.perf_counter()
        R = oracle.trace(G, geo, h, threads=threads)
        t1 = time.perf_counter()
        oracle.drop(R, h["wepl"], mask.astype(np.float64), order, cfg.block, cfg.lam, cfg.sweeps, mask=mask,
                    threads=threads)
        t2 = time.perf_counter()
        sample = (f"first {n_sample} histories of the workload: FP64 trace ({t1 - t0:.1f} s) + "
                  f"{cfg.sweeps} DROP sweeps with per-sweep residual ({t2 - t1:.1f} s)")
        value = n_sample * cfg.sweeps / (t2 - t0)
    return {"value": round(value, 1), "unit": "histories/s/sweep", "cores": threads, "kind": "oracle",
            "sample": sample, "host": info}


if __name__ == "__main__":
    main()

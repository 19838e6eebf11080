"""Benchmark: corrected GPix/s of the whole correction path on one MI355X.

One step = one frame-set through every step of the path: band statistics,
estimate, tables, apply with fused whole-frame statistics.  By default steps
go through rt_pipe with several apply lanes (the statistics and estimates of
consecutive frame-sets run in order on one stream, ahead of the applies,
which go over LANES streams, so that consecutive applies overlap; with
--fuse 1 a group's applies are one launch and groups take the lanes in
turn); --lanes 1 keeps every apply on the caller's stream, --mode eager
issues one rt_frameset per step on one stream, --mode graph /
graph-pipelined replay captured HIP graphs (the frames rebound before each
launch, so one graph, or two for alternating tables, serves every buffer),
--mode ahead issues one rt_frameset_ahead launch per step (the apply of a
frame-set beside the estimate of the next).
Inputs are seeded synthetic rigs already resident in HBM; NBUF distinct
input/output frame-set buffers rotate so that the 256 MB Infinity Cache
cannot serve repeats.

    python bench.py [--gpus 1] [--steps 300] [--warmup 20] [--config rig14]

Prints ONE JSON line.  In the pipe mode the launch knobs (apply lanes, group
size, fused or not, segment height, apply grid) come from the autotuner, timed in that
mode on the benchmark rig before the timed region unless cached or given on
the command line ("tuned" says which).  After the timed region, further
legs add their own objects to the line: "removal" (object removal with the
smoothing fallback, eager, and the seam-cost monitor), "surrogate" (the
network trained on the device from the plain estimator, then its inference
path against the plain one), "serving" (three rigs behind the server,
paced at 30 fps and saturated), "uneven" (the three-ring rig of mixed
sizes in the same launch mode) and "moving_object" (the methods compared
around a vehicle that crosses a seam, 16 and 64 blocks).
The roofline figure is for the dominant kernel (the apply pass with fused
statistics), timed by HIP events the library attaches to its dispatches in
the timed region (every n-th), next to the streaming-copy ceiling of the
same bytes; with overlapping apply lanes it also gives the apply bytes per
frame-set over the time per frame-set ("per_step") and the same launches
back to back on one stream after the timed region ("alone").  The CPU
baseline leg times the CPU oracle (test infrastructure) on a bounded sample
of the same workload.
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

HBM_PEAK_GBS = 8000.0
METRIC = "corrected GPix/s and % HBM roofline; p50/p99 frame-set latency, plain vs surrogate"
KERNEL_SOURCES = ["dev_common.h", "dev_apply.h", "dev_estimate.h", "k_apply.hip", "rt_internal.h"]
# Counter-derived HBM traffic of each form of the dominant kernel.
TRAFFIC_FILES = {"k_apply_sets<false>": os.path.join(ROOT, "profiles", "k_apply_sets_rig14_traffic.txt"),
                 "k_apply<true,true,false>": os.path.join(ROOT, "profiles", "k_apply_rig14_traffic.txt")}


def log(msg: str) -> None:
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the apply kernel's sources without comments and blank lines (a
    comment edit does not make the stored traffic measurement stale)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_03517_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def config(name: str):
    """Rig of a workload name (rig14, uneven, vga)."""
    from paper_1910_03517_amd import synth
    if name == "rig14":
        return synth.rig14_1080p()
    if name == "uneven":
        return synth.uneven_rig()
    if name == "vga":
        return synth.single_vga()
    raise ValueError(f"unknown config {name}")


def algorithmic_bytes(cams, band_width: int) -> int:
    """Bytes one frame-set must move: every sample read and written once, plus
    the two border bands of every row read once more for the statistics."""
    total = 0
    for c in cams:
        bps = 1 if c.bit_depth == 8 else 2
        frame = c.width * c.height * c.channels * bps
        band = min(band_width, c.width // 2)
        total += 2 * frame + 2 * band * c.height * c.channels * bps
    return total


def traffic_from_profile(khash: str, workload: str, kernel: str):
    """Counter-derived HBM bytes per frame-set of the apply kernel from the
    committed rocprofv3 summary, if it was taken on this exact kernel source,
    kernel form and workload; else None."""
    if kernel not in TRAFFIC_FILES:
        return None
    try:
        with open(TRAFFIC_FILES[kernel]) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_hash") != khash or kv.get("workload") != workload or kv.get("kernel") != kernel:
        return None
    try:
        return float(kv["hbm_bytes_per_frameset"])
    except (KeyError, ValueError):
        return None


def oracle_setup(rig, smoothing: bool):
    from oracle import ringcorr as rc
    cams = [rc.Camera(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos) for c in rig.cams]
    return rc, cams, rc.Options(smoothing=smoothing)


def cpu_baseline(rig, smoothing: bool, budget_s: float = 10.0) -> dict:
    """The oracle as it stands, single process, on whole frame-sets of the same workload."""
    from paper_1910_03517_amd import synth
    rc, cams, opts = oracle_setup(rig, smoothing)
    frames = synth.rig_frames(rig, 0)
    px = sum(c.width * c.height for c in cams)
    n, t_total = 0, 0.0
    prev_p = prev_v = None
    while t_total < budget_s or n == 0:
        t0 = time.perf_counter()
        r = rc.frameset(cams, opts, frames, prev_p, prev_v)
        t_total += time.perf_counter() - t0
        prev_p, prev_v = r["params"], r["valid"]
        n += 1
    return {"value": round(px * n / t_total / 1e9, 6), "unit": "GPix/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} whole frame-sets of {rig.name} ({px * n / 1e6:.1f} MPix) through the numpy oracle, "
                      f"{t_total:.1f} s single process"}


# Worker state of the process-pool baseline (each worker process builds the
# same seeded frame-set once, outside the timed loop).
_POOL = {}


def _pool_init(config_name: str, smoothing: bool) -> None:
    # A failing initializer would make the pool start workers over and over:
    # keep the error and let every task raise it instead.
    try:
        from paper_1910_03517_amd import synth
        rig = config(config_name)
        rc, cams, opts = oracle_setup(rig, smoothing)
        _POOL.update(rc=rc, cams=cams, opts=opts, frames=synth.rig_frames(rig, 0))
    except BaseException as e:  # noqa: BLE001 - reported by the first task
        _POOL["error"] = repr(e)


def _pool_stats(k: int):
    if "error" in _POOL:
        raise RuntimeError("pool worker set-up failed: " + _POOL["error"])
    rc, cam, f = _POOL["rc"], _POOL["cams"][k], _POOL["frames"][k]
    bh, bs = rc.band_stats(f, cam, _POOL["opts"])
    wh, ws = rc.whole_stats(f, cam)
    return bh, bs, wh, ws


def _pool_apply(args):
    k, params_k = args
    rc, cam, opts = _POOL["rc"], _POOL["cams"][k], _POOL["opts"]
    lut8, qq = rc.build_luts([cam], opts, params_k[None])
    out = rc.apply_camera(_POOL["frames"][k], cam, opts, lut8[0], qq[0])
    return int(out[::97, ::89].sum())     # the corrected frame stays in the worker


def cpu_baseline_pool(config_name: str, smoothing: bool, budget_s: float = 10.0) -> dict:
    """The same oracle functions over a process pool, one task per camera:
    statistics of every camera, the estimate in the parent, then tables and
    apply of every camera.  Workers = the host cores this process may use
    (at most 16, the host share of one GPU)."""
    import multiprocessing as mp
    rig = config(config_name)
    rc, cams, opts = oracle_setup(rig, smoothing)
    K = len(cams)
    workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    px = sum(c.width * c.height for c in cams)
    ctx = mp.get_context("spawn")   # fresh interpreters: nothing of this process's device state is inherited
    with ctx.Pool(workers, initializer=_pool_init, initargs=(config_name, smoothing)) as pool:
        pool.map(_pool_stats, range(K))          # every worker initialised before timing
        n, t_total = 0, 0.0
        prev_p = prev_v = None
        while t_total < budget_s or n == 0:
            t0 = time.perf_counter()
            st = pool.map(_pool_stats, range(K), chunksize=1)
            bs = np.stack([x[1] for x in st])
            params, valid = rc.estimate(cams, opts, bs, prev_p, prev_v)
            pool.map(_pool_apply, [(k, params[k]) for k in range(K)], chunksize=1)
            t_total += time.perf_counter() - t0
            prev_p, prev_v = params, valid
            n += 1
    return {"value": round(px * n / t_total / 1e9, 6), "unit": "GPix/s", "cores": min(workers, K),
            "workers": workers, "host_cores_available": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"{n} whole frame-sets of {rig.name} ({px * n / 1e6:.1f} MPix) through the numpy oracle, "
                      f"{t_total:.1f} s over a pool of {workers} processes, one task per camera "
                      f"(corrected frames stay in the workers)"}


def apply_bytes(cams) -> int:
    """Algorithmic bytes of one apply launch: every sample read and written once."""
    return sum(2 * c.width * c.height * c.channels * (1 if c.bit_depth == 8 else 2) for c in cams)


MLP_FLOP_PER_SAMPLE_STEP = 3 * 2 * (576 * 256 + 256 * 256 + 256 * 6)   # forward + backward (2x forward)


def feature_moment_estimate(X):
    """The six targets estimated from the network's own inputs without the
    network: per channel, the mean and standard deviation of the own band's
    and of the facing band's 64-bin densities (regions 1 and 2 of X) from the
    bin centres with Sheppard's correction of the 4-wide bins, then the
    midway fit (a = (sigma_own + sigma_fac) / (2 sigma_own) clamped to
    [1/8, 8], b = mu* - a mu_own).  An evaluation baseline: it shows how
    closely any function of 64-bin histograms can follow the exact-moment
    estimate (float64 [N][6] on X's device)."""
    import torch
    X = X.double()
    centres = 4.0 * torch.arange(64, dtype=torch.float64, device=X.device) + 1.5
    out = torch.zeros((X.shape[0], 6), dtype=torch.float64, device=X.device)
    for c in range(3):
        mom = []
        for region in (1, 2):
            d = X[:, region * 192 + c * 64: region * 192 + (c + 1) * 64]
            w = d / d.sum(dim=1, keepdim=True).clamp_min(1e-300)
            mu = (w * centres).sum(dim=1)
            var = ((w * centres * centres).sum(dim=1) - mu * mu - 16.0 / 12.0).clamp_min(0.0)
            mom.append((mu, var.sqrt()))
        (mo, so), (mf, sf) = mom
        a = torch.where(so > 0, (so + sf) / (2 * so.clamp_min(1e-300)), torch.ones_like(so)).clamp(0.125, 8.0)
        out[:, c] = a
        out[:, 3 + c] = ((mo + mf) / 2 - a * mo) / 255.0
    return out


def surrogate_leg(args, rig, ins, outs):
    """Train the surrogate on the device (dataset from the plain estimator on
    seeded rigs), then time its inference path on the benchmark rig and
    report how often and how closely it replaces the plain estimate."""
    import torch
    from paper_1910_03517_amd import rt, synth
    from paper_1910_03517_amd import surrogate as sg

    log("surrogate: building the dataset")
    t0 = time.perf_counter()
    data = sg.build_dataset("rig14", n_bases=args.sur_bases, draws_per_base=args.sur_draws, seed=0)
    held = sg.build_dataset("rig14", n_bases=2, draws_per_base=16, seed=1)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n = int(data.X.shape[0])
    log(f"surrogate: {n} samples in {t_data:.1f} s; training")
    tr = sg.Trainer(synth.mlp_init(0), lr=args.sur_lr, batch=1024)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    def lr_at(e):                                   # cosine decay from sur_lr to sur_lr_min
        return args.sur_lr_min + 0.5 * (args.sur_lr - args.sur_lr_min) * (1 + math.cos(math.pi * e / args.sur_epochs))

    tr.lr = lr_at(0)
    losses = [tr.epoch(data)]                      # first epoch: warm-up, not timed
    steps0 = tr.step
    e0.record()
    for e in range(1, args.sur_epochs):
        tr.lr = lr_at(e)
        losses.append(tr.epoch(data))
    e1.record()
    torch.cuda.synchronize()
    train_s = e0.elapsed_time(e1) / 1e3
    samples = (tr.step - steps0) * tr.batch
    # The same training kernels at larger mini-batches (throughput only, a
    # fresh network each, not the trained model): how much of the gap to the
    # FP32 peak is the 1024-sample batch's small products.
    scaling = {}
    for bs in (4096, 16384):
        tb = sg.Trainer(synth.mlp_init(1), lr=args.sur_lr, batch=bs)
        tb.epoch(data)
        s0 = tb.step
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            tb.epoch(data)
        z.record()
        torch.cuda.synchronize()
        sec = a.elapsed_time(z) / 1e3
        ns = (tb.step - s0) * bs
        scaling[str(bs)] = {"samples_per_s": round(ns / sec, 1),
                            "TFLOP_s": round(ns * MLP_FLOP_PER_SAMPLE_STEP / sec / 1e12, 3)}
        del tb
    # Held-out residuals (max over the unit's six outputs, normalised units).
    y = sg.predict(tr.w, held.X)
    res = (y - held.T).abs().amax(dim=1).cpu().numpy()
    floor = (feature_moment_estimate(held.X) - held.T.double()).abs().amax(dim=1).cpu().numpy()

    log(f"surrogate: trained, loss {losses[0]:.3g} -> {losses[-1]:.3g}; timing inference")
    # Inference: the surrogate frame-set on the benchmark rig, eager, against the plain one.
    sur = sg.Surrogate(tr.w, tol=args.sur_tol)
    ws = sg.Workspace(rig.sizes)
    b = rig.bufs
    px = sum(c.width * c.height for c in rig.cams)
    nb = len(ins)

    def timed(fn, k):
        for i in range(5):
            fn(i)
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(k):
            fn(i)
        z.record()
        torch.cuda.synchronize()
        return a.elapsed_time(z) / k

    k = max(args.steps // 3, 20)
    ms_plain = timed(lambda i: rig.frameset(ins[i % nb], outs[i % nb]), k)
    ms_sur = timed(lambda i: sur.frameset(rig, ins[i % nb], outs[i % nb], b.whole_hist, ws), k)
    used = ws.used.float().mean().item()
    r_used = ws.residual[ws.used.bool()]
    sur_hi = sg.Surrogate(tr.w, tol=args.sur_tol_engaged)
    ms_hi = timed(lambda i: sur_hi.frameset(rig, ins[i % nb], outs[i % nb], b.whole_hist, ws), k)
    used_hi = ws.used.float().mean().item()
    r_hi = ws.residual[ws.used.bool()]
    rig.check()

    def residuals(r):
        return {"p50": round(float(np.percentile(r, 50)), 5), "p90": round(float(np.percentile(r, 90)), 5),
                "used_at": {str(t): round(float((r <= t).mean()), 4) for t in (1e-3, 3e-3, 1e-2, 3e-2, 1e-1)}}
    return tr.w, {
        "dataset": {"samples": n, "build_s": round(t_data, 2), "source": "plain estimator on seeded 14x1920x1080 rigs",
                    "bases": args.sur_bases, "draws_per_base": args.sur_draws},
        "training": {"epochs": args.sur_epochs, "batch": tr.batch, "lr": args.sur_lr, "lr_min": args.sur_lr_min,
                     "schedule": "cosine decay per epoch",
                     "loss_first_epoch": round(losses[0], 7), "loss_last_epoch": round(losses[-1], 7),
                     "samples_per_s": round(samples / train_s, 1),
                     "TFLOP_s": round(samples * MLP_FLOP_PER_SAMPLE_STEP / train_s / 1e12, 3),
                     "fp32_peak_TFLOP_s": 157.3,
                     "larger_batches": {**scaling, "what": "the same kernels at larger mini-batches, three epochs "
                                                           "of a fresh network each (throughput only)"}},
        "held_out_residual": {**residuals(res), "units": int(res.size)},
        "held_out_floor": {**residuals(floor),
                           "what": "moment estimate from the same 64-bin features (bin centres, Sheppard's "
                                   "correction, the midway fit): the quantisation floor of the network's inputs"},
        "inference": {"tol": args.sur_tol, "GPix_s": round(px / (ms_sur / 1e3) / 1e9, 2),
                      "plain_GPix_s": round(px / (ms_plain / 1e3) / 1e9, 2),
                      "ms_per_frameset": round(ms_sur, 4), "plain_ms_per_frameset": round(ms_plain, 4),
                      "used_fraction": round(used, 4),
                      "max_residual_used": float(r_used.max().item()) if r_used.numel() else None,
                      "launch": "eager, one stream, both paths"},
        "inference_engaged": {"tol": args.sur_tol_engaged, "GPix_s": round(px / (ms_hi / 1e3) / 1e9, 2),
                              "ms_per_frameset": round(ms_hi, 4), "used_fraction": round(used_hi, 4),
                              "max_residual_used": float(r_hi.max().item()) if r_hi.numel() else None,
                              "what": "the same inference path at a tolerance where the network is used"},
    }


def vga_leg(reps: int = 200) -> dict:
    """One 640x480 RGB camera through the four separate calls and through
    rt_frameset: microseconds per call (launch-latency bound)."""
    import torch
    from paper_1910_03517_amd import rt, synth
    spec = synth.single_vga()
    cams = [rt.Camera(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos).with_pitch() for c in spec.cams]
    rig = rt.Rig(cams, rt.Options())
    dev = rig.upload(synth.rig_frames(spec, 0))
    out = rig.alloc_frames()
    calls = {"rt_stats": lambda: rig.stats(dev, whole=False), "rt_estimate": rig.estimate,
             "rt_build_lut": rig.build_lut, "rt_apply": lambda: rig.apply(dev, out, whole=True),
             "rt_frameset": lambda: rig.frameset(dev, out)}
    res = {}
    for name, fn in calls.items():
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        z.record()
        torch.cuda.synchronize()
        res[name + "_us"] = round(a.elapsed_time(z) / reps * 1e3, 2)
    rig.check()
    rig.close()
    res["what"] = "1x640x480 rgb8, back-to-back calls on one stream, device time per call"
    return res


def serving_leg(args, base, surrogate_w=None) -> dict:
    """Three rigs of the benchmark camera ring in one context behind the
    server: paced (30 fps per rig, exponential jitter of mean 2 ms), the same
    arrival process replayed `serve_speedup` times faster (a load near the
    server's capacity, where batches across rigs form), and saturated
    (every frame-set submitted at once); then more rigs than one context
    takes, spread over contexts (ShardedBackend), saturated."""
    import threading

    import torch
    from paper_1910_03517_amd import synth
    from paper_1910_03517_amd.serving import GpuBackend, Server, ShardedBackend
    from paper_1910_03517_amd.surrogate import Surrogate

    spec = synth.rig14_1080p()
    n_rigs, pool = 3, 4
    out = {"rigs": n_rigs, "rig": spec.name, "fps": 30, "jitter_ms": 2.0, "mem_budget_framesets": 4,
           "accelerated_speedup": args.serve_speedup, "accelerated_seconds": args.serve_accel_seconds,
           "plain_apply_lanes": args.serve_lanes}
    tuned_plain = None
    for path in ("plain", "surrogate"):
        if path == "surrogate" and surrogate_w is None:
            continue
        sur = Surrogate(surrogate_w, tol=args.sur_tol) if path == "surrogate" else None
        be = GpuBackend([spec.cams] * n_rigs, surrogate=sur, lanes=args.serve_lanes)
        frames = []
        for r in range(n_rigs):
            cams = [be.cams[i] for i in be.idx[r]]
            per = []
            for i in range(pool):
                dev = [torch.zeros((c.height, c.pitch_bytes), dtype=torch.uint8, device="cuda") for c in cams]
                for d, c, f in zip(dev, cams, base[(r + i) % len(base)]):
                    raw = np.ascontiguousarray(f).view(np.uint8).reshape(c.height, c.row_bytes)
                    d[:, :c.row_bytes].copy_(torch.from_numpy(raw))
                per.append(dev)
            frames.append(per)
        torch.cuda.synchronize()
        if path == "plain":
            if be.tuned is None:
                be.autotune([frames[r][0] for r in range(n_rigs)])
            out["tuned"] = {"source": be.tuned_source, "tile_rows": be.tuned.tile_rows, "grid": be.tuned.grid,
                            "us_per_batch_of_3_when_tuned": round(be.tuned.us_per_frameset, 2)}
        elif tuned_plain is not None:
            be.rig.tune(tuned_plain.tile_rows, tuned_plain.grid)
        fs_bytes = be.frameset_bytes(0)
        res = {}
        # Paced: arrivals of each rig at phase + i/30 s + Exp(2 ms), seeded.
        rng = np.random.default_rng([1910, 5])
        n_each = int(args.serve_seconds * 30)
        arrivals = sorted((float(rng.uniform(0, 1 / 30)) + i / 30 + float(rng.exponential(2e-3)), r, i)
                          for r in range(n_rigs) for i in range(n_each))
        S = args.serve_speedup
        n_acc = int(args.serve_accel_seconds * 30 * S)
        arrivals_acc = sorted((float(rng.uniform(0, 1 / (30 * S))) + i / (30 * S) + float(rng.exponential(2e-3 / S)),
                               r, i) for r in range(n_rigs) for i in range(n_acc))
        for mode in ("paced", "accelerated", "saturated"):
            log(f"serving: {path} {mode}")
            srv = Server(be, mem_budget=4 * fs_bytes, max_batches_in_flight=3, queue_limit=1 << 20)
            # warm-up outside the measurement
            for r in range(n_rigs):
                srv.submit(r, frames[r][0])
            srv.drain()
            srv.finished.clear()
            srv.batch_sizes.clear()
            srv.start()
            if mode in ("paced", "accelerated"):
                t_start = time.perf_counter()
                for t, r, i in (arrivals if mode == "paced" else arrivals_acc):
                    dt = t_start + t - time.perf_counter()
                    if dt > 2e-4:
                        time.sleep(dt - 1e-4)
                    while t_start + t > time.perf_counter():
                        pass
                    srv.submit(r, frames[r][i % pool])
            else:
                n_sat = args.serve_saturated
                for i in range(n_sat):
                    for r in range(n_rigs):
                        srv.submit(r, frames[r][i % pool])
            srv.stop(drain=True)
            rep = srv.report()
            res[mode] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
        res["offered_GPix_s"] = round(n_rigs * 30 * be.rig_pixels(0) / 1e9, 3)
        res["accelerated_offered_GPix_s"] = round(n_rigs * 30 * S * be.rig_pixels(0) / 1e9, 3)
        if path == "plain":
            tuned_plain = be.tuned
        be.close()
        out[path] = res
    if args.serve_sharded_rigs > 0:
        n6 = args.serve_sharded_rigs
        log(f"serving: {n6} rigs over several contexts, saturated")
        be = ShardedBackend([spec.cams] * n6, lanes=args.serve_lanes)
        frames = []
        for r in range(n6):
            cams = be.rig_cams(r)
            per = []
            for i in range(2):
                dev = [torch.zeros((c.height, c.pitch_bytes), dtype=torch.uint8, device="cuda") for c in cams]
                for d, c, f in zip(dev, cams, base[(r + i) % len(base)]):
                    raw = np.ascontiguousarray(f).view(np.uint8).reshape(c.height, c.row_bytes)
                    d[:, :c.row_bytes].copy_(torch.from_numpy(raw))
                per.append(dev)
            frames.append(per)
        torch.cuda.synchronize()
        srv = Server(be, mem_budget=2 * n6 * be.frameset_bytes(0), max_batches_in_flight=3, queue_limit=1 << 20)
        for r in range(n6):
            srv.submit(r, frames[r][0])
        srv.drain()
        srv.finished.clear()
        srv.batch_sizes.clear()
        srv.start()
        for i in range(args.serve_saturated):
            for r in range(n6):
                srv.submit(r, frames[r][i % 2])
        srv.stop(drain=True)
        rep = srv.report()
        out["sharded"] = {"rigs": n6, "cameras": n6 * len(spec.cams), "contexts": len(be.shards),
                          "saturated": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()},
                          "what": "rigs filled into contexts of at most 64 cameras, one launch per context and "
                                  "batch on the context's own stream; every frame-set submitted at once"}
        be.close()
    return out


def removal_leg(rig, ins, outs, lanes: int = 2, group: int = 3, fuse: bool = True) -> dict:
    """Object removal with the smoothing fallback (section 3.1) on the
    benchmark rig: one rt_frameset_removal per frame-set (the previous
    frame-set's input as the reference for the frame difference), eager on
    one stream, next to eager rt_frameset on the same buffers, then both
    through the frame-set pipeline in the given form; and the seam gradient
    cost monitor (section 4.2) per call on the corrected frames."""
    import torch
    from paper_1910_03517_amd import rt
    K, NB = rig.sizes.n_cams, rig.sizes.n_blocks
    kept = torch.zeros((K, 2, NB, 3, 3), dtype=torch.int64, device="cuda")
    method = torch.zeros((K, 2, NB), dtype=torch.uint8, device="cuda")
    seam = torch.zeros(K, dtype=torch.float64, device="cuda")
    inter = torch.zeros(K, dtype=torch.float64, device="cuda")
    nb = len(ins)
    px = sum(c.width * c.height for c in rig.cams)

    def timed(fn, k=60):
        for i in range(5):
            fn(i)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(k):
            fn(5 + i)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k * 1e3

    rm_us = timed(lambda i: rig.frameset_removal(ins[i % nb], ins[(i - 1) % nb], outs[i % nb], kept, method))
    m = method.cpu().numpy()
    plain_us = timed(lambda i: rig.frameset(ins[i % nb], outs[i % nb]))

    def pipe_us(removal: bool, k: int = 60) -> float:
        pipe = rt.Pipe.for_rig(rig, depth=8, lanes=lanes, group=group, fuse=fuse)
        if removal:
            pipe.set_removal(kept, method)
        try:
            for i in range(6):
                pipe.submit(ins[i % nb], outs[i % nb])
            pipe.join()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(k):
                pipe.submit(ins[(6 + i) % nb], outs[(6 + i) % nb])
            pipe.join()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / k * 1e3
        finally:
            pipe.close()

    rm_pipe_us = pipe_us(True)
    m_pipe = method.cpu().numpy()
    plain_pipe_us = pipe_us(False)
    seam_us = timed(lambda i: rt.rt_seam_cost(rig.ctx, outs[i % nb], 8, seam, inter))
    vb = rt.Rig(rig.cams, rt.Options(vblend=True))
    vblend_us = timed(lambda i: vb.frameset(ins[i % nb], outs[i % nb]))
    vb.check()
    vb.close()
    qf = rt.Rig(rig.cams, rt.Options(fit="quantile"))
    quantile_us = timed(lambda i: qf.frameset(ins[i % nb], outs[i % nb]))
    qf.check()
    qf.close()
    xr = rt.Rig(rig.cams, rt.Options())
    xs = rt.CrossSet(xr.sizes)
    cross_us = timed(lambda i: rt.rt_frameset_cross(xr.ctx, ins[i % nb], outs[i % nb], xr.bufs, xs))
    cross_apply_us = timed(lambda i: rt.rt_apply_cross(xr.ctx, ins[i % nb], outs[i % nb], xs, xr.bufs.whole_hist,
                                                       xr.bufs.whole_sums))
    p3 = xs.params3.cpu().numpy()
    units_3x3 = int((abs(p3[..., [1, 2, 3, 5, 6, 7]]).max(axis=-1) > 0).sum())
    xr.check()
    xr.close()
    att = rig.attention(ins[0], ins[1])            # buffers of the leg, then the timed calls
    att_us = timed(lambda i: rt.rt_attention(rig.ctx, ins[i % nb], ins[(i - 1) % nb], 20, 16, 8, 256, *att))
    att_bytes = 2 * sum(c.width * c.height * c.channels * c.bps for c in rig.cams)
    s_out = seam.cpu().numpy()
    rt.rt_seam_cost(rig.ctx, ins[0], 8, seam, inter)
    s_in = seam.cpu().numpy()
    rig.check()
    return {"removal_us_per_frameset": round(rm_us, 2), "removal_GPix_s": round(px / rm_us / 1e3, 2),
            "plain_us_per_frameset": round(plain_us, 2), "plain_GPix_s": round(px / plain_us / 1e3, 2),
            "removal_pipe_us_per_frameset": round(rm_pipe_us, 2), "removal_pipe_GPix_s": round(px / rm_pipe_us / 1e3, 2),
            "plain_pipe_us_per_frameset": round(plain_pipe_us, 2),
            "plain_pipe_GPix_s": round(px / plain_pipe_us / 1e3, 2),
            "pipe_form": {"lanes": lanes, "group": group, "fuse": int(bool(fuse)), "frame_sets": 60},
            "units_removal_pipe": int((m_pipe == 1).sum()),
            "units_removal": int((m == 1).sum()), "units_smoothing": int((m == 2).sum()),
            "seam_monitor_us": round(seam_us, 2),
            "vblend_us_per_frameset": round(vblend_us, 2), "vblend_GPix_s": round(px / vblend_us / 1e3, 2),
            "quantile_fit_us_per_frameset": round(quantile_us, 2),
            "quantile_fit_GPix_s": round(px / quantile_us / 1e3, 2),
            "cross3x3_us_per_frameset": round(cross_us, 2), "cross3x3_GPix_s": round(px / cross_us / 1e3, 2),
            "cross3x3_apply_us": round(cross_apply_us, 2),
            "cross3x3_apply_hbm_frac": round(6 * px / cross_apply_us / 1e3 / HBM_PEAK_GBS, 4),
            "cross3x3_units_3x3": units_3x3, "cross3x3_units": int(p3.shape[0] * p3.shape[1] * p3.shape[2]),
            "attention_us": round(att_us, 2), "attention_GB_s": round(att_bytes / att_us / 1e3, 1),
            "attention_hbm_frac": round(att_bytes / att_us / 1e3 / HBM_PEAK_GBS, 4),
            "seam_cost_input_mean": round(float(s_in.mean()), 3), "seam_cost_corrected_mean": round(float(s_out.mean()), 3),
            "interior_cost_corrected_mean": round(float(inter.cpu().numpy().mean()), 3),
            "what": "eager, one stream, unless named pipe; removal: rt_frameset_removal with the previous "
                    "frame-set as reference (tau 20, min_kept 0.25); removal_pipe / plain_pipe: the same through "
                    "rt_pipe (rt_pipe_set_removal) in pipe_form, submits back to back and one join; seam monitor: rt_seam_cost (factor 8) of every seam and image centre; "
                    "vblend: rt_frameset with the maps of adjacent blocks blended row by row; quantile fit: "
                    "rt_frameset with fit = quantile; cross3x3: rt_frameset_cross (band and cross sums, 3x3 fit, "
                    "maps, apply with whole-frame statistics) and rt_apply_cross alone (units_3x3: units whose map "
                    "has off-diagonal terms, the rest took the per-channel fallback); attention: "
                    "rt_attention (tau 20, 16-pixel cells, 8x8-cell windows) on two consecutive frame-sets, "
                    "both frames read once"}


def moving_object_leg() -> dict:
    """Section 4.1's comparison on the device: a striped vehicle crosses the
    seam between the first two cameras of a 4 x 1920x1080 ring in 16 frames;
    each method (standard, removal alone, removal with the smoothing
    fallback, smoothing) with 16 and 64 blocks corrects the scene with and
    without the vehicle; reported: the discolouration of the seam-side
    correction domains in the blocks the vehicle overlaps (mean absolute
    difference of the two corrected results over background samples, grey
    levels; per frame, its maximum and mean over the sequence) and the seam
    gradient cost of the corrected frames at that seam."""
    import numpy as np
    import torch
    from paper_1910_03517_amd import evaluate, rt, synth
    W, H, K, T = 1920, 1080, 4, 16
    spec = synth.RigSpec("moving-object 4x1920x1080 rgb8", 41, [synth.CamSpec(W, H, 3, 8, 0, p) for p in range(K)])
    # 40 px per frame: the stripes of the vehicle (period 16 px) move by half a
    # period between frames, so its inside changes too (at a multiple of the
    # period it would look still to the frame difference).
    ob = synth.seam_crossing(spec, 0, speed=40.0, frames=T, rows=(0.62, 0.657), width_frac=0.08)
    cams = [rt.Camera(W, H, 3, 8, 0, p).with_pitch() for p in range(K)]
    host = {tag: [synth.rig_frames(spec, t, objects=objs) for t in range(T)]
            for tag, objs in (("obj", (ob,)), ("ref", ()))}
    up = rt.Rig(cams, rt.Options())
    dev = {tag: [up.upload(f) for f in fr] for tag, fr in host.items()}
    up.close()
    out = {"workload": spec.name, "frames": T, "object_rows": [ob.y0, ob.y0 + ob.h], "object_width": ob.w,
           "speed_px_per_frame": ob.speed}
    for nb in (16, 64):
        rows = evaluate.affected_rows(H, nb, ob.y0, ob.h)
        ml, mr = evaluate.seam_halves_mask(H, W, W, rows)
        aff = [j for j in range(nb) if rows[j * H // nb]]
        for mode in ("standard", "removal", "auto", "smoothing"):
            res, seams, units = {}, {}, [0, 0]
            for tag in ("obj", "ref"):
                rig = rt.Rig(cams, rt.Options(n_blocks=nb, smoothing=(mode == "smoothing")))
                kept = torch.zeros((K, 2, nb, 3, 3), dtype=torch.int64, device="cuda")
                method = torch.zeros((K, 2, nb), dtype=torch.uint8, device="cuda")
                o = rig.alloc_frames()
                seq, sc = [], []
                for t in range(T):
                    if mode in ("removal", "auto"):
                        rig.frameset_removal(dev[tag][t], dev[tag][t - 1] if t else None, o, kept, method,
                                             min_kept=0.0 if mode == "removal" else 0.25)
                        if tag == "obj":
                            m = method.cpu().numpy()
                            for k, s in ((0, 1), (1, 0)):
                                units[0] += int((m[k, s, aff] == 1).sum())
                                units[1] += int((m[k, s, aff] == 2).sum())
                    else:
                        rig.frameset(dev[tag][t], o)
                    sc.append(float(rig.seam_cost(o)[0][0]))
                    seq.append([o[k][:, :W * 3].reshape(H, W, 3).cpu().numpy() for k in (0, 1)])
                rig.check()
                rig.close()
                res[tag], seams[tag] = seq, sc
            d = [evaluate.discolouration([(host["obj"][t][0], host["ref"][t][0], res["obj"][t][0], res["ref"][t][0], ml),
                                          (host["obj"][t][1], host["ref"][t][1], res["obj"][t][1], res["ref"][t][1], mr)])
                 for t in range(T)]
            entry = {"discolouration_max": round(max(d), 3), "discolouration_mean": round(float(np.mean(d)), 3),
                     "seam_cost_mean": round(float(np.mean(seams["obj"])), 3),
                     "seam_cost_without_object_mean": round(float(np.mean(seams["ref"])), 3)}
            if mode in ("removal", "auto"):
                entry["affected_units_removal"], entry["affected_units_smoothing"] = units
            out[f"{mode}@{nb}"] = entry
    return out


def copy_ceiling(rt, torch, frame_bytes: int, nbuf: int, steps: int, warmup: int) -> float:
    """GB/s of a read+write stream of the same bytes with the apply's vector width."""
    src = [torch.empty(frame_bytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    dst = [torch.empty(frame_bytes, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    for i in range(warmup):
        rt.rt_stream_copy(dst[i % nbuf], src[i % nbuf], frame_bytes, 12)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    c0.record()
    for i in range(steps):
        rt.rt_stream_copy(dst[i % nbuf], src[i % nbuf], frame_bytes, 12)
    c1.record()
    torch.cuda.synchronize()
    return 2 * frame_bytes * steps / (c0.elapsed_time(c1) / 1e3) / 1e9


def plain_leg(args, rig_spec, steps: int, warmup: int, timing_every: int = 0):
    """The timed region of the plain path on one rig: `steps` frame-sets back
    to back in the chosen launch mode, the apply launches timed by the
    library's events (every timing_every-th; 0: about five launches of the
    region), then the single-frame-set launches alone and the frame-set
    latency.  Returns (rig, report, ins, outs, base)."""
    import torch
    from paper_1910_03517_amd import rt, synth

    cams = [rt.Camera(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos).with_pitch() for c in rig_spec.cams]
    px = sum(c.width * c.height for c in cams)
    frame_bytes = apply_bytes(cams) // 2
    copy_gbs = copy_ceiling(rt, torch, frame_bytes, args.nbuf, steps, warmup)

    opts = rt.Options(smoothing=args.smoothing)
    rig = rt.Rig(cams, opts)
    if args.tile_rows or args.grid is not None:
        rig.tune(args.tile_rows or rig.tuning()[0], rig.tuning()[1] if args.grid is None else args.grid)
    alg_bytes = algorithmic_bytes(cams, opts.band_width)

    # Distinct frame-sets rotated through NBUF buffer pairs (distinct addresses).
    base = [synth.rig_frames(rig_spec, t, drift=True) for t in range(2)]
    ins = [rig.upload(base[i % 2]) for i in range(args.nbuf)]
    outs = [rig.alloc_frames() for _ in range(args.nbuf)]
    torch.cuda.synchronize()

    # Launch knobs of the pipe mode: given on the command line, else the
    # autotuner's (cached for this rig and device, or timed now in the pipe
    # mode itself; the knobs never change results).
    lanes, group, fuse = args.lanes or 3, args.group or 3, max(args.fuse, 0)
    tuned = {"source": "command line" if (args.lanes or args.group or args.tile_rows or args.grid is not None
                                          or args.fuse >= 0) else "default"}
    if args.mode == "pipe" and tuned["source"] == "default" and not args.no_autotune:
        from paper_1910_03517_amd import autotune
        t_tune = time.perf_counter()
        choice = autotune.cached_pipe(rig)
        src = "cache"
        if choice is None:
            log(f"{rig_spec.name}: autotuning the pipe (lanes, group, fused or not, tile rows, grid)")
            choice = autotune.tune_pipe(rig, ins, outs, depth=args.depth)
            src = "tuned"
        lanes, group, fuse = choice.lanes, choice.group, choice.fuse
        tuned = {"source": src, "lanes": lanes, "group": group, "fuse": fuse, "tile_rows": choice.tile_rows,
                 "grid": choice.grid, "us_per_frameset_when_tuned": round(choice.us_per_frameset, 2),
                 "seconds": round(time.perf_counter() - t_tune, 2)}
        # The tuning advanced the estimator state: back to the initial one.
        rig.bufs.params.zero_()
        rig.bufs.params[..., 0] = 1.0
        rig.bufs.valid.zero_()
        torch.cuda.synchronize()
    tile_rows, grid, n_tiles = rig.tuning()

    stream = torch.cuda.current_stream()
    pipe, graphs = None, None
    b = rig.bufs
    if args.mode == "pipe":
        # A frame-set's buffers are reused `nbuf` steps later: with nbuf a
        # multiple of depth that apply starts only after the earlier one ended.
        assert max(lanes, group) <= args.depth and args.nbuf % args.depth == 0, \
            "need lanes, group <= depth and depth | nbuf"
        pipe = rt.Pipe.for_rig(rig, depth=args.depth, lanes=lanes, group=group, fuse=bool(fuse))
        in_ptrs = [rt.ptr_array(x) for x in ins]
        out_ptrs = [rt.ptr_array(x) for x in outs]
    elif args.mode == "graph":
        # One captured frame-set; each step rebinds its frames (rt_graph_set_frames) and launches it.
        whole = rt.WholeSet(rig.sizes)
        graphs = [rt.Graph(rig.ctx, ins[0], outs[0], rt.LutSet(rig.sizes), whole, b)]
        in_ptrs = [rt.ptr_array(x) for x in ins]
        out_ptrs = [rt.ptr_array(x) for x in outs]
    elif args.mode == "graph-pipelined":
        # Two two-branch graphs (the table buffers alternate), frames rebound every step.
        assert args.nbuf % 2 == 0
        luts = [rt.LutSet(rig.sizes) for _ in range(2)]
        wholes = [rt.WholeSet(rig.sizes) for _ in range(2)]
        rt.rt_stats(rig.ctx, ins[0], b.band_hist, b.band_sums)
        rt.rt_estimate(rig.ctx, b.band_hist, b.band_sums, b.params, b.valid)
        rt.rt_build_lut(rig.ctx, b.params, b.valid, luts[0].lut8, luts[0].q16, luts[0].weights)
        graphs = [rt.Graph(rig.ctx, ins[p], outs[p], luts[p], wholes[p], b, ins[p + 1], luts[1 - p]) for p in range(2)]
        in_ptrs = [rt.ptr_array(x) for x in ins]
        out_ptrs = [rt.ptr_array(x) for x in outs]
    elif args.mode == "ahead":
        # One rt_frameset_ahead launch per step: the apply of frame-set i with
        # the tables the previous launch built, beside the estimate of i + 1;
        # two table and two whole-statistics buffers taken in turn.
        ahead = ([rt.LutSet(rig.sizes) for _ in range(2)], [rt.WholeSet(rig.sizes) for _ in range(2)])
        in_ptrs = [rt.ptr_array(x) for x in ins]
        out_ptrs = [rt.ptr_array(x) for x in outs]
        rt.rt_frameset_ahead(rig.ctx, None, None, None, None, ins[0], ahead[0][0], ahead[1][0], b, stream,
                             ptrs=(None, None, in_ptrs[0]))

    def step(i, ready=None):
        if graphs is not None:
            j = i % args.nbuf
            g = graphs[i % len(graphs)]
            if args.mode == "graph":
                g.set_frames(None, None, frame_ptrs=in_ptrs[j], out_ptrs=out_ptrs[j])
            else:
                g.set_frames(None, None, frame_ptrs=in_ptrs[j], out_ptrs=out_ptrs[j],
                             next_ptrs=in_ptrs[(j + 1) % args.nbuf])
            g.launch(stream)
        elif pipe is not None:
            j = i % args.nbuf
            pipe.submit(ins[j], outs[j], stream, in_ptrs[j], out_ptrs[j], ready_event=ready)
        elif args.mode == "ahead":
            j, p = i % args.nbuf, i % 2
            luts, wholes = ahead
            rt.rt_frameset_ahead(rig.ctx, None, None, luts[p], wholes[p], None, luts[1 - p], wholes[1 - p], b, stream,
                                 ptrs=(in_ptrs[j], out_ptrs[j], in_ptrs[(j + 1) % args.nbuf]))
        else:
            rig.frameset(ins[i % args.nbuf], outs[i % args.nbuf])

    # The pipe takes the timed frame-sets a group at a time in one library
    # call each (rt_pipe_submit_n, pointer arrays built beforehand).
    chunks = {}
    if pipe is not None:
        for j in range(args.nbuf):
            idx = [(j + u) % args.nbuf for u in range(group)]
            chunks[j] = (rt.ptr_array_n([ins[x] for x in idx]), rt.ptr_array_n([outs[x] for x in idx]), group)

    def steps_from(i0, n):
        if pipe is None:
            for i in range(n):
                step(i0 + i)
            return
        i = 0
        while i < n:
            c = min(group, n - i)
            j = (i0 + i) % args.nbuf
            if c == group:
                pipe.submit_n(None, None, stream, ptrs=chunks[j])
            else:
                for u in range(c):
                    step(i0 + i + u)
            i += c

    log(f"{rig_spec.name}: timing {steps} steps ({args.mode})")
    for i in range(warmup):
        step(i)
    if pipe is not None:
        pipe.join(stream)
    torch.cuda.synchronize()
    rig.check()
    first = warmup          # continue the step sequence (pipelined graphs chain step to step)

    # Timed region: exactly `steps` frame-sets back to back, bracketed by a
    # start and an end event.  The library attaches its own events to every
    # n-th apply dispatch in the region (the dominant kernel's durations).
    if timing_every <= 0:
        # Apply launches in the region: one per frame-set, or, fused, the
        # first `lanes` alone and then one per group.
        launches = steps if not (pipe is not None and pipe.fuse) else \
            min(steps, lanes) + -(-max(0, steps - lanes) // group)
        timing_every = max(1, launches // 5)
    rt.rt_ctx_timing(rig.ctx, steps, timing_every)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    steps_from(first, steps)
    if pipe is not None:
        pipe.join(stream)
    ev1.record(stream)
    host_issue = time.perf_counter() - w0
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    rig.check()
    ms_total = ev0.elapsed_time(ev1)
    apply_ms = np.array(rt.rt_ctx_apply_times(rig.ctx, steps))
    apply_sets = np.array(rt.rt_ctx_apply_sets(rig.ctx, steps), dtype=np.float64)
    rt.rt_ctx_timing(rig.ctx, 0)
    first += steps
    apply_where = f"inside the timed region, every {timing_every}th apply launch"
    if apply_ms.size == 0:
        # Captured graphs and the look-ahead launches carry no apply timing
        # events: time the apply launches on their own.
        apply_where = ("separate loop (graph modes record no events inside the graph)" if args.mode != "ahead" else
                       "separate loop (the look-ahead launch is timed as the step)")
        rt.rt_ctx_timing(rig.ctx, steps)
        for i in range(steps):
            rt.rt_apply(rig.ctx, ins[i % args.nbuf], outs[i % args.nbuf], b.lut8, b.q16, b.weights,
                        b.whole_hist, b.whole_sums, stream=stream)
        torch.cuda.synchronize()
        apply_ms = np.array(rt.rt_ctx_apply_times(rig.ctx, steps))
        apply_sets = np.ones(apply_ms.size)
        rt.rt_ctx_timing(rig.ctx, 0)

    # The single-frame-set apply with no other work beside it (one stream,
    # launches back to back).
    rt.rt_ctx_timing(rig.ctx, steps)
    for i in range(steps):
        rt.rt_apply(rig.ctx, ins[i % args.nbuf], outs[i % args.nbuf], b.lut8, b.q16, b.weights,
                    b.whole_hist, b.whole_sums, stream=stream)
    torch.cuda.synchronize()
    single_ms = np.array(rt.rt_ctx_apply_times(rig.ctx, steps))
    rt.rt_ctx_timing(rig.ctx, 0)
    # The timed region's kernel form alone: fused, rt_apply_sets with the
    # group's frame-sets per launch (the pipeline's slot tables); else the
    # single-frame-set launches above.
    alone_ms, alone_sets = single_ms, np.ones(single_ms.size)
    if pipe is not None and pipe.fuse:
        n = min(group, 4)
        fused = [(rt.ptr_array_n([ins[(i * n + u) % args.nbuf] for u in range(n)]),
                  rt.ptr_array_n([outs[(i * n + u) % args.nbuf] for u in range(n)])) for i in range(args.nbuf)]
        launches = max(4, steps // n)
        rt.rt_ctx_timing(rig.ctx, launches)
        for i in range(launches):
            rt.rt_apply_sets(rig.ctx, None, None, pipe.luts[:n], pipe.whole[:n], stream=stream,
                             ptrs=fused[i % args.nbuf])
        torch.cuda.synchronize()
        alone_ms = np.array(rt.rt_ctx_apply_times(rig.ctx, launches))
        alone_sets = np.array(rt.rt_ctx_apply_sets(rig.ctx, launches), dtype=np.float64)
        rt.rt_ctx_timing(rig.ctx, 0)

    # Frame-set latency, outside the timed region: per-step start and end events.
    n_lat = min(steps, 100)
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    torch.cuda.synchronize()
    for i in range(n_lat):
        ev_s[i].record(stream)
        # The pipeline's statistics stream waits for the start event as for
        # arriving frames, so that no part of the step runs before it.
        step(first + i, ev_s[i])
        if pipe is not None:
            pipe.join(stream)
        ev_e[i].record(stream)
    torch.cuda.synchronize()
    lat_ms = np.array([a.elapsed_time(z) for a, z in zip(ev_s, ev_e)])
    if pipe is not None:
        pipe.close()
    ms_step = ms_total / steps
    gpix = px * steps / (ms_total / 1e3) / 1e9

    ab = apply_bytes(cams)
    launch_us = float(apply_ms.mean() * 1e3)
    sets_per_launch = float(apply_sets.mean())
    achieved = ab * sets_per_launch / (launch_us * 1e-6) / 1e9
    by_sets = {str(int(n)): round(float(apply_ms[apply_sets == n].mean() * 1e3), 2) for n in np.unique(apply_sets)}
    alone_us = float(alone_ms.mean() * 1e3)
    alone_gbs = ab * float(alone_sets.mean()) / (alone_us * 1e-6) / 1e9
    single_us = float(single_ms.mean() * 1e3)
    single_gbs = ab / (single_us * 1e-6) / 1e9
    step_gbs = ab / (ms_step * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": ("k_apply_sets<false> (apply + fused whole-frame statistics, up to 4 frame-sets per launch)"
                       if pipe is not None and pipe.fuse else
                       "k_apply<true,true,false> (apply + fused whole-frame statistics)"),
            "bytes_per_launch": round(ab * sets_per_launch), "bytes_per_frameset": ab,
            "frame_sets_per_launch": round(sets_per_launch, 3), "launch_us_by_frame_sets": by_sets,
            "launch_us": round(launch_us, 2), "launch_timing": apply_where, "launches_timed": int(apply_ms.size),
            "copy_ceiling_GBs": round(copy_gbs, 1), "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
            "alone": {"launch_us": round(alone_us, 2), "achieved": round(alone_gbs, 1),
                      "frac": round(alone_gbs / HBM_PEAK_GBS, 4), "frac_of_copy_ceiling": round(alone_gbs / copy_gbs, 4),
                      "launches_timed": int(alone_ms.size), "frame_sets_per_launch": round(float(alone_sets.mean()), 3),
                      "what": "the timed region's kernel form back to back on one stream after it (fused: "
                              "rt_apply_sets with the group's frame-sets per launch)"},
            "alone_single": {"launch_us": round(single_us, 2), "achieved": round(single_gbs, 1),
                             "frac": round(single_gbs / HBM_PEAK_GBS, 4), "launches_timed": int(single_ms.size),
                             "what": "k_apply<true,true,false>, one frame-set per launch, back to back on one stream"},
            "per_step": {"achieved": round(step_gbs, 1), "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                         "what": "apply bytes per frame-set / time per frame-set (launches may overlap)"}}
    rep = {
        "workload": rig_spec.name, "GPix_s": round(gpix, 3), "ms_per_step": round(ms_step, 5),
        "hbm_frac": round(alg_bytes * steps / (ms_total / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "algorithmic_bytes_per_frameset": alg_bytes, "pixels_per_frameset": px,
        "n_blocks": opts.n_blocks, "band_width": opts.band_width,
        "tile_rows": tile_rows, "apply_grid": grid, "n_tiles": n_tiles, "lanes": lanes, "group": group,
        "fuse": int(bool(pipe is not None and pipe.fuse)),
        "tuned": tuned,
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4),
                       "what": "start to end of each step's GPU work, steps back to back, measured after the timed "
                               "region (in graph-pipelined and ahead modes a frame-set's estimate ran one step earlier)"},
        "wall_s": round(wall, 4), "host_issue_us_per_step": round(host_issue / steps * 1e6, 2),
        "roofline": roof,
    }
    return rig, rep, ins, outs, base


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="rig14", choices=["rig14", "uneven", "vga"])
    ap.add_argument("--nbuf", type=int, default=8)
    ap.add_argument("--smoothing", action="store_true")
    ap.add_argument("--mode", default="pipe", choices=["pipe", "graph-pipelined", "graph", "ahead", "eager"],
                    help="pipe: rt_pipe_submit per step (statistics and estimates on their own stream, applies "
                         "round-robin over --lanes streams); graph-pipelined: one two-branch graph launch per step; "
                         "graph: one captured rt_frameset per step (frames rebound each step); eager: one "
                         "rt_frameset call per step")
    ap.add_argument("--lanes", type=int, default=0,
                    help="apply streams of the pipe mode (default: the autotuner's choice, else 3)")
    ap.add_argument("--group", type=int, default=0,
                    help="frame-sets whose applies the pipe mode issues together (default: the autotuner's, else 3)")
    ap.add_argument("--fuse", type=int, default=-1, choices=[-1, 0, 1],
                    help="pipe mode: 1 issues each group's applies as one launch of up to 4 frame-sets, groups over "
                         "the lanes in turn; 0 one launch per frame-set (default -1: the autotuner's choice, else 0)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="pipe mode: skip the autotuner (3 lanes in groups of 3 and the context's work split)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-sharded-rigs", type=int, default=6,
                    help="serving leg: rigs of the benchmark ring spread over contexts (0: skip)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--grid", type=int, default=None,
                    help="apply workgroups (rt_ctx_tune; 0 = one per tile; default: the context's own choice)")
    ap.add_argument("--depth", type=int, default=8, help="slots of the pipe mode (>= lanes, >= group, divides --nbuf)")
    ap.add_argument("--copy-only", action="store_true", help="time the streaming copy of the frame bytes only")
    ap.add_argument("--timing-every", type=int, default=0,
                    help="time every n-th apply launch of the timed region with HIP events "
                         "(default: about five launches of the region are timed)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate training/inference leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-vga", action="store_true", help="skip the 1x640x480 per-call leg")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven three-ring rig leg")
    ap.add_argument("--no-removal", action="store_true", help="skip the object-removal / seam-monitor leg")
    ap.add_argument("--no-moving-object", action="store_true",
                    help="skip the moving-object comparison of the methods (section 4.1)")
    ap.add_argument("--uneven-steps", type=int, default=0, help="steps of the uneven leg (default: --steps)")
    ap.add_argument("--sur-bases", type=int, default=16)
    ap.add_argument("--sur-draws", type=int, default=28, help="gain draws per base scene (448 units each)")
    ap.add_argument("--sur-epochs", type=int, default=1000)
    ap.add_argument("--sur-lr", type=float, default=1e-3)
    ap.add_argument("--sur-lr-min", type=float, default=1e-5, help="end of the cosine decay of the step size")
    ap.add_argument("--sur-tol", type=float, default=1e-3)
    ap.add_argument("--sur-tol-engaged", type=float, default=3e-2,
                    help="second inference tolerance, one at which the network is used")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="paced serving: 30 frame-sets per second per rig")
    ap.add_argument("--serve-lanes", type=int, default=1,
                    help="apply lanes of the serving backend's frame-set pipeline (plain path; 1 = one stream)")
    ap.add_argument("--serve-saturated", type=int, default=40, help="frame-sets per rig in the saturated run")
    ap.add_argument("--serve-speedup", type=float, default=50.0,
                    help="replay factor of the accelerated serving run (30 fps per rig times this)")
    ap.add_argument("--serve-accel-seconds", type=float, default=0.5,
                    help="wall-clock seconds of the accelerated serving run")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle work per CPU-baseline leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (the correction of one rig "
              f"runs on one device; across GPUs the path would shard by camera, one arc of the ring per GPU, "
              f"exchanging only the facing band statistics of the seams between arcs)", file=sys.stderr)
        return 2

    import torch
    from paper_1910_03517_amd import rt

    torch.cuda.set_device(0)
    rig_spec = config(args.config)
    timing_every = args.timing_every
    if args.copy_only:
        cams = [rt.Camera(c.width, c.height, c.channels, c.bit_depth, c.ring, c.pos).with_pitch()
                for c in rig_spec.cams]
        frame_bytes = apply_bytes(cams) // 2
        gbs = copy_ceiling(rt, torch, frame_bytes, args.nbuf, args.steps, args.warmup)
        print(json.dumps({"copy_bytes_per_launch": 2 * frame_bytes, "copy_GBs": round(gbs, 1)}), flush=True)
        return 0

    rig, rep, ins, outs, base = plain_leg(args, rig_spec, args.steps, args.warmup, timing_every)
    khash = kernel_hash()
    workload = rig_spec.name
    roof = rep.pop("roofline")
    per_set = traffic_from_profile(khash, workload, roof["kernel"].split()[0])
    roof["traffic"] = round(per_set * roof["frame_sets_per_launch"]) if per_set else None
    out = {
        "metric": METRIC, "value": rep["GPix_s"], "unit": "GPix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rep["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": workload, "path": "plain", "mode": "smoothing" if args.smoothing else "standard",
                   "launch_mode": args.mode + (f", {rep['lanes']} apply lanes, depth {args.depth}, group {rep['group']}"
                                               + (", fused applies" if rep["fuse"] else "")
                                               if args.mode == "pipe" else ""),
                   "n_blocks": rep["n_blocks"], "band_width": rep["band_width"],
                   "pixels_per_frameset": rep["pixels_per_frameset"], "rotating_buffers": args.nbuf,
                   "tile_rows": rep["tile_rows"], "apply_grid": rep["apply_grid"], "n_tiles": rep["n_tiles"]},
        "hbm_frac": rep["hbm_frac"],
        "algorithmic_bytes_per_frameset": rep["algorithmic_bytes_per_frameset"],
        "latency_ms": rep["latency_ms"],
        "wall_s": rep["wall_s"],
        "host_issue_us_per_step": rep["host_issue_us_per_step"],
        "roofline": roof,
        "kernel_hash": khash,
        "tuned": rep["tuned"],
    }
    if args.config == "rig14" and not args.no_vga:
        log("vga calls")
        out["vga"] = vga_leg()
    if args.config == "rig14" and not args.no_removal:
        log("object removal and seam monitor")
        out["removal"] = removal_leg(rig, ins, outs, rep["lanes"], rep["group"], bool(rep["fuse"]))
    sur_w = None
    if not args.no_surrogate and args.config == "rig14":
        sur_w, out["surrogate"] = surrogate_leg(args, rig, ins, outs)
    rig.close()
    del ins, outs
    if not args.no_serving and args.config == "rig14":
        out["serving"] = serving_leg(args, base, sur_w)
    if not args.no_uneven and args.config == "rig14":
        # The uneven three-ring rig (4 x 4096x2160 RGB8, 8 x 1920x1080 RGB8,
        # 4 x 640x512 gray16) in the same launch configuration.
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        us = args.uneven_steps or args.steps
        urig, urep, _, _, _ = plain_leg(args, config("uneven"), us, args.warmup, args.timing_every)
        urig.close()
        uroof = urep.pop("roofline")
        out["uneven"] = {**urep, "steps": us, "roofline": {k: uroof[k] for k in (
            "achieved", "frac", "launch_us", "launches_timed", "copy_ceiling_GBs", "alone", "per_step")}}
    if args.config == "rig14" and not args.no_moving_object:
        log("moving object: standard, removal, removal with fallback, smoothing at 16 and 64 blocks")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["moving_object"] = moving_object_leg()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(rig_spec, args.smoothing, args.cpu_budget)
        log("cpu baseline (oracle, process pool over cameras)")
        out["cpu_baseline_pool"] = cpu_baseline_pool(args.config, args.smoothing, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

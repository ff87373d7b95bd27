#!/usr/bin/env python3
"""Throughput of the pose-graph optimisation on one MI355X.

One step = one pose_graph_optimize call on a resident 10-keyframe 640x480
window: 7 Gauss-Newton iterations, each with dense association and
point-to-plane residuals of all 90 ordered keyframe pairs, the 45 x 200
feature matches (20 % outliers), the fused reduction into the 60 x 60 normal
equations, the FP64 solve and the SE(3) update, then the pose read-back.
Poses are reset to the same initial values before every step.

Prints one JSON line: GN iterations/s (value), residual pixels/s, the
association kernel's achieved algorithmic bandwidth against the HBM peak
(HIP events on the library's stream during the timed steps), and the FP64
CPU oracle timed on the host on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GN iters/s + residual px/s, 10-KF 640×480 graph; learned vs plain at ≤1e-4 rad"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the association kernel: one source record (float4
# normal+depth and the packed pixel coordinate) per valid source pixel and
# ordered pair, one float4 per target pixel read
SRC_BYTES = 20
TGT_BYTES = 16
# the feature match sets run in the same launch: two float4 point records per
# feature match
FEAT_BYTES = 32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assoc_traffic.json")
# the association kernel's translation unit and the headers it includes
ASSOC_SOURCES = [os.path.join(ROOT, "paper_2108_00516_amd", "csrc", f)
                 for f in ("pg_assoc.hip", "pg_device.hpp", "pg_mlp.hpp", "pg_util.hpp")]


def kernel_sha():
    h = hashlib.sha256()
    for f in ASSOC_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def traffic_entry(workload):
    """HBM bytes per association launch of `workload` from the committed
    counter runs, only while the kernel source is the one they were taken on."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("workloads", {}).get(workload, {}).get("traffic_bytes_per_launch")


def counter_rate(roof):
    """Beside the algorithmic rate: the counters' HBM bytes per launch over the
    same launch time (the association re-reads targets from L2 and the
    memory-side cache, so its DRAM traffic is below the algorithmic bytes)."""
    t = roof.get("traffic")
    if t:
        rate = t / (roof["avg_launch_us"] * 1e-6) / 1e9
        roof["traffic_GBps"] = round(rate, 1)
        roof["traffic_frac"] = round(rate / HBM_PEAK_GBS, 4)
    return roof


def cpu_baseline(g, iters, seconds, P_gpu):
    """The FP64 oracle on the host: full optimisations of the same window for
    about `seconds` with 16 threads (the host share of one GPU on these
    machines; os.cpu_count() is reported beside it), value from the median
    run time; then at least five single-thread optimisations (median)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    threads = max(1, min(os.cpu_count() or 1, 16))
    oracle.set_threads(threads)
    pb = oracle.OracleProblem.from_synth(g)
    times = []
    t_start = time.perf_counter()
    P = None
    while True:
        t0 = time.perf_counter()
        P, st = pb.optimize(g.poses_init, iters)
        times.append(time.perf_counter() - t0)
        el = time.perf_counter() - t_start
        if (el >= seconds and len(times) >= 5) or len(times) >= 200:
            break
    worst_r = max(oracle.pose_error(P_gpu[k], P[k])[0] for k in range(g.n_frames))
    worst_t = max(oracle.pose_error(P_gpu[k], P[k])[1] for k in range(g.n_frames))
    oracle.set_threads(1)
    t1s = []
    for _ in range(5):
        t1 = time.perf_counter()
        pb.optimize(g.poses_init, iters)
        t1s.append(time.perf_counter() - t1)
    oracle.set_threads(threads)
    med = float(np.median(times))
    med1 = float(np.median(t1s))
    return dict(value=iters / med, unit="GN iters/s", cores=threads, kind="oracle",
                sample=f"{len(times)} full optimisations of the same {g.n_frames}-keyframe {g.width}x{g.height} "
                       f"window ({iters} GN iterations each) in {el:.1f} s, {threads} threads, median run "
                       f"{1000 * med:.1f} ms, {cpu_model()}",
                host_cpu_count=os.cpu_count(),
                one_thread={"value": iters / med1, "unit": "GN iters/s", "cores": 1,
                            "sample": f"5 optimisations ({iters} GN iterations each), median {med1:.2f} s"}), \
        (worst_r, worst_t)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-events", action="store_true", help="time without per-kernel events")
    ap.add_argument("--no-forms", action="store_true", help="skip the learned / BF16x3 forms")
    ap.add_argument("--forms", default="window,pcg,X,B",
                    help="forms to run: window (learned / BF16x3 on the window), pcg (matrix-free PCG), "
                         "X (20-keyframe window), B (64-window batch)")
    ap.add_argument("--assoc-reps", type=int, default=200, help="back-to-back association launches timed")
    ap.add_argument("--workload", choices=["paper", "batch"], default="paper",
                    help="paper: the 10-keyframe 640x480 window (the headline); batch: 64 uneven windows "
                         "(4-20 keyframes, 320x240 / 480x360 / 640x480) in one batched schedule")
    ap.add_argument("--graphs", type=int, default=64, help="windows in the batched workload")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="CPU processes building the batched workload's scenes (0 or 1: in this process)")
    ap.add_argument("--window", choices=["P", "X"], default="P",
                    help="paper workload window: P = 10 keyframes 640x480 (the headline), X = 20 keyframes 640x480")
    ap.add_argument("--tile", type=int, default=0, help="association tile (pixels); 0 = library choice")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="1: replay the timed steps from a captured hipGraph (default: direct launches)")
    ap.add_argument("--autotune", metavar="JSON", default="",
                    help="time every association tile for the workload, write the table to JSON and exit")
    ap.add_argument("--tune-table", default="", metavar="JSON",
                    help="autotuner table to take the association tile from (batched workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent windows shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        a = torch.arange(n, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "repeats": 5}), flush=True)
        return

    import synth
    from paper_2108_00516_amd import Config, from_synth

    graphs = None
    forms = set() if args.no_forms else set(f for f in args.forms.split(",") if f)
    if args.workload == "batch" or "B" in forms:
        # scene generation in forked CPU workers, before this process touches
        # the GPU; the workers finish and exit on their own (close + join)
        if args.gen_workers > 1:
            import multiprocessing as mp
            pool = mp.get_context("fork").Pool(min(args.gen_workers, os.cpu_count() or 1))
            graphs = pool.map(_make_batch_graph, range(args.graphs))
            pool.close()
            pool.join()
        else:
            graphs = [_make_batch_graph(k) for k in range(args.graphs)]
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    if args.workload == "batch":
        return run_batch(args, graphs)
    batch_graphs = graphs
    iters = 7
    g = synth.make_graph(args.window)
    if args.autotune:
        from paper_2108_00516_amd import autotune

        def make(tile):
            c = Config(max_frames=g.n_frames, gn_iters=iters, tile_pixels=tile)
            return [from_synth(g, c, device_inputs=True)], [g.poses_init]
        table = autotune.tune({autotune.bucket_key(g.width, g.height, g.n_frames): make},
                              log=lambda m: print(m, file=sys.stderr, flush=True))
        autotune.save(table, args.autotune)
        print(json.dumps(table), flush=True)
        return
    cfg = Config(max_frames=g.n_frames, gn_iters=iters, use_graph=args.graph, timing=0, tile_pixels=args.tile)
    pg = from_synth(g, cfg, device_inputs=True)

    def run(steps, timing):
        """steps optimize calls; returns (seconds, last stats, summed kernel ms)."""
        ms = np.zeros(5)
        launches, reads = 0, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pg.set_poses(g.poses_init)
            st = pg.optimize()
            if timing:
                ms += [st["ms_assoc"], st["ms_feature"], st["ms_reduce"], st["ms_solve"], st["ms_total"]]
                launches += st["n_assoc_launches"]
            reads.append(st["n_target_reads"])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st, ms, launches, reads

    # the timed steps of 'value' (direct launches, or the graph replay with --graph 1)
    for _ in range(args.warmup):
        pg.set_poses(g.poses_init)
        pg.optimize()
    el, st, _, _, reads = run(args.steps, False)
    src = st["src_pixels"]
    P_gpu = pg.poses
    # the association kernel alone at the starting poses (iteration 0):
    # back-to-back launches between HIP events on the library's stream
    pg.set_poses(g.poses_init)
    assoc_ms = pg.time_assoc(args.assoc_reps) if not args.no_events else None
    reads0 = float(st["n_target_reads"][0])
    # the same steps launched directly with HIP events around every kernel on
    # the library's stream: per-kernel durations for the roofline
    ev = None
    if not args.no_events:
        pg.close()
        cfg_t = Config(max_frames=g.n_frames, gn_iters=iters, use_graph=0, timing=1, tile_pixels=args.tile)
        pg = from_synth(g, cfg_t, device_inputs=True)
        for _ in range(args.warmup):
            pg.set_poses(g.poses_init)
            pg.optimize()
        ev = run(args.steps, True)
    gated = float(np.mean(st["n_valid_g"]))
    mean_reads = float(np.mean(np.concatenate(reads)))
    value = iters * args.steps / el
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GN iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{g.n_frames} keyframes, {g.width}x{g.height} depth, "
                               f"{g.n_frames * (g.n_frames - 1)} ordered pairs, {len(g.matches)} x 200 feature "
                               "matches (20% outliers), 7 Gauss-Newton iterations per step",
                   "keyframes": g.n_frames, "width": g.width, "height": g.height, "gn_iters": iters,
                   "valid_source_pixels_per_frame": [pg.frame_info(f, with_map=False)[1]
                                                     for f in range(g.n_frames)],
                   "parallelism": "single GPU"},
        "residual_px_per_s": round(src * iters * args.steps / el, 1),
        "gated_in_residuals_per_s": round(gated * iters * args.steps / el, 1),
        "hw_pixel_pairs_per_s": round(g.n_frames * (g.n_frames - 1) * g.width * g.height * iters * args.steps / el, 1),
        "source_pixels_per_iteration": int(src),
        "target_reads_per_iteration": int(round(mean_reads)),
    }
    if ev is not None:
        el_ev, _, ms_phase, n_launch, _ = ev
        avg_s = assoc_ms / 1000.0
        n_feat = sum(len(m.uv_i) for m in g.matches)
        bytes_alg = SRC_BYTES * src + TGT_BYTES * reads0 + FEAT_BYTES * n_feat
        achieved = bytes_alg / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_entry("paper_window"),
                           "kernel": "assoc_kernel", "avg_launch_us": round(avg_s * 1e6, 3),
                           "launches_timed": args.assoc_reps,
                           "algorithmic_bytes_per_launch": int(bytes_alg),
                           "in_step_avg_launch_us": round(ms_phase[0] / n_launch * 1000.0, 3),
                           "frac_in_step": round(bytes_alg / (ms_phase[0] / n_launch / 1000.0) / 1e9 / HBM_PEAK_GBS,
                                                 4)}
        counter_rate(out["roofline"])
        out["events_pass"] = {"ms_per_step": round(1000.0 * el_ev / args.steps, 4),
                              "gpu_ms_per_step": {k: round(v / args.steps, 4) for k, v in
                                                  zip(["assoc", "feature", "assemble", "solve", "total"],
                                                      ms_phase)}}
    if not args.no_cpu_baseline:
        cb, (dr, dt) = cpu_baseline(g, iters, args.cpu_seconds, P_gpu)
        out["cpu_baseline"] = cb
        out["max_pose_diff_vs_oracle"] = {"rad": dr, "m": dt}
    pg.close()
    if forms:
        out["forms"] = other_forms(g, iters, P_gpu, min(args.steps, 50), args.tile) if "window" in forms else {}
        if "pcg" in forms:
            out["forms"]["pcg_matrix_free"] = matrix_free_form(g, iters, P_gpu, min(args.steps, 20))
        if "X" in forms:
            out["forms"]["window_X"] = window_x_form(iters, min(args.steps, 20))
        if "B" in forms:
            out["forms"]["batch_B"] = batch_forms(batch_graphs, iters, min(args.steps, 10))
    print(json.dumps(out), flush=True)


WEIGHTS = os.path.join(ROOT, "paper_2108_00516_amd", "weights", "weightnet.npy")


def other_forms(g, iters, P_plain, steps, tile):
    """The learned (25% of source pixels pruned), BF16x3 and combined forms on
    the same window: GN iterations/s over the same kind of steps and the largest
    pose difference to the plain FP32 result; pose error of each against the
    generator's ground truth."""
    import numpy as np
    import torch

    import oracle
    from paper_2108_00516_amd import Config, _lib, from_synth
    trained = os.path.exists(WEIGHTS)
    if trained:
        p16 = np.load(WEIGHTS, allow_pickle=False).astype(np.float16)
    else:
        from paper_2108_00516_amd.learn import init_params
        p16 = init_params(0).astype(np.float16)

    def gt_err(P):
        e = [oracle.pose_error(P[k], g.poses_gt[k]) for k in range(g.n_frames)]
        return {"rad": max(x[0] for x in e), "m": max(x[1] for x in e)}

    res = {"weights": "trained (learn.py)" if trained else "untrained initialisation",
           "plain_fp32": {"error_vs_ground_truth": gt_err(P_plain)}}
    for name, kw in [("learned", dict(weighting=_lib.PG_WEIGHT_LEARNED, prune_frac=0.25)),
                     ("bf16x3", dict(precision=_lib.PG_PREC_BF16X3)),
                     ("learned_bf16x3", dict(weighting=_lib.PG_WEIGHT_LEARNED, prune_frac=0.25,
                                             precision=_lib.PG_PREC_BF16X3)),
                     ("persistent_association", dict(persistent=1))]:
        pg = from_synth(g, Config(max_frames=g.n_frames, gn_iters=iters, tile_pixels=tile, **kw),
                        device_inputs=True)
        if kw.get("weighting") == _lib.PG_WEIGHT_LEARNED:
            pg.set_mlp(p16)
        for _ in range(3):
            pg.set_poses(g.poses_init)
            pg.optimize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pg.set_poses(g.poses_init)
            st = pg.optimize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        P = pg.poses
        dr = max(oracle.pose_error(P[k], P_plain[k])[0] for k in range(g.n_frames))
        dt = max(oracle.pose_error(P[k], P_plain[k])[1] for k in range(g.n_frames))
        res[name] = {"gn_iters_per_s": round(iters * steps / el, 2), "ms_per_step": round(1000 * el / steps, 4),
                     "source_pixels_per_iteration": int(st["src_pixels"]),
                     "max_pose_diff_vs_plain": {"rad": dr, "m": dt}, "meets_1e-4": bool(dr <= 1e-4 and dt <= 1e-4),
                     "error_vs_ground_truth": gt_err(P)}
        if name == "persistent_association":
            res[name]["poses_equal_plain"] = bool(np.array_equal(P, P_plain))
            res[name]["assoc_us_per_launch"] = round(1000 * pg.time_assoc(200), 3)
        pg.close()
    return res


def matrix_free_form(g, iters, P_plain, steps):
    """The 10-keyframe window with the matrix-free PCG (J^T W J applied from
    per-pair Gram blocks, never assembled): GN iterations/s, PCG iterations
    per GN iteration, pose difference to the direct solve."""
    import numpy as np
    import torch

    import oracle
    from paper_2108_00516_amd import Config, _lib, from_synth
    pg = from_synth(g, Config(max_frames=g.n_frames, gn_iters=iters, solver=_lib.PG_SOLVER_PCG_MATRIX_FREE),
                    device_inputs=True)
    for _ in range(3):
        pg.set_poses(g.poses_init)
        pg.optimize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pg.set_poses(g.poses_init)
        st = pg.optimize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    P = pg.poses
    pg.close()
    return {"gn_iters_per_s": round(iters * steps / el, 2), "ms_per_step": round(1000 * el / steps, 4),
            "pcg_iters_per_gn_iter": [int(x) for x in st["pcg_iters"]],
            "max_pose_diff_vs_direct": {"rad": max(oracle.pose_error(P[k], P_plain[k])[0] for k in range(len(P))),
                                        "m": max(oracle.pose_error(P[k], P_plain[k])[1] for k in range(len(P)))}}


def window_x_form(iters, steps):
    """The 20-keyframe 640x480 window (380 ordered pairs), plain FP32."""
    import torch

    import synth
    from paper_2108_00516_amd import Config, from_synth
    gx = synth.make_graph("X")
    pg = from_synth(gx, Config(max_frames=gx.n_frames, gn_iters=iters), device_inputs=True)
    for _ in range(3):
        pg.set_poses(gx.poses_init)
        pg.optimize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pg.set_poses(gx.poses_init)
        st = pg.optimize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pg.close()
    return {"keyframes": gx.n_frames, "gn_iters_per_s": round(iters * steps / el, 2),
            "ms_per_step": round(1000 * el / steps, 4), "source_pixels_per_iteration": int(st["src_pixels"]),
            "residual_px_per_s": round(st["src_pixels"] * iters * steps / el, 1)}


def batch_forms(graphs, iters, steps):
    """The 64 uneven windows (4-20 keyframes, 320x240 / 480x360 / 640x480) in
    one batched schedule: plain FP32 (graph-iterations/s, the association's
    algorithmic bytes over its launch time from HIP events), then the same
    batch with BF16x3 and with learned weighting + BF16x3 (the metric's
    learned + batched + mixed-precision form), each against the plain batch:
    largest pose difference over all windows and whether it is within
    1e-4 rad / 1e-4 m."""
    import numpy as np
    import torch

    from paper_2108_00516_amd import Config, _lib, from_synth, optimize_batch
    trained = os.path.exists(WEIGHTS)
    if trained:
        p16 = np.load(WEIGHTS, allow_pickle=False).astype(np.float16)
    else:
        from paper_2108_00516_amd.learn import init_params
        p16 = init_params(0).astype(np.float16)
    import oracle

    def build(timing=0, **kw):
        pgs = []
        for g in graphs:
            pg = from_synth(g, Config(max_frames=g.n_frames, gn_iters=iters, timing=timing, **kw),
                            device_inputs=True)
            if kw.get("weighting") == _lib.PG_WEIGHT_LEARNED:
                pg.set_mlp(p16)
            pgs.append(pg)
        return pgs

    def timed(pgs):
        for _ in range(2):
            optimize_batch(pgs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for pg, g in zip(pgs, graphs):
                pg.set_poses(g.poses_init)
            rc, st = optimize_batch(pgs)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    pgs = build()
    el, st = timed(pgs)
    plain = [pg.poses for pg in pgs]
    src = sum(x["src_pixels"] for x in st)
    reads = sum(float(np.mean(x["n_target_reads"])) for x in st)
    for pg in pgs:
        pg.close()
    out = {"windows": len(graphs), "keyframes_total": int(sum(g.n_frames for g in graphs)),
           "plain_fp32": {"graph_gn_iters_per_s": round(iters * len(graphs) * steps / el, 2),
                          "ms_per_step": round(1000 * el / steps, 4), "source_pixels_per_iteration": int(src)}}
    # the association's launch time from HIP events around each kernel
    pgs = build(timing=1)
    for _ in range(2):
        optimize_batch(pgs)
    launches, ms = 0, 0.0
    for _ in range(steps):
        for pg, g in zip(pgs, graphs):
            pg.set_poses(g.poses_init)
        rc, st = optimize_batch(pgs)
        launches += st[0]["n_assoc_launches"]
        ms += st[0]["ms_assoc"]
    for pg in pgs:
        pg.close()
    n_feat = sum(len(m.uv_i) for g in graphs for m in g.matches)
    bytes_alg = SRC_BYTES * src + TGT_BYTES * reads + FEAT_BYTES * n_feat
    avg_s = ms / launches / 1000.0
    out["plain_fp32"]["assoc_avg_launch_us"] = round(avg_s * 1e6, 2)
    out["plain_fp32"]["assoc_algorithmic_bytes_per_launch"] = int(bytes_alg)
    out["plain_fp32"]["assoc_algorithmic_GBps"] = round(bytes_alg / avg_s / 1e9, 1)
    # the counters' HBM bytes: the batch's sources re-read their targets from
    # L2 and the memory-side cache, so the algorithmic rate can pass the HBM peak
    traffic = traffic_entry("batch64")
    out["plain_fp32"]["assoc_hbm_bytes_per_launch"] = traffic
    out["plain_fp32"]["assoc_hbm_GBps"] = round(traffic / avg_s / 1e9, 1) if traffic else None
    # the same batch replayed as one captured hipGraph, and with one tile
    # (1024 pixels) for every window instead of the tuned per-class tiles
    from paper_2108_00516_amd import autotune
    shipped = autotune.load(autotune.TABLE_PATH)
    out["plain_fp32"]["tiles"] = sorted({f"{g.width}x{g.height}/{g.n_frames}": autotune.lookup(
        shipped, g.width, g.height, g.n_frames, 1024) for g in graphs}.items())
    for name, kw in [("graph_replay", dict(use_graph=1)), ("uniform_tile_1024", dict(tile_pixels=1024)),
                     ("persistent_association", dict(persistent=1))]:
        pgs = build(**kw)
        el2, _ = timed(pgs)
        same = all(np.array_equal(pg.poses, P0) for pg, P0 in zip(pgs, plain))
        for pg in pgs:
            pg.close()
        out[name] = {"graph_gn_iters_per_s": round(iters * len(graphs) * steps / el2, 2),
                     "ms_per_step": round(1000 * el2 / steps, 4), "speedup_vs_plain": round(el / el2, 3),
                     "poses_equal_plain": bool(same) if name != "uniform_tile_1024" else None}
    for name, kw in [("bf16x3", dict(precision=_lib.PG_PREC_BF16X3)),
                     ("learned_bf16x3", dict(weighting=_lib.PG_WEIGHT_LEARNED, prune_frac=0.25,
                                             precision=_lib.PG_PREC_BF16X3))]:
        pgs = build(**kw)
        el2, _ = timed(pgs)
        P = [pg.poses for pg in pgs]
        for pg in pgs:
            pg.close()
        dr = max(oracle.pose_error(a, b)[0] for Pa, Pb in zip(P, plain) for a, b in zip(Pa, Pb))
        dt = max(oracle.pose_error(a, b)[1] for Pa, Pb in zip(P, plain) for a, b in zip(Pa, Pb))
        out[name] = {"graph_gn_iters_per_s": round(iters * len(graphs) * steps / el2, 2),
                     "ms_per_step": round(1000 * el2 / steps, 4), "speedup_vs_plain": round(el / el2, 3),
                     "max_pose_diff_vs_plain": {"rad": dr, "m": dt},
                     "meets_1e-4": bool(dr <= 1e-4 and dt <= 1e-4)}
    return out


def _make_batch_graph(k):
    import synth
    return synth.make_graph(f"B{k}")


def run_batch(args, graphs):
    """64 independent windows of uneven node counts (4-20) and resolutions in
    one batched schedule: one launch per phase for all graphs, 7 iterations
    per step (direct launches, or one hipGraph with --graph 1).  value = graph-iterations per second
    (GN iterations summed over the graphs)."""
    import numpy as np
    import torch

    from paper_2108_00516_amd import Config, from_synth, optimize_batch
    iters = 7

    tile = args.tile
    if tile == 0 and args.tune_table:
        from paper_2108_00516_amd import autotune
        tile = autotune.load(args.tune_table).get(autotune.BATCH_KEY, {}).get("tile", 0)

    def build(timing):
        return [from_synth(g, Config(max_frames=g.n_frames, gn_iters=iters, use_graph=0 if timing else args.graph,
                                     timing=1 if timing else 0, tile_pixels=tile), device_inputs=True)
                for g in graphs]

    def run(pgs, steps):
        launches, ms, reads, src = 0, np.zeros(5), 0.0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for pg, g in zip(pgs, graphs):
                pg.set_poses(g.poses_init)
            rc, st = optimize_batch(pgs)
            s0 = st[0]
            launches += s0["n_assoc_launches"]
            ms += [s0["ms_assoc"], s0["ms_feature"], s0["ms_reduce"], s0["ms_solve"], s0["ms_total"]]
            reads = sum(float(np.mean(x["n_target_reads"])) for x in st)
            src = sum(x["src_pixels"] for x in st)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, launches, ms, reads, src

    if args.autotune:
        # per window class: its largest window alone with every tile; then the
        # best single tile for the whole batch (recorded, not used by the library)
        from paper_2108_00516_amd import autotune
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731

        def make_one(g, tile):
            return ([from_synth(g, Config(max_frames=g.n_frames, gn_iters=iters, tile_pixels=tile),
                                device_inputs=True)], [g.poses_init])

        def make(tile):
            return ([from_synth(g, Config(max_frames=g.n_frames, gn_iters=iters, tile_pixels=tile),
                                device_inputs=True) for g in graphs], [g.poses_init for g in graphs])
        # a batch runs at the largest pixels per thread of its graphs, so the
        # classes are tuned among the tiles that share the best uniform tile's
        table = autotune.tune({autotune.BATCH_KEY: make}, steps=5, log=log)
        best = table[autotune.BATCH_KEY]["tile"]
        same = [t for t in autotune.TILES if autotune.pixels_per_thread(t) == autotune.pixels_per_thread(best)]
        table.update(autotune.tune_classes(graphs, make_one, tiles=same, steps=10, log=log))
        # the batch with the class tiles against the uniform tile
        autotune.apply(table)
        t_cls = autotune.time_optimize(lambda t: make(0), 0, steps=5)
        t_uni = autotune.time_optimize(make, best, steps=5)
        table[autotune.BATCH_KEY]["check_ms"] = {"class_tiles": round(t_cls, 4), "uniform": round(t_uni, 4)}
        if t_cls > t_uni:
            # no gain in the batch: every class takes the uniform tile
            for k in table:
                if k != autotune.BATCH_KEY:
                    table[k]["tile"] = best
        autotune.save(table, args.autotune)
        print(json.dumps(table), flush=True)
        return
    pgs = build(False)
    for _ in range(args.warmup):
        optimize_batch(pgs)
    el, _, _, reads, src = run(pgs, args.steps)
    for pg in pgs:
        pg.close()
    out = {
        "metric": "batched GN graph-iterations/s (64 uneven windows)",
        "value": round(iters * len(graphs) * args.steps / el, 2),
        "unit": "graph GN iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(graphs)} windows, 4-20 keyframes, 320x240/480x360/640x480, 7 GN iterations",
                   "tile_pixels": tile,
                   "keyframes": [g.n_frames for g in graphs],
                   "resolutions": [f"{g.width}x{g.height}" for g in graphs]},
        "residual_px_per_s": round(src * iters * args.steps / el, 1),
        "source_pixels_per_iteration": int(src),
    }
    if not args.no_events:
        pgs = build(True)
        for _ in range(args.warmup):
            optimize_batch(pgs)
        _, launches, ms, reads, src = run(pgs, args.steps)
        for pg in pgs:
            pg.close()
        avg_s = ms[0] / launches / 1000.0
        n_feat = sum(len(m.uv_i) for g in graphs for m in g.matches)
        bytes_alg = SRC_BYTES * src + TGT_BYTES * reads + FEAT_BYTES * n_feat
        achieved = bytes_alg / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_entry("batch64"),
                           "kernel": "assoc_kernel",
                           "avg_launch_us": round(avg_s * 1e6, 3), "algorithmic_bytes_per_launch": int(bytes_alg)}
        counter_rate(out["roofline"])
        out["events_pass"] = {"gpu_ms_per_step": {k: round(v / args.steps, 4) for k, v in
                                                  zip(["assoc", "feature", "assemble", "solve", "total"], ms)}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

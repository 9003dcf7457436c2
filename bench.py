#!/usr/bin/env python3
"""Benchmark of the ELAS hot path on one MI355X.

One step = one elas_process_batch call over --batch resident 640x480 pairs
with disparities 0..127 (seeded synthetic piecewise-planar scenes, pair i from
seed + i): every stage of the path (descriptor, support matching and
filtering, support lists, device mesh, prior raster, dense matching of both
views, final left/right check) runs once for all pairs of the step, one
launch per stage, from a captured graph. Consecutive steps are issued
round-robin on --streams HIP streams, so up to streams x batch frames are in
flight (each stream has its own buffers in the library); the process asks HIP
for --hw-queues hardware queues. With --batch 1 a step is one elas_process
call on one pair. Prints one JSON line.

value           frames/s over the timed steps (inputs already in HBM)
fps_plain_calls one elas_process call per pair (pair seed), round-robin on
                --plain-streams streams
fps_one_stream  the same plain calls on a single stream (one frame at a time)
roofline        the kernel with the largest share of chip time in a step
                (duration x the fraction of the 256 CUs it occupies; the mesh
                kernel holds one CU per view and pair), its algorithmic work
                per launch over its mean duration (HIP events on the stream the
                library launches on), against the MI355X peak
batch           96 pairs of mixed resolutions and disparity ranges (seeded
                synthetic, pair i from seed i), one batched call each repetition,
                against 96 sequential plain calls
serve           16 camera streams with Poisson arrivals at the six swept
                aggregate rates 200..2000 pairs/s and one beyond them: p50/p99
                latency and sustained pairs/s of the batching server and of the
                one-pair-at-a-time server
variants        frames/s of the same pair under the embedded variant and the
                optional steps (census descriptors, eq. 3, past-only redundancy,
                support down-sampling, median filter), each bit-exact to the
                oracle in the test-suite (plain calls on --plain-streams streams)
cpu_baseline    the CPU oracle (single-threaded C) on a bounded sample of the
                same workload, on this host; per stage, the median of 5 runs at
                320x240, 640x480 and 1242x375; the CPU model and core count

--mode calib runs a plain device copy of a known size (reads and writes
COPY_BYTES per launch) so that rocprofv3's FETCH_SIZE / WRITE_SIZE counters
can be scaled to bytes; profiles/ keeps the scaled per-launch traffic of the
kernels that can be dominant, each with a hash of the kernel source it was
taken on, and roofline.traffic reports it only while that source is unchanged.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fps & pixel·disparity evals/s at 640×480 D=128; served p50/p99 latency"

# MI355X peaks: 256 CUs at 2.4 GHz, 64 VALU lanes per CU per clock; v_sad_u8
# does 4 byte absolute differences (with accumulation) per lane.
PEAK_HBM_GBS = 8000.0
PEAK_SAD_TOPS = 256 * 64 * 2.4e9 * 4 / 1e12    # 157.3 T byte-|diff| per second

STAGES = ["descriptor", "support", "filter", "rows", "mesh", "raster", "dense", "lrcheck"]
KERNEL_NAMES = {"descriptor": "k_descriptor8", "support": "k_support", "filter": "k_filter",
                "rows": "k_rows", "mesh": "k_mesh", "raster": "k_raster", "dense": "k_dense_r2",
                "lrcheck": "k_check"}


COPY_BYTES = 256 << 20
CSRC = os.path.join(ROOT, "paper_1802_07210_amd", "csrc")
# the kernels' source and the headers compiled into them (the stored
# profiles carry the same hash)
KERNEL_SOURCES = [os.path.join(CSRC, n) for n in ("elas_kernels.hip", "elas_internal.h", "elas_wave.h")]
PROFILES = os.path.join(ROOT, "profiles")

# Variants measured beside the headline configuration (parameter overrides).
VARIANTS = {
    "census_9x9_5x5": dict(descriptor=1, census_support_window=9, census_dense_window=5),
    "census_13x13_7x7": dict(descriptor=1, census_support_window=13, census_dense_window=7),
    "shiftsum_eq3": dict(ambiguity=1),
    "past_only_redundancy": dict(redundancy=1),
    "support_1_of_8": dict(support_subsample=8),
    "support_1_of_32": dict(support_subsample=32),
    "median_5x5": dict(median_window=5),
    "embedded_best": dict(descriptor=1, census_support_window=9, census_dense_window=5,
                          ambiguity=1, redundancy=1, support_subsample=8, median_window=5),
}


def source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_file(kernel: str, workload: str) -> str:
    """Counter summary of one kernel on one workload (e.g. 640x480_D128, or
    640x480_D128_x8 for launches over 8 pairs)."""
    return os.path.join(PROFILES, f"traffic_{kernel}_{workload}.json")


def stored_traffic(kernel: str, workload: str = "640x480_D128"):
    """Per-launch HBM bytes of `kernel` on `workload` from the committed
    counter runs, or None when there are none or they were taken on another
    version of the kernel source."""
    try:
        with open(traffic_file(kernel, workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("source_sha256_16") != source_hash():
        return None
    return t.get("bytes_per_launch")


def copy_calibration(torch, reps: int = 20):
    """A plain copy kernel of known size (neg of a float32 buffer: COPY_BYTES
    read and COPY_BYTES written per launch)."""
    dev = torch.device("cuda:0")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "calib", "copy_bytes_read": COPY_BYTES,
                      "copy_bytes_written": COPY_BYTES, "launches": reps}), flush=True)


def variant_fps(torch, Elas, L, R, D, steps: int, streams):
    """Frames/s of each variant on the bench pair, same stream round-robin."""
    H, W = L.shape
    dev = L.device
    K = len(streams)
    outs = [(torch.empty((H, W), dtype=torch.int16, device=dev),
             torch.empty((H, W), dtype=torch.int16, device=dev)) for _ in range(K)]
    res = {}
    for name, kw in VARIANTS.items():
        e = Elas(disp_max=D - 1, **kw)
        for i in range(max(8, K)):
            e.process(L, R, outs[i % K][0], outs[i % K][1], stream=streams[i % K])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            e.process(L, R, outs[i % K][0], outs[i % K][1], stream=streams[i % K])
        torch.cuda.synchronize()
        fps = steps / (time.perf_counter() - t0)
        st = e.stats()
        res[name] = {"fps": round(fps, 1), "params": kw,
                     "support_points": [st["n_support_left"], st["n_support_right"]],
                     "evals_per_frame": st["support_evals"] + st["dense_evals"]}
        e.close()
    return res


def algorithmic_work(stage: str, w: int, h: int, st: dict, pairs: int = 1):
    """(HBM bytes, byte-|diff| ops) one launch of a stage's kernel over `pairs`
    pairs of w x h must move and compute, counted from the algorithm (not
    from the counters); st: the pairs' statistics summed, lattice sizes per
    pair."""
    npx = w * h * pairs
    if stage == "descriptor":   # read 1 B image, write a 16 B descriptor; 2 views
        return 2 * npx * (1 + 16), 0
    if stage == "support":      # descriptor rows v-2 and v+2 of each lattice row, 2 views;
        # 64 byte-|diff| per 512-bit evaluation
        return 2 * 2 * 16 * w * max(1, st.get("lattice_rows", 0)) * pairs, 64 * st["support_evals"]
    if stage == "dense":        # own descriptor 16 B + prior 2 B read, raw 2 B written;
        return 2 * npx * (16 + 2 + 2), 16 * st["dense_evals"]       # 2 views
    if stage == "lrcheck":      # read 2 B + partner 2 B, write 2 B per pixel, 2 views
        return 2 * npx * 6, 0
    if stage == "raster":       # a 4 B owner and a 2 B prior per pixel, 2 views
        return 2 * npx * 6, 0
    if stage == "filter":       # lattice read + three lattice writes
        return 8 * max(1, st.get("lattice", 0)) * pairs, 0
    if stage == "rows":         # final lattice + evaluation counts read, lists written
        return 6 * max(1, st.get("lattice", 0)) * pairs, 0
    if stage == "mesh":         # support points in, raster records out (24 B per triangle)
        n = st["n_support_left"] + st["n_support_right"]
        return 12 * n + 24 * (st["n_tri_left"] + st["n_tri_right"]), 0
    return 0, 0


def workgroups(w: int, h: int, D: int, step: int = 5) -> dict:
    """Workgroups each stage launches for one frame (default tile variants)."""
    cd = lambda a, b: -(-a // b)
    lw, lh = (w - 5) // step, (h - 5) // step
    return {"descriptor": 2 * cd(w, 128) * cd(h, 8), "support": lh * cd(lw, 32 if D <= 192 else 16),
            "filter": (cd(lw, 8) * cd(lh, 8) if cd(lw, 8) * cd(lh, 8) <= 256
                       else cd(lw, 16) * cd(lh, 16)), "rows": lh, "mesh": 2,
            "raster": 2 * cd(h, max(1, min(4, 4096 // w))),
            "dense": 2 * cd(h, 2) * cd(w, 256), "lrcheck": 2 * cd(w * h, 1024)}


VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions per second (4 cycles each)


def stored_valu(kernel: str, workload: str = "640x480_D128"):
    """VALU instructions per launch of `kernel` on `workload` from the
    committed SQ counter run, or None (none, or another kernel source)."""
    try:
        with open(os.path.join(PROFILES, f"valu_{workload}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != source_hash():
        return None
    rec = t.get("kernels", {}).get(kernel)
    return rec.get("sq_insts_valu") if rec else None


def roofline_of(stage: str, w: int, h: int, st: dict, ms: float, kernel: str,
                pairs: int = 1, workload: str = "640x480_D128") -> dict:
    """The binding roofline of one kernel: the resource whose floor (work over
    peak) is the larger; achieved = that work over the kernel's mean duration.
    st holds the statistics summed over the `pairs` pairs of one launch."""
    nbytes, ops = algorithmic_work(stage, w, h, st, pairs)
    dur_s = ms / 1e3
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    t_alu = ops / (PEAK_SAD_TOPS * 1e12)
    if t_alu > t_hbm:
        achieved, peak, unit, bound, work, wunit = (ops / dur_s / 1e12, PEAK_SAD_TOPS, "Tops/s",
                                                    "alu", ops, "byte-|diff| (v_sad_u8: 4 per lane)")
    else:
        achieved, peak, unit, bound, work, wunit = (nbytes / dur_s / 1e9, PEAK_HBM_GBS, "GB/s",
                                                    "hbm", nbytes, "bytes")
    roof = {"bound": bound, "achieved": round(achieved, 4), "peak": round(peak, 1),
            "unit": unit, "frac": round(achieved / peak, 6), "traffic": stored_traffic(kernel, workload),
            "kernel": kernel, "kernel_ms": round(ms, 5), "work_per_launch": work,
            "work_unit": wunit}
    valu = stored_valu(kernel, workload)
    if valu:  # the share of the chip's VALU instruction issue this launch used
        roof["valu_issue"] = {"insts_per_launch": round(valu), "achieved": round(valu / dur_s / 1e9, 2),
                              "peak": round(VALU_ISSUE_PEAK / 1e9, 1), "unit": "G wave64 instr/s",
                              "frac": round(valu / dur_s / VALU_ISSUE_PEAK, 4)}
    if bound == "hbm" and ops:
        roof["alu_view"] = {"achieved": round(ops / dur_s / 1e12, 4), "peak": round(PEAK_SAD_TOPS, 1),
                            "unit": "Tops/s", "frac": round(ops / dur_s / 1e12 / PEAK_SAD_TOPS, 6),
                            "work_per_launch": ops}
    return roof


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


ORACLE_STAGES = ("descriptor", "support_match_filter_lists", "triangulate_plane_raster", "grid",
                 "dense", "lrcheck")


def cpu_baseline(left, right, disp_max, budget_s=12.0, max_frames=200):
    """The oracle on this host: frames/s of the bench pair over a bounded
    sample (one thread), and per stage the median of 5 runs (monotonic clock)
    at the three single-frame workload shapes."""
    import synth
    from oracle import ref   # the CPU oracle, timed as a reported baseline
    p = ref.params(disp_max=disp_max)
    ref.process(p, left[:64, :64].copy(), right[:64, :64].copy())  # load + warm
    n, t0 = 0, time.perf_counter()
    while n < max_frames:
        ref.process(p, left, right)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    h, w = left.shape
    per_config = {}
    for name in ("320x240", "640x480", "1242x375"):
        cfg = synth.SHAPES[name]
        pr = synth.make_pair(cfg)
        pc = ref.params(disp_max=cfg.disp_range - 1)
        runs = [ref.process(pc, pr.left, pr.right).stage_ms for _ in range(5)]
        med = [float(np.median([r[k] for r in runs])) for k in range(len(ORACLE_STAGES))]
        per_config[f"{name} D={cfg.disp_range}"] = {
            "stage_ms_median_of_5": {k: round(v, 3) for k, v in zip(ORACLE_STAGES, med)},
            "frame_ms": round(sum(med), 3), "fps": round(1000.0 / sum(med), 3)}
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} full {w}x{h} D={disp_max + 1} frames of the bench pair, "
                      f"{dt:.1f} s, single-threaded C oracle (-O2), {cpu_model()}",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "usable_cores": usable,
            "per_config": per_config}


def batch_c4(torch, Elas, reps=5, n=96):
    """C4: n pairs, resolutions uniform over the four shapes (index stream
    seeded 0), pair i generated from seed i; one batched call per repetition
    against n sequential plain calls on one stream."""
    import synth
    names = synth.batch_shapes(n, 0)
    dev = torch.device("cuda:0")
    hs = {}
    items, seq_outs, mix = [], [], {}
    for i, nm in enumerate(names):
        cfg = synth.SHAPES[nm].with_seed(i)
        pair = synth.make_pair(cfg)
        D = cfg.disp_range
        if D not in hs:
            hs[D] = Elas(disp_max=D - 1)
        L = torch.from_numpy(pair.left).to(dev)
        R = torch.from_numpy(pair.right).to(dev)
        H, W = pair.left.shape
        mk = lambda: torch.empty((H, W), dtype=torch.int16, device=dev)
        items.append((L, R, mk(), mk(), hs[D]))
        seq_outs.append((mk(), mk()))
        mix[nm] = mix.get(nm, 0) + 1
    base = hs[128] if 128 in hs else next(iter(hs.values()))
    base.set_batch_flags(graph=True, autotune=True)
    s0 = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    base.process_batch(items, stream=s0)      # autotunes new sizes, captures the graph
    base.process_batch(items, stream=s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        base.process_batch(items, stream=s0)
    torch.cuda.synchronize()
    fps_batch = reps * n / (time.perf_counter() - t0)

    def sequential():
        for (L, R, _, _, e), (oL, oR) in zip(items, seq_outs):
            e.process(L, R, oL, oR, stream=s0)

    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sequential()
    torch.cuda.synchronize()
    fps_seq = reps * n / (time.perf_counter() - t0)
    same = all(torch.equal(a[2], b[0]) and torch.equal(a[3], b[1])
               for a, b in zip(items, seq_outs))
    evals = 0
    for (L, R, _, _, e), (oL, oR) in zip(items, seq_outs):
        e.process(L, R, oL, oR, stream=s0)
        st = e.stats()
        evals += st["support_evals"] + st["dense_evals"]
    tuned = {}
    for nm in mix:
        cfg = synth.SHAPES[nm]
        try:
            tuned[nm] = list(base.tuned_variants(cfg.width, cfg.height)) \
                if cfg.disp_range == 128 else None
        except Exception:
            tuned[nm] = None
    return {"pairs": n, "mix": mix, "reps": reps, "value": round(fps_batch, 2),
            "unit": "frames/s", "sequential_fps": round(fps_seq, 2),
            "speedup_vs_sequential": round(fps_batch / fps_seq, 3),
            "evals_per_s_algorithmic": round(evals * fps_batch / n, 1),
            "identical_to_sequential": bool(same),
            "graph": True, "autotune": True,
            "tuned_desc_rows_dense_rows_support_run_at_D128": tuned}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="640x480")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--streams", type=int, default=2,
                    help="steps are issued round-robin on this many streams")
    ap.add_argument("--batch", type=int, default=32,
                    help="pairs per step (one batched call); 1: one plain call per step")
    ap.add_argument("--plain-streams", type=int, default=3,
                    help="streams of the plain-call and variant rates (one elas_process "
                         "call per pair)")
    ap.add_argument("--hw-queues", type=int, default=4,
                    help="hardware queues of this process (GPU_MAX_HW_QUEUES, read when HIP "
                         "starts; 4 is HIP's default); 0 keeps the environment's value")
    ap.add_argument("--mode", choices=["frame", "serve", "calib"], default="frame",
                    help="frame: the 640x480 frame rate (default); serve: the camera-stream "
                         "serving sweep (batched and plain servers); calib: a plain copy "
                         "kernel of known size for scaling the PMC byte counters")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the per-variant frame rates")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the short serving sweep of the default run")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="seconds per arrival-rate level in --mode serve")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 96-pair batched measurement")
    ap.add_argument("--mesh-on-host", action="store_true",
                    help="triangulate on the host between the GPU phases (the paper's split)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the ELAS path runs on a single MI355X "
              "(frames are independent, so more GPUs would each take whole frames)",
              file=sys.stderr)
        sys.exit(2)

    if args.hw_queues > 0:
        # HIP maps the process's streams onto this many hardware queues
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))
    import torch
    import synth
    from paper_1802_07210_amd import Elas

    if args.mode == "calib":
        copy_calibration(torch)
        return

    if args.mode == "serve":
        from paper_1802_07210_amd import serve
        cams, handles = serve.build_cameras()
        # the swept rates 200..2000 pairs/s, then rates beyond what one pair
        # at a time can sustain, where continuous batching shows
        rates = (200, 400, 800, 1200, 1600, 2000, 4000, 8000, 12000)
        batched = serve.run_sweep(rates=rates, seconds=args.serve_seconds, cams=cams,
                                  handles=handles)
        plain = serve.run_sweep(rates=rates, seconds=args.serve_seconds, plain=True, cams=cams,
                                handles=handles)
        top = [lv for lv in batched["levels"] if lv["rate"] == 2000][0]
        print(json.dumps({
            "metric": METRIC, "mode": "serve", "value": top["sustained_pairs_per_s"],
            "unit": "pairs/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
            "dtype": "u8", "data": "synthetic",
            "config": {"workload": "16 camera streams, camera j at shape j mod 4 (320x240 D64, "
                                   "640x480 D128, 1242x375 D256, 1280x720 D192), Poisson "
                                   "arrivals swept over aggregate rates, seconds per level "
                                   f"{args.serve_seconds}", "cameras": 16, "pool_per_camera": 4},
            "p50_ms_at_2000": top["p50_ms"], "p99_ms_at_2000": top["p99_ms"],
            "batched": batched, "plain": plain}), flush=True)
        return

    cfg = synth.SHAPES[args.workload].with_seed(args.seed)
    pair = synth.make_pair(cfg)
    W, H, D = cfg.width, cfg.height, cfg.disp_range
    dev = torch.device("cuda:0")
    B = max(1, args.batch)
    imgs = [(torch.from_numpy(pair.left).to(dev), torch.from_numpy(pair.right).to(dev))]
    for i in range(1, B):
        p = synth.make_pair(synth.SHAPES[args.workload].with_seed(args.seed + i))
        imgs.append((torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)))
    L, R = imgs[0]
    K = max(1, args.streams)
    KP = max(1, args.plain_streams)
    NS = max(K, KP)
    streams = [torch.cuda.Stream(device=dev) for _ in range(NS)]  # default priority
    outs = [[(torch.empty((H, W), dtype=torch.int16, device=dev),
              torch.empty((H, W), dtype=torch.int16, device=dev)) for _ in range(B)]
            for _ in range(NS)]
    items = [[(imgs[i][0], imgs[i][1], outs[k][i][0], outs[k][i][1]) for i in range(B)]
             for k in range(K)]
    e = Elas(disp_max=D - 1, mesh_on_host=int(args.mesh_on_host))
    e.set_batch_flags(graph=True, autotune=False)  # default tile variants
    stream = streams[0]

    def run(nsteps, nstreams):
        for i in range(nsteps):
            k = i % nstreams
            if B > 1:
                e.process_batch(items[k], stream=streams[k])
            else:
                e.process(L, R, outs[k][0][0], outs[k][0][1], stream=streams[k])

    def run_plain(nsteps, nstreams):
        for i in range(nsteps):
            k = i % nstreams
            e.process(L, R, outs[k][0][0], outs[k][0][1], stream=streams[k])

    def rate(fn, nsteps, nstreams, warm):
        fn(max(warm, nstreams), nstreams)   # allocates every stream's buffers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(nsteps, nstreams)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt = rate(run, args.steps, K, args.warmup)
    fps = args.steps * B / dt
    plain_steps = args.steps * B
    fps_plain = plain_steps / rate(run_plain, plain_steps, KP, args.warmup)
    fps_one = plain_steps / rate(run_plain, plain_steps, 1, args.warmup)
    # statistics of the pairs of a step (plain calls), summed over the pairs
    st = {}
    for (Li, Ri) in imgs:
        e.process(Li, Ri, outs[0][0][0], outs[0][0][1], stream=stream)
        for k2, v2 in e.stats().items():
            if isinstance(v2, list):
                st[k2] = [a + b for a, b in zip(st.get(k2, [0] * len(v2)), v2)]
            else:
                st[k2] = st.get(k2, 0) + v2
    st["lattice"] = ((W - 5) // 5) * ((H - 5) // 5)   # per pair
    st["lattice_rows"] = (H - 5) // 5
    evals = (st["support_evals"] + st["dense_evals"]) / B
    nominal = 2 * W * H * D

    # single-frame latency (the plain path, one frame at a time on one stream):
    # host wall time from the call to the end of its work, and the device span
    # from the first kernel's start to the last one's end (HIP events)
    lat_wall, lat_dev = [], []
    for i in range(60):
        torch.cuda.synchronize()
        e.set_timing(i >= 30)
        t0 = time.perf_counter()
        e.process(L, R, outs[0][0][0], outs[0][0][1], stream=stream)
        stream.synchronize()
        if i >= 30:
            lat_wall.append((time.perf_counter() - t0) * 1e3)
            lat_dev.append(e.timing()["device_span_ms"])
        else:
            lat_wall.append((time.perf_counter() - t0) * 1e3)
    e.set_timing(False)
    single = {"wall_ms_median": round(float(np.median(lat_wall[:30])), 4),
              "device_span_ms_median": round(float(np.median(lat_dev)), 4),
              "fps_one_stream": None}

    # per-stage device times of one step: HIP events (hipExtLaunchKernel)
    # recorded by the library on `stream` around each launch
    e.set_timing(True)
    acc = {s: [] for s in STAGES}
    host = {"host_wait_ms": [], "host_mesh_ms": [], "device_span_ms": []}
    for _ in range(args.profile_steps):
        if B > 1:
            e.process_batch(items[0], stream=stream)
        else:
            e.process(L, R, outs[0][0][0], outs[0][0][1], stream=stream)
        tm = e.timing()
        for s in STAGES:
            acc[s].append(tm[s + "_ms"])
        for k in host:
            host[k].append(tm[k])
    e.set_timing(False)
    stage_ms = {s: float(np.mean(v)) if v else float("nan") for s, v in acc.items()}
    kernel_ms = {s: stage_ms[s] for s in KERNEL_NAMES}
    names = dict(KERNEL_NAMES)
    if B > 1:  # the batched kernels (their untuned tile variants; the raster's 256 threads;
        # descriptors by non-temporal stores and loads once a batch's reach 192 MiB)
        nt = "nt" if B * 32 * W * H >= (192 << 20) else ""
        names = {s: {"raster": "k_raster256", "descriptor": "k_descriptor16" + nt,
                     "dense": "k_dense_r2" + nt}.get(s, n) + "_batch"
                 for s, n in names.items()}
    # share of chip time: duration x the fraction of the 256 CUs the kernel's
    # workgroups can occupy (launch geometry of each stage at this size)
    wgs = workgroups(W, H, D)
    chip_ms = {s: v * min(1.0, B * wgs[s] / 256.0) for s, v in kernel_ms.items()}
    dom = max(chip_ms, key=lambda k: chip_ms[k] if chip_ms[k] == chip_ms[k] else -1.0)
    wl = f"{W}x{H}_D{D}" + (f"_x{B}" if B > 1 else "")
    roof = roofline_of(dom, W, H, st, kernel_ms[dom], names[dom], pairs=B, workload=wl)

    out = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "fps_plain_calls": round(fps_plain, 2), "fps_one_stream": round(fps_one, 2),
        "single_frame": dict(single, fps_one_stream=round(fps_one, 2)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{W}x{H} D={D}, {B} stereo pair(s) per step (one batched call), "
                               f"seeded synthetic piecewise-planar scenes ({cfg.planes} planes), "
                               f"pair i from seed + i",
                   "width": W, "height": H, "disp_range": D, "pairs_per_step": B,
                   "seed": args.seed, "streams": K, "frames_in_flight": K * B,
                   "plain_call_streams": KP,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "0")) or None,
                   "mesh": "host" if args.mesh_on_host else "device"},
        "evals_per_frame": evals,
        "evals_per_s_algorithmic": round(evals * fps, 1),
        "evals_per_s_nominal": round(nominal * fps, 1),
        "support_points_per_pair": [round(st["n_support_left"] / B, 1),
                                    round(st["n_support_right"] / B, 1)],
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "host_ms": {k: round(float(np.mean(v)), 5) if v else None for k, v in host.items()},
        "roofline": roof,
    }
    if not args.no_variants:
        out["variants"] = variant_fps(torch, Elas, L, R, D, min(args.steps, 200), streams[:KP])
    if not args.no_batch:
        out["batch"] = batch_c4(torch, Elas)
    if not args.no_serve:
        # the serving sweep over the six swept rates 200..2000 pairs/s (2 s each;
        # --mode serve runs longer levels) and one rate beyond them, where one
        # pair at a time no longer keeps up: p50/p99 latency of the batched
        # server and of the plain one
        from paper_1802_07210_amd import serve
        cams, handles = serve.build_cameras()
        rates = (200, 400, 800, 1200, 1600, 2000, 12000)
        sb = serve.run_sweep(rates=rates, seconds=2.0, cams=cams, handles=handles)
        sp = serve.run_sweep(rates=rates, seconds=2.0, plain=True, cams=cams, handles=handles)
        out["serve"] = {"cameras": 16, "seconds_per_rate": 2.0,
                        "memory_budget": sb["memory_budget"],
                        "batched": [{k: lv[k] for k in ("rate", "sustained_pairs_per_s", "p50_ms",
                                                        "p99_ms", "mean_batch")}
                                    for lv in sb["levels"]],
                        "plain": [{k: lv[k] for k in ("rate", "sustained_pairs_per_s", "p50_ms",
                                                      "p99_ms")} for lv in sp["levels"]],
                        "peak_bytes_in_flight": sb["peak_bytes_in_flight"],
                        "peak_resident_bytes": sb["peak_resident_bytes"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pair.left, pair.right, D - 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Serving measurement: camera streams with Poisson arrivals into the
continuous-batching server (or the one-pair-at-a-time plain server).

Camera j has the resolution of shape j mod 4 (320x240 D=64, 640x480 D=128,
1242x375 D=256, 1280x720 D=192) and cycles through a small pool of seeded
synthetic pairs resident in device memory. Arrivals are a Poisson process of
the given aggregate rate; each arrival goes to a camera chosen uniformly.
Inter-arrival gaps and camera choices come from a SplitMix64 stream. Latency
is the server's submission-to-completion time; sustained throughput is
completions over the time from the first submission to the last completion.
"""
from __future__ import annotations

import math
import sys
import time
from typing import Dict, List, Sequence


def _arrivals(rate: float, seconds: float, cameras: int, seed: int):
    import synth
    rng = synth.SplitMix64(seed)
    t, out = 0.0, []
    while True:
        u = rng.uniform(2)
        t += -math.log(max(u[0], 1e-300)) / rate
        if t >= seconds:
            return out
        out.append((t, min(cameras - 1, int(u[1] * cameras))))


def build_cameras(cameras: int = 16, pool: int = 4, ring: int = 64):
    import torch
    import synth
    from .elas import Elas
    names = list(synth.SHAPES)
    dev = torch.device("cuda:0")
    handles: Dict[int, Elas] = {}
    cams = []
    for j in range(cameras):
        cfg = synth.SHAPES[names[j % len(names)]]
        D = cfg.disp_range
        if D not in handles:
            handles[D] = Elas(disp_max=D - 1)
        pairs = []
        for k in range(pool):
            p = synth.make_pair(cfg.with_seed(1000 * j + k))
            pairs.append((torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)))
        H, W = cfg.height, cfg.width
        outs = [(torch.empty((H, W), dtype=torch.int16, device=dev),
                 torch.empty((H, W), dtype=torch.int16, device=dev)) for _ in range(ring)]
        cams.append({"name": names[j % len(names)], "D": D, "pairs": pairs, "outs": outs,
                     "slot_ticket": [None] * ring, "next": 0, "count": 0})
    return cams, handles


def run_level(server, cams, handles, rate: float, seconds: float, seed: int) -> dict:
    import numpy as np
    arr = _arrivals(rate, seconds, len(cams), seed)
    lat: List[float] = []
    pending = []
    t0 = time.perf_counter()
    for t_arr, j in arr:
        while True:  # sleep, then spin, until the arrival time
            dt = t0 + t_arr - time.perf_counter()
            if dt <= 0:
                break
            if dt > 4e-4:
                time.sleep(dt - 3e-4)
        cam = cams[j]
        slot = cam["next"]
        cam["next"] = (slot + 1) % len(cam["outs"])
        prev = cam["slot_ticket"][slot]
        if prev is not None:  # the output slot is reused only once its pair is done
            lat.append(server.wait(prev))
            pending.remove(prev)
        L, R = cam["pairs"][cam["count"] % len(cam["pairs"])]
        cam["count"] += 1
        oL, oR = cam["outs"][slot]
        tk = server.submit(L, R, oL, oR, handles[cam["D"]])
        cam["slot_ticket"][slot] = tk
        pending.append(tk)
    for tk in pending:
        lat.append(server.wait(tk))
    t_end = time.perf_counter()
    for cam in cams:
        cam["slot_ticket"] = [None] * len(cam["outs"])
    lat_arr = np.array(lat) if lat else np.zeros(1)
    return {"rate": rate, "requests": len(arr),
            "sustained_pairs_per_s": round(len(arr) / (t_end - t0), 1),
            "p50_ms": round(float(np.percentile(lat_arr, 50)), 3),
            "p99_ms": round(float(np.percentile(lat_arr, 99)), 3),
            "mean_ms": round(float(lat_arr.mean()), 3)}


def run_sweep(rates: Sequence[float] = (200, 400, 800, 1200, 1600, 2000),
              seconds: float = 10.0, cameras: int = 16, pool: int = 4, plain: bool = False,
              max_batch: int = 32, max_inflight: int = 3, budget: int = 32 << 30,
              seed: int = 0, cams=None, handles=None) -> dict:
    from .elas import Elas, Server
    if cams is None:
        cams, handles = build_cameras(cameras, pool)
    base = Elas(disp_max=127)
    base.set_batch_flags(graph=True, autotune=True)
    server = Server(base, max_batch=max_batch, max_inflight=max_inflight,
                    memory_budget=budget, plain=plain)
    # warm every size and stream (allocations, autotuning, graph capture)
    run_level(server, cams, handles, 400.0, 1.0, seed + 999)
    levels = []
    for i, r in enumerate(rates):
        st0 = server.stats()
        lv = run_level(server, cams, handles, float(r), seconds, seed + i)
        st1 = server.stats()
        nb = st1["batches"] - st0["batches"]
        lv["mean_batch"] = round((st1["batched_pairs"] - st0["batched_pairs"]) / max(1, nb), 2)
        levels.append(lv)
        print(f"serve {'plain' if plain else 'batched'} rate {r}: {lv}", file=sys.stderr,
              flush=True)
    st = server.stats()
    server.close()
    return {"mode": "plain" if plain else "batched", "max_batch": max_batch,
            "max_inflight": max_inflight if not plain else 1, "memory_budget": budget,
            "peak_bytes_in_flight": st["peak_bytes_in_flight"],
            "peak_resident_bytes": st["peak_resident_bytes"], "levels": levels}

#!/usr/bin/env python3
"""Benchmark: VELO reconstruction events/s on one MI355X.

One step = the whole reconstruction (clustering -> track finding -> fit and
plain quality cut, all in libvelo's HIP kernels) over one batch of 1000
nominal-occupancy synthetic events already resident in device memory.

As in the paper's throughput protocol (Sec. 3.2: several CPU-thread / GPU-
stream pairs, each processing its own set of 1000 events), steps are issued
round-robin on several HIP streams, each with its own workspace, so batches
overlap on the device.  Steps rotate over several distinct batches (with
their own output buffers) so the 256 MB Infinity Cache cannot hold the
working set.

Prints one JSON line with events/s, the roofline of the dominant kernel
(stage durations from HIP events recorded on the launch streams), physics
figures of merit from generator truth, and the CPU oracle's throughput on a
bounded sample of the same events.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = ("nominal occupancy: 1000 events/batch, 26 planes, PVs/event Poisson(7.6), "
            "tracks/PV Poisson(25), 98% hit efficiency, 1-3 px clusters, noise 1e-5/px, "
            "50 urad scattering; uint32 raw words, binary32 hits and fits")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--events", type=int, default=1000, help="events per batch (one step)")
    ap.add_argument("--batches", type=int, default=8, help="distinct device-resident batches")
    ap.add_argument("--streams", type=int, default=4, help="concurrent HIP streams")
    ap.add_argument("--cpu-events", type=int, default=0,
                    help="oracle sample size (default: all generated events)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-physics", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the batched + classifier form")
    ap.add_argument("--train-events", type=int, default=5500, help="classifier training events (~1M tracks)")
    ap.add_argument("--val-events", type=int, default=2000)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the run, 4 device-to-device copies of this many MiB (calibrates HBM "
                         "byte counters against a transfer of known size)")
    return ap.parse_args()


def run_learned(args, allb, batches, bufs, streams, params, velo, torch, n_ev, R, S, phys_plain):
    """Batched form with the learned classifier fused after the fit: train the
    network on tracks the method produces on separate nominal-occupancy events
    (generator-truth labels), choose its threshold on validation events for an
    efficiency at least the plain cut's, then time the batched form (autotuned
    persistent kernels replayed as HIP graphs) over the same rotating batches."""
    from paper_1912_09161_amd import learn
    from synth import generate
    from synth.truth import Truth, efficiency_ghosts, track_labels
    dev = torch.device("cuda:0")
    workers = min(16, os.cpu_count() or 1)

    def tracks_of(b):
        px = torch.from_numpy(b.pixels.view(np.int32)).to(dev)
        off = torch.from_numpy(b.offsets.view(np.int64)).to(dev)
        out = velo.reconstruct(px, off, params=params)
        feat = velo.track_features(out["hits"], out["tracks"], out["states"], off, b.n_pixels)
        torch.cuda.synchronize()
        hits = {k: v.cpu().numpy() for k, v in out["hits"].items()}
        hits["key"] = hits["key"].view(np.uint32)
        tr = {k: v.cpu().numpy() for k, v in out["tracks"].items()}
        tr["hit_idx"] = tr["hit_idx"].view(np.uint32).reshape(-1, 26)
        slot, lab, uid, reco = track_labels(Truth(b), tr, hits, b.offsets)
        acc = out["states"]["accepted"].cpu().numpy()[slot]
        return feat[torch.from_numpy(slot).to(dev)].contiguous(), lab, uid, reco, acc

    t0 = time.time()
    F, lab, _, _, _ = tracks_of(generate("learn_train", args.train_events, workers=workers))
    trainer = learn.Trainer(F, torch.from_numpy(lab).to(dev), seed=7)
    for _ in range(8):
        trainer.epoch()
    Fv, _, uid, reco, acc = tracks_of(generate("learn_val", args.val_events, workers=workers))
    plain_val = efficiency_ghosts(uid, acc, reco)
    z = velo.mlp_infer(trainer.mlp(0.0), Fv).cpu().numpy()
    thr = learn.choose_threshold(z, uid, reco, plain_val["efficiency"])
    mlp = trainer.mlp(thr)
    train_s = time.time() - t0

    ctxs = [velo.Context() for _ in range(S)]
    wss = [velo.alloc_batched_workspace(max(b.n_pixels for b in batches), n_ev, dev) for _ in range(S)]
    lbufs = [dict(hits=B["hits"], tracks=B["tracks"], states=B["states"]) for B in bufs]

    def step(i):
        B = bufs[i % R]
        k = i % S
        lb = dict(lbufs[i % R], ws=wss[k])
        ctxs[k].reconstruct(B["px"], B["off"], params=params, mlp=mlp, bufs=lb, stream=streams[k])

    for i in range(max(args.warmup, 2 * R)):  # autotune + capture every (batch, stream) graph
        step(i)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    value = args.steps * n_ev / wall

    physics = None
    if not args.no_physics:
        b = batches[0]
        step(0)
        torch.cuda.synchronize()
        B = bufs[0]
        hits = {k: v.cpu().numpy() for k, v in B["hits"].items()}
        hits["key"] = hits["key"].view(np.uint32)
        tr = {k: v.cpu().numpy() for k, v in B["tracks"].items()}
        tr["hit_idx"] = tr["hit_idx"].view(np.uint32).reshape(-1, 26)
        slot, lab, uid, reco = track_labels(Truth(b), tr, hits, b.offsets)
        acc = B["states"]["accepted"].cpu().numpy()[slot]
        physics = {k: (round(v, 6) if isinstance(v, float) else v)
                   for k, v in efficiency_ghosts(uid, acc, reco).items()}
    cfg = ctxs[0].config()
    for c in ctxs:
        c.close()
    return dict(value=round(value, 1), ms_per_step=round(wall * 1e3 / args.steps, 5), physics=physics,
                threshold=thr, training=dict(events=args.train_events, tracks=int(F.shape[0]),
                                             epochs=8, seconds=round(train_s, 1)),
                autotuned=cfg)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); events are independent, "
              "so several GPUs would each run this benchmark on their own share.", file=sys.stderr)
        sys.exit(2)

    from synth import generate
    n_ev = args.events
    R = args.batches
    t0 = time.time()
    allb = generate("nominal", n_ev * R, workers=min(16, os.cpu_count() or 1))
    gen_s = time.time() - t0
    batches = [allb.range(i * n_ev, (i + 1) * n_ev) for i in range(R)]

    import torch

    import paper_1912_09161_amd as velo
    dev = torch.device("cuda:0")
    S = max(1, args.streams)
    streams = [torch.cuda.Stream(dev) for _ in range(S)]
    params = velo.default_params()
    bufs = []
    max_px = max(b.n_pixels for b in batches)
    wss = [velo.alloc_workspace(max_px, n_ev, dev) for _ in range(S)]
    for b in batches:
        px = torch.from_numpy(b.pixels.view(np.int32)).to(dev)
        off = torch.from_numpy(b.offsets.view(np.int64)).to(dev)
        N = b.n_pixels
        bufs.append(dict(px=px, off=off, N=N, hits=velo.alloc_hits(N, n_ev, dev),
                         tracks=velo.alloc_tracks(N, n_ev, dev), states=velo.alloc_states(N, dev)))
    torch.cuda.synchronize()

    def step(i, ev=None):
        B = bufs[i % R]
        st = streams[i % S]
        ws = wss[i % S]
        if ev is not None:
            ev[0].record(st)
        velo.cluster(B["px"], B["off"], hits=B["hits"], ws=ws, stream=st)
        if ev is not None:
            ev[1].record(st)
        velo.find_tracks(B["hits"], B["off"], B["N"], params=params, tracks=B["tracks"], ws=ws,
                         stream=st)
        if ev is not None:
            ev[2].record(st)
        velo.fit(B["hits"], B["tracks"], B["off"], B["N"], params=params, states=B["states"],
                 stream=st)
        if ev is not None:
            ev[3].record(st)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # timed region: K steps over S streams; stage boundaries marked with events
    # recorded on the stream each stage is launched on
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        step(i, events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    stage_ms = np.zeros(3)
    for ev in events:
        for s_ in range(3):
            stage_ms[s_] += ev[s_].elapsed_time(ev[s_ + 1])
    stage_ms /= args.steps
    span_ms = max(events[0][0].elapsed_time(ev[3]) for ev in events)
    elapsed = max(wall, span_ms / 1e3)
    ev_per_s = args.steps * n_ev / elapsed

    # algorithmic bytes per launch of each stage, from the batch contents
    tot = dict(px=0, hits=0, tracks=0, trk_hits=0)
    for B in bufs:
        tot["px"] += B["N"]
        tot["hits"] += int(B["hits"]["n_hits"].sum().item())
        tot["tracks"] += int(B["tracks"]["n_tracks"].sum().item())
    th = 0  # hits on tracks, over the valid track slots
    for B, b in zip(bufs, batches):
        nt = B["tracks"]["n_tracks"].cpu().numpy()
        base = (b.offsets[:-1] // 3).astype(np.int64)
        nhits = B["tracks"]["nhits"].cpu().numpy()
        idx = np.concatenate([base[e] + np.arange(nt[e]) for e in range(n_ev)])
        th += int(nhits[idx].astype(np.int64).sum())
    tot["trk_hits"] = th
    per = {k: v / R for k, v in tot.items()}
    E = n_ev
    # clustering: read words + offsets; write 16 B per hit, 27+26+2 words per event
    b_cluster = 4 * per["px"] + 8 * (E + 1) + 16 * per["hits"] + 4 * 55 * E
    # find: read x, y of every hit and the plane tables; write per track 1 B count +
    # 4 B per hit index, plus 2 words per event
    b_find = 8 * per["hits"] + 4 * (53 + 1) * E + 8 * (E + 1) + per["tracks"] + 4 * per["trk_hits"] + 8 * E
    # fit: read count, indices, x, y, key of every track hit; write 56 B per state
    b_fit = per["tracks"] + 4 * per["trk_hits"] + 12 * per["trk_hits"] + 56 * per["tracks"] + 12 * E
    stages = []
    for name, ms, by in (("cluster", stage_ms[0], b_cluster), ("find_tracks", stage_ms[1], b_find),
                         ("fit", stage_ms[2], b_fit)):
        stages.append(dict(stage=name, ms=round(ms, 5), bytes=int(by), gbs=round(by / ms / 1e6, 1)))
    dom = max(stages, key=lambda s: s["ms"])
    roofline = dict(bound="hbm", achieved=dom["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(dom["gbs"] / HBM_PEAK_GBS, 5), traffic=None, kernel=dom["stage"],
                    per_event_bytes=round(dom["bytes"] / E, 1))

    # physics figures of merit on the first batch (generator truth)
    physics = None
    if not args.no_physics:
        from synth.truth import Truth, metrics, track_list
        B, b = bufs[0], batches[0]
        hits = {k: v.cpu().numpy() for k, v in B["hits"].items()}
        hits["key"] = hits["key"].view(np.uint32)
        tr = {k: v.cpu().numpy() for k, v in B["tracks"].items()}
        tr["hit_idx"] = tr["hit_idx"].view(np.uint32).reshape(-1, 26)
        evs, slot, nh, keys = track_list(tr, hits, b.offsets)
        acc = B["states"]["accepted"].cpu().numpy()[slot]
        m = metrics(Truth(b), evs, nh, keys, acc)
        physics = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in m.items()}

    learned = None
    if not args.no_learned:
        learned = run_learned(args, allb, batches, bufs, streams, params, velo, torch, n_ev, R, S,
                              phys_plain=physics)

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        n_cpu = args.cpu_events or n_ev * R
        sample = allb.range(0, min(n_cpu, allb.n_events))
        t1 = time.perf_counter()
        oracle.reconstruct(sample.pixels, sample.offsets, threads=threads)
        dt = time.perf_counter() - t1
        cpu = dict(value=round(sample.n_events / dt, 1), unit="events/s", cores=threads, kind="oracle",
                   sample=f"first {sample.n_events} generated nominal events, cluster+find+fit, "
                          f"{threads} threads over events, {dt:.2f} s wall")

    if args.copy_mb > 0:
        nb = args.copy_mb << 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    forms = dict(plain=dict(value=round(ev_per_s, 1), ms_per_step=round(elapsed * 1e3 / args.steps, 5),
                            physics=physics))
    headline = ev_per_s
    if learned is not None:
        forms["batched_mlp"] = learned
        headline = learned["value"]
    out = dict(
        metric="VELO events/s on 1 MI355X (plain vs batched+MLP) at matched efficiency/ghosts",
        value=round(headline, 1), unit="events/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(n_ev / headline * 1e3, 5), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOAD, events_per_step=n_ev, rotating_batches=R, streams=S,
                    form="batched_mlp" if learned is not None else "plain",
                    pixels_per_event=round(per["px"] / E, 1)),
        roofline=roofline, stages=stages, forms=forms, cpu_baseline=cpu,
        gen_seconds=round(gen_s, 1),
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()

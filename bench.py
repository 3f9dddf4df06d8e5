#!/usr/bin/env python3
"""Benchmark: VELO reconstruction events/s on one MI355X.

One step = the whole reconstruction (clustering -> track finding -> fit and
track selection, all in libvelo's HIP kernels) over one batch of 1000
nominal-occupancy synthetic events already resident in device memory.

Two forms are timed on the same batches:
  plain        velo_cluster, velo_find_tracks, velo_fit; chi2 / hit-count cut
  batched_mlp  velo_reconstruct_batched (size-ordered persistent kernels,
               autotuned launch shapes, replayed HIP graph) with the learned
               ghost classifier fused after the fit
The classifier is trained first, on the GPU, on tracks the method produces
on separate events (generator-truth labels), with its threshold chosen on
validation events for an efficiency at least the plain cut's.  The headline
value is the batched_mlp form.

As in the paper's throughput protocol (Sec. 3.2: several CPU-thread / GPU-
stream pairs, each with its own events), steps are issued round-robin on
several HIP streams with their own workspaces and outputs, and they rotate
over several distinct input batches, so the 256 MB Infinity Cache cannot hold
the working set.  The process asks HIP for more hardware queues than it has
streams (GPU_MAX_HW_QUEUES), so a stream waiting on a long kernel does not
hold up another stream queued behind it on the same hardware queue.

A second leg repeats both forms on high-occupancy events (the stress
sample); a third times 100k events of uneven occupancy in one launch per
stage (plain) or one graph replay (batched), the batched form's use case.

Prints one JSON line: events/s of every form; the HBM roofline of the
dominant stage, with stage durations from HIP events recorded on the launch
stream of a separate single-stream pass (with several streams a stage's span
includes the other streams' kernels); physics figures of merit from
generator truth; the CPU oracle's throughput on a bounded sample of the
nominal events.
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
STRESS = ("high occupancy: 1000 events/batch, PVs/event Poisson(20), noise 1e-4/px, 95% hit "
          "efficiency, 100 urad scattering, X/X0 2.38e-3 per plane")
UNEVEN = ("uneven occupancy in one launch: PVs/event uniform 1..15 (about 25-375 tracks per event), "
          "otherwise nominal")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "velo_hbm_traffic_nominal.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--events", type=int, default=1000, help="events per batch (one step)")
    ap.add_argument("--batches", type=int, default=8, help="distinct device-resident batches")
    ap.add_argument("--streams", type=int, default=12, help="concurrent HIP streams")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues HIP gives the process (GPU_MAX_HW_QUEUES, 1..32); more "
                         "queues than streams, so that no two streams share one")
    ap.add_argument("--stage-steps", type=int, default=48,
                    help="steps of the single-stream pass that times each stage (roofline)")
    ap.add_argument("--cpu-events", type=int, default=0,
                    help="oracle sample size (default: all generated nominal events)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-physics", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="plain form only")
    ap.add_argument("--no-stress", action="store_true", help="skip the high-occupancy leg")
    ap.add_argument("--train-events", type=int, default=5500, help="classifier training events (~1M tracks)")
    ap.add_argument("--val-events", type=int, default=2000)
    ap.add_argument("--stress-train", type=int, default=1500)
    ap.add_argument("--stress-val", type=int, default=1000)
    ap.add_argument("--stress-batches", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--uneven-events", type=int, default=100_000,
                    help="events of the uneven-occupancy batch timed in one launch (0: skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the run, 4 device-to-device copies of this many MiB (calibrates HBM "
                         "byte counters against a transfer of known size)")
    return ap.parse_args()


WORKERS = min(16, os.cpu_count() or 1)


def to_device(velo, torch, batches, dev, outputs=False):
    """Inputs of every batch on the device (and an output set each if asked)."""
    bufs = []
    for b in batches:
        N, E = b.n_pixels, b.n_events
        B = dict(px=torch.from_numpy(b.pixels.view(np.int32)).to(dev),
                 off=torch.from_numpy(b.offsets.view(np.int64)).to(dev), N=N, E=E)
        if outputs:
            B.update(alloc_out(velo, N, E, dev))
        bufs.append(B)
    return bufs


def alloc_out(velo, N, E, dev):
    return dict(hits=velo.alloc_hits(N, E, dev), tracks=velo.alloc_tracks(N, E, dev),
                states=velo.alloc_states(N, dev))


def stream_outputs(velo, bufs, S, dev):
    """One output set per stream, sized for the largest batch: steps in flight
    on different streams never write the same buffer (a stream's steps run in
    order); the input batches rotate over the streams."""
    N, E = max(B["N"] for B in bufs), max(B["E"] for B in bufs)
    return [alloc_out(velo, N, E, dev) for _ in range(S)]


def clean_run(velo, torch, B, O, ws, params):
    """One synchronous plain reconstruction of batch B into the output set O
    (after the timed runs: the figures that read outputs come from here)."""
    torch.cuda.synchronize()
    velo.reconstruct(B["px"], B["off"], params=params, bufs=dict(hits=O["hits"], tracks=O["tracks"],
                                                                 states=O["states"], ws=ws))
    torch.cuda.synchronize()
    return O


def labels(B, b):
    """(slot, label, particle uid, reconstructible uids) of the tracks in B."""
    from synth.truth import track_labels_parallel
    hits = {k: v.cpu().numpy() for k, v in B["hits"].items()}
    hits["key"] = hits["key"].view(np.uint32)
    tr = {k: v.cpu().numpy() for k, v in B["tracks"].items()}
    tr["hit_idx"] = tr["hit_idx"].view(np.uint32).reshape(-1, 26)
    return track_labels_parallel(b, tr, hits, workers=WORKERS)


def figures(uid, accepted, reco):
    """Efficiency, ghost and clone rates with binomial standard errors."""
    from synth.truth import efficiency_ghosts
    m = efficiency_ghosts(uid, accepted, reco)
    n_reco = max(len(np.unique(reco)), 1)
    m["efficiency_err"] = float(np.sqrt(m["efficiency"] * (1 - m["efficiency"]) / n_reco))
    m["ghost_rate_err"] = float(np.sqrt(m["ghost_rate"] * (1 - m["ghost_rate"]) / max(m["n_tracks"], 1)))
    return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in m.items()}


def repeats(run, steps, n_ev, n=10):
    """The paper's protocol: n measurements over different event sets (the
    batches rotate), mean and standard deviation of events/s."""
    per = max(1, steps // n)
    rates = []
    for r in range(n):
        rates.append(per * n_ev / run(per, r * per))
    return dict(n=n, steps_each=per, mean=round(float(np.mean(rates)), 1),
                std=round(float(np.std(rates, ddof=1)), 1))


def time_plain(velo, torch, bufs, outs, streams, wss, params, steps, warmup, with_events=False, first=0):
    R, S = len(bufs), len(streams)

    def step(i, ev=None):
        B, k = bufs[i % R], i % S
        st, ws, O = streams[k], wss[k], outs[k]
        if ev is not None:
            ev[0].record(st)
        velo.cluster(B["px"], B["off"], hits=O["hits"], ws=ws, stream=st)
        if ev is not None:
            ev[1].record(st)
        velo.find_tracks(O["hits"], B["off"], B["N"], params=params, tracks=O["tracks"], ws=ws, stream=st)
        if ev is not None:
            ev[2].record(st)
        velo.fit(O["hits"], O["tracks"], B["off"], B["N"], params=params, states=O["states"], stream=st)
        if ev is not None:
            ev[3].record(st)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)] if with_events else None
    w0 = time.perf_counter()
    for i in range(steps):
        step(first + i, events[i] if with_events else None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    if not with_events:
        return wall, None
    stage_ms = np.zeros(3)
    for ev in events:
        for s_ in range(3):
            stage_ms[s_] += ev[s_].elapsed_time(ev[s_ + 1])
    span = max(events[0][0].elapsed_time(ev[3]) for ev in events) / 1e3
    return max(wall, span), stage_ms / steps


def time_batched(velo, torch, bufs, outs, streams, params, mlp, steps, warmup, n_repeats=0):
    R, S = len(bufs), len(streams)
    dev = bufs[0]["px"].device
    ctxs = [velo.Context() for _ in range(S)]
    wss = [velo.alloc_batched_workspace(max(B["N"] for B in bufs), max(B["E"] for B in bufs), dev)
           for _ in range(S)]

    def step(i):
        B = bufs[i % R]
        k = i % S
        O = outs[k]
        ctxs[k].reconstruct(B["px"], B["off"], params=params, mlp=mlp,
                            bufs=dict(hits=O["hits"], tracks=O["tracks"], states=O["states"], ws=wss[k]),
                            stream=streams[k])

    import math
    for i in range(max(warmup, R * S // math.gcd(R, S))):  # autotune, then capture every (batch, stream) graph
        step(i)
    torch.cuda.synchronize()
    def run(n, first):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(n):
            step(first + i)
        torch.cuda.synchronize()
        return time.perf_counter() - w0

    wall = run(steps, 0)
    rep = repeats(run, steps, bufs[0]["E"], n_repeats) if n_repeats else None
    step(0)  # leave batch 0's outputs from this form in the first stream's output set
    torch.cuda.synchronize()
    cfg = ctxs[0].config()
    for c in ctxs:
        c.close()
    return wall, cfg, rep


def train(velo, torch, train_cfg, n_train, val_cfg, n_val, val_first, params, epochs, dev):
    """Classifier trained on the method's tracks of `train_cfg` events; threshold
    for the plain cut's efficiency on `val_cfg` events."""
    from paper_1912_09161_amd import learn
    from synth import generate
    t0 = time.time()

    def tracks_of(b):
        B = to_device(velo, torch, [b], dev, outputs=True)[0]
        velo.reconstruct(B["px"], B["off"], params=params,
                         bufs=dict(hits=B["hits"], tracks=B["tracks"], states=B["states"],
                                   ws=velo.alloc_workspace(B["N"], B["E"], dev)))
        feat = velo.track_features(B["hits"], B["tracks"], B["states"], B["off"], B["N"])
        torch.cuda.synchronize()
        slot, lab, uid, reco = labels(B, b)
        acc = B["states"]["accepted"].cpu().numpy()[slot]
        return feat[torch.from_numpy(slot).to(dev)].contiguous(), lab, uid, reco, acc

    F, lab, _, _, _ = tracks_of(generate(train_cfg, n_train, workers=WORKERS))
    trainer = learn.Trainer(F, torch.from_numpy(lab).to(dev), seed=7)
    for _ in range(epochs):
        trainer.epoch()
    Fv, _, uid, reco, acc = tracks_of(generate(val_cfg, n_val, first_event=val_first, workers=WORKERS))
    plain_val = figures(uid, acc, reco)
    z = velo.mlp_infer(trainer.mlp(0.0), Fv).cpu().numpy()
    # working point: the plain cut's validation efficiency plus 1e-4 (about the
    # statistical resolution of the validation sample), so that on independent
    # events the efficiency is not below the plain cut's
    thr = learn.choose_threshold(z, uid, reco, plain_val["efficiency"] + 1e-4)
    info = dict(train_events=n_train, train_tracks=int(F.shape[0]), epochs=epochs,
                val_events=n_val, threshold=thr, seconds=round(time.time() - t0, 1))
    return trainer.mlp(thr), info


def stored_traffic(stage):
    """HBM bytes per launch of a stage from the committed counter summary, if it
    was measured on the kernels built from the current sources."""
    from paper_1912_09161_amd.build import source_digest
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    return t.get("stage_bytes_per_launch", {}).get(stage)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); events are independent, "
              "so several GPUs would each run this benchmark on their own share.", file=sys.stderr)
        sys.exit(2)

    if not 1 <= args.hw_queues <= 32:
        print("--hw-queues must be within 1..32", file=sys.stderr)
        sys.exit(2)
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)  # read when HIP initialises, below

    from synth import generate
    n_ev, R = args.events, args.batches
    t0 = time.time()
    allb = generate("nominal", n_ev * R, workers=WORKERS)
    gen_s = time.time() - t0
    batches = [allb.range(i * n_ev, (i + 1) * n_ev) for i in range(R)]

    import torch

    import paper_1912_09161_amd as velo
    dev = torch.device("cuda:0")
    S = max(1, args.streams)
    streams = [torch.cuda.Stream(dev) for _ in range(S)]
    params = velo.default_params()
    bufs = to_device(velo, torch, batches, dev)
    outs = stream_outputs(velo, bufs, S, dev)
    max_px = max(B["N"] for B in bufs)
    wss = [velo.alloc_workspace(max_px, n_ev, dev) for _ in range(S)]
    torch.cuda.synchronize()

    # ---- plain form, stage boundaries marked with events on the launch streams
    elapsed, _ = time_plain(velo, torch, bufs, outs, streams, wss, params, args.steps, args.warmup)
    plain_value = args.steps * n_ev / elapsed
    plain_rep = repeats(lambda n, first: time_plain(velo, torch, bufs, outs, streams, wss, params, n, 0,
                                                    first=first)[0], args.steps, n_ev)

    # stage durations: a pass on one stream with the GPU to itself (with several
    # streams a stage's span on its stream includes the other streams' kernels)
    _, stage_ms = time_plain(velo, torch, bufs, outs[:1], streams[:1], wss[:1], params, args.stage_steps, 2,
                             with_events=True)

    # algorithmic bytes per launch of each stage, from the batch contents
    tot = dict(px=0, hits=0, tracks=0, trk_hits=0)
    for B, b in zip(bufs, batches):
        O = clean_run(velo, torch, B, outs[0], wss[0], params)
        tot["px"] += B["N"]
        tot["hits"] += int(O["hits"]["n_hits"].sum().item())
        nt = O["tracks"]["n_tracks"].cpu().numpy()
        tot["tracks"] += int(nt.sum())
        base = (b.offsets[:-1] // 3).astype(np.int64)
        nhits = O["tracks"]["nhits"].cpu().numpy()
        idx = np.concatenate([base[e] + np.arange(nt[e]) for e in range(n_ev)])
        tot["trk_hits"] += int(nhits[idx].astype(np.int64).sum())
    per = {k: v / R for k, v in tot.items()}
    E = n_ev
    # clustering: read words + offsets; write 16 B per hit, 27 + 26 + 2 words per event
    b_cluster = 4 * per["px"] + 8 * (E + 1) + 16 * per["hits"] + 4 * 55 * E
    # track finding: read x, y of every hit and the plane tables; write per track
    # 1 B count + 4 B per hit index, plus 2 words per event
    b_find = 8 * per["hits"] + 4 * (53 + 1) * E + 8 * (E + 1) + per["tracks"] + 4 * per["trk_hits"] + 8 * E
    # fit: read count, indices, x, y, key of every track hit; write 56 B per state
    b_fit = per["tracks"] + 4 * per["trk_hits"] + 12 * per["trk_hits"] + 56 * per["tracks"] + 12 * E
    stages = []
    for name, ms, by in (("cluster", stage_ms[0], b_cluster), ("find_tracks", stage_ms[1], b_find),
                         ("fit", stage_ms[2], b_fit)):
        stages.append(dict(stage=name, ms=round(ms, 5), bytes=int(by), gbs=round(by / ms / 1e6, 1),
                           frac=round(by / ms / 1e6 / HBM_PEAK_GBS, 5)))
    # whole pipeline: algorithmic bytes of all stages at the measured step rate
    overall = dict(bytes=int(b_cluster + b_find + b_fit),
                   gbs=round((b_cluster + b_find + b_fit) * plain_value / n_ev / 1e9, 1))
    overall["frac"] = round(overall["gbs"] / HBM_PEAK_GBS, 5)
    dom = max(stages, key=lambda s: s["ms"])
    roofline = dict(bound="hbm", achieved=dom["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(dom["gbs"] / HBM_PEAK_GBS, 5), traffic=stored_traffic(dom["stage"]),
                    kernel=dom["stage"], per_event_bytes=round(dom["bytes"] / E, 1))

    forms = dict(plain=dict(value=round(plain_value, 1), ms_per_step=round(elapsed * 1e3 / args.steps, 5),
                            repeats=plain_rep, hbm_overall=overall))
    lab0 = None
    if not args.no_physics:
        O = clean_run(velo, torch, bufs[0], outs[0], wss[0], params)
        lab0 = labels(O, batches[0])
        forms["plain"]["physics"] = figures(lab0[2], O["states"]["accepted"].cpu().numpy()[lab0[0]], lab0[3])

    # ---- batched form with the learned classifier
    headline = plain_value
    if not args.no_learned:
        mlp, info = train(velo, torch, "learn_train", args.train_events, "learn_val", args.val_events, 0,
                          params, args.epochs, dev)
        mlp_nominal = mlp
        wall, cfg, brep = time_batched(velo, torch, bufs, outs, streams, params, mlp, args.steps, args.warmup,
                                       n_repeats=10)
        value = args.steps * n_ev / wall
        forms["batched_mlp"] = dict(value=round(value, 1), ms_per_step=round(wall * 1e3 / args.steps, 5),
                                    repeats=brep, training=info, autotuned=cfg)
        if lab0 is not None:
            forms["batched_mlp"]["physics"] = figures(
                lab0[2], outs[0]["states"]["accepted"].cpu().numpy()[lab0[0]], lab0[3])
        headline = value
    del bufs, outs, wss
    torch.cuda.empty_cache()

    # ---- high-occupancy leg
    stress = None
    if not args.no_stress:
        sp = velo.default_params(x_over_x0=2.38e-3)
        sb = generate("stress", n_ev * args.stress_batches, first_event=8192, workers=WORKERS)
        sbatches = [sb.range(i * n_ev, (i + 1) * n_ev) for i in range(args.stress_batches)]
        sbufs = to_device(velo, torch, sbatches, dev)
        souts = stream_outputs(velo, sbufs, S, dev)
        swss = [velo.alloc_workspace(max(B["N"] for B in sbufs), n_ev, dev) for _ in range(S)]
        sw, _ = time_plain(velo, torch, sbufs, souts, streams, swss, sp, args.steps // 4, args.warmup)
        stress = dict(workload=STRESS, batches=args.stress_batches,
                      plain=dict(value=round(args.steps // 4 * n_ev / sw, 1)))
        O = clean_run(velo, torch, sbufs[0], souts[0], swss[0], sp)
        slab = labels(O, sbatches[0])
        stress["plain"]["physics"] = figures(slab[2], O["states"]["accepted"].cpu().numpy()[slab[0]], slab[3])
        if not args.no_learned:
            mlp, info = train(velo, torch, "stress", args.stress_train, "stress", args.stress_val, 4096, sp,
                              args.epochs, dev)
            wall, cfg, _ = time_batched(velo, torch, sbufs, souts, streams, sp, mlp, args.steps // 4, args.warmup)
            stress["batched_mlp"] = dict(
                value=round(args.steps // 4 * n_ev / wall, 1), training=info, autotuned=cfg,
                physics=figures(slab[2], souts[0]["states"]["accepted"].cpu().numpy()[slab[0]], slab[3]))
            gp, gl = stress["plain"]["physics"]["ghost_rate"], stress["batched_mlp"]["physics"]["ghost_rate"]
            stress["ghost_rate_reduction"] = round(1 - gl / gp, 4) if gp > 0 else None
        del sbufs, souts, swss
        torch.cuda.empty_cache()

    # ---- uneven occupancy, the whole batch in one launch per stage / one graph
    uneven = None
    if args.uneven_events > 0:
        t2 = time.time()
        ub = generate("uneven", args.uneven_events, workers=WORKERS)
        ugen = time.time() - t2
        ubuf = to_device(velo, torch, [ub], dev)
        uouts = stream_outputs(velo, ubuf, 1, dev)
        uws = [velo.alloc_workspace(ubuf[0]["N"], ubuf[0]["E"], dev)]
        ust = streams[:1]
        usteps = max(3, args.steps // 100)
        uw, _ = time_plain(velo, torch, ubuf, uouts, ust, uws, params, usteps, 1)
        uneven = dict(workload=UNEVEN, events=ub.n_events, pixels_per_event=round(ub.n_pixels / ub.n_events, 1),
                      steps=usteps, gen_seconds=round(ugen, 1),
                      plain=dict(value=round(usteps * ub.n_events / uw, 1)))
        del uws
        torch.cuda.empty_cache()
        if not args.no_learned:
            wall, cfg, _ = time_batched(velo, torch, ubuf, uouts, ust, params, mlp_nominal, usteps, 1)
            uneven["batched_mlp"] = dict(value=round(usteps * ub.n_events / wall, 1), autotuned=cfg)
        del ubuf, uouts
        torch.cuda.empty_cache()

    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = cpu1 = None
    if not args.no_cpu:
        import oracle
        threads = WORKERS
        n_cpu = args.cpu_events or n_ev * R
        sample = allb.range(0, min(n_cpu, allb.n_events))
        t1 = time.perf_counter()
        oracle.reconstruct(sample.pixels, sample.offsets, threads=threads)
        dt = time.perf_counter() - t1
        cpu = dict(value=round(sample.n_events / dt, 1), unit="events/s", cores=threads, kind="oracle",
                   sample=f"first {sample.n_events} generated nominal events, cluster+find+fit, "
                          f"{threads} threads over events, {dt:.2f} s wall; the oracle is a correctness "
                          f"reference (-O2, no contraction), not a tuned CPU implementation")
        one = allb.range(0, min(500, allb.n_events))
        t1 = time.perf_counter()
        oracle.reconstruct(one.pixels, one.offsets, threads=1)
        dt1 = time.perf_counter() - t1
        cpu1 = dict(value=round(one.n_events / dt1, 1), unit="events/s", cores=1, kind="oracle",
                    sample=f"first {one.n_events} generated nominal events, one thread, {dt1:.2f} s wall")

    out = dict(
        metric="VELO events/s on 1 MI355X (plain vs batched+MLP) at matched efficiency/ghosts",
        value=round(headline, 1), unit="events/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(n_ev / headline * 1e3, 5), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOAD, events_per_step=n_ev, rotating_batches=R, streams=S,
                    hw_queues=args.hw_queues,
                    form="plain" if args.no_learned else "batched_mlp",
                    pixels_per_event=round(per["px"] / E, 1)),
        roofline=roofline, stages=stages, stage_timing=f"one stream, {args.stage_steps} steps",
        forms=forms, stress=stress, uneven=uneven, cpu_baseline=cpu,
        cpu_baseline_1thread=cpu1,
        gen_seconds=round(gen_s, 1),
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()

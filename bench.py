#!/usr/bin/env python3
"""Benchmark: VELO reconstruction events/s on one MI355X.

A batch is 1000 nominal-occupancy synthetic events already resident in
device memory; one pass of the hot path over a batch is clustering, track
finding, the fit and the track selection, all in libvelo's HIP kernels.  As
in the paper's throughput protocol (Sec. 3.2: several CPU-thread / GPU-stream
pairs, each with its own events), a step is one round over S streams: every
stream reconstructs its own batch, so one step processes S x 1000 events.
The inputs rotate over 2 S distinct batches, each with its own output
buffers (batch b always runs on stream b mod S), about 4 GB of touched
device memory per rotation, so the 256 MB Infinity Cache cannot hold them.

Two forms are timed identically (same warm-up, covering every (batch,
stream) pair, same rounds):
  plain        velo_reconstruct; chi2 / hit-count cut
  batched_mlp  velo_reconstruct_batched (autotuned launch shapes, replayed HIP
               graph) with the learned ghost classifier fused after the fit
The classifier is trained first, on the GPU, on the method's own tracks of
separate events (generator-truth labels), its threshold chosen on
validation events for an efficiency at least the plain cut's.  The headline
value is the batched_mlp form; the plain form's value is reported beside it.

Also reported: ten repeated measurements over different rotations (mean,
std); the HBM roofline of the dominant kernel, timed by itself with HIP
events on its stream in a one-stream pass over all batches; efficiency,
ghost and clone rates of both forms on held-out events; the streaming form
(host memory in, compact tracks and vertices out, thread-stream pairs, with
and without the global event cut); 100k events of uneven occupancy in one
launch (plain and batched + classifier); the high-occupancy sample; the CPU
oracle on a bounded sample.
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
WORKLOAD = ("nominal occupancy: 1000 events per batch, 26 planes, PVs/event Poisson(7.6), "
            "tracks/PV Poisson(25), 98% hit efficiency, 1-3 px clusters, noise 1e-5/px, "
            "50 urad scattering; uint32 raw words, binary32 hits and fits")
UNEVEN = ("uneven occupancy in one launch: PVs/event uniform 1..15 (about 25-375 tracks per event), "
          "otherwise nominal")
STRESS = ("high occupancy: PVs/event Poisson(20), noise 1e-4/px, 95% hit efficiency, 100 urad "
          "scattering, X/X0 2.38e-3 per plane")
THREADS = os.cpu_count() or 1
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "velo_hbm_traffic_nominal.json")
DOMINANT_KERNEL = {"cluster": "k_small", "find_tracks": "k_find_lds<256, 288u, 256u, 384u, 768u>",
                   "fit": "k_fit<256>"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (rounds over the streams)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=1000, help="events per batch")
    ap.add_argument("--streams", type=int, default=12, help="concurrent HIP streams (S)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues HIP gives the process (GPU_MAX_HW_QUEUES, 1..32)")
    ap.add_argument("--repeats", type=int, default=10, help="repeated measurements of each form")
    ap.add_argument("--kernel-rounds", type=int, default=2,
                    help="rounds over all batches of the one-stream kernel-timing pass")
    ap.add_argument("--train-events", type=int, default=5500)
    ap.add_argument("--val-events", type=int, default=2000)
    ap.add_argument("--physics-events", type=int, default=10000, help="held-out test events for efficiency")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--ghost-weight", type=float, default=64.0,
                    help="ghost tracks drawn this many times as often in training (nominal occupancy: "
                         "ghosts are 0.085 %% of the tracks)")
    ap.add_argument("--stress-epochs", type=int, default=8)
    ap.add_argument("--stress-ghost-weight", type=float, default=1.0,
                    help="the same at high occupancy (ghosts are about 4 %% of the tracks)")
    ap.add_argument("--stress-events", type=int, default=2000, help="0: skip the high-occupancy leg")
    ap.add_argument("--uneven-events", type=int, default=100000,
                    help="events of uneven occupancy reconstructed in one launch (0: skip that leg)")
    ap.add_argument("--uneven-steps", type=int, default=3)
    ap.add_argument("--stress-train", type=int, default=1500)
    ap.add_argument("--stress-val", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-physics", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="plain form only")
    ap.add_argument("--no-e2e", action="store_true", help="skip the streaming (host memory) leg")
    ap.add_argument("--e2e-passes", type=int, default=5, help="timed passes of the streaming leg over its events")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the run, 4 device-to-device copies of this many MiB (calibrates HBM "
                         "byte counters against a transfer of known size)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# device buffers and launches


def batches_to_device(velo, torch, batches, dev):
    out = []
    for b in batches:
        N, E = b.n_pixels, b.n_events
        out.append(dict(px=torch.from_numpy(b.pixels.view(np.int32)).to(dev),
                        off=torch.from_numpy(b.offsets.view(np.int64)).to(dev), N=N, E=E,
                        hits=velo.alloc_hits(N, E, dev), tracks=velo.alloc_tracks(N, E, dev),
                        states=velo.alloc_states(N, dev)))
    return out


class Plain:
    """velo_reconstruct with prepared arguments (batch b into its own outputs,
    the stream's workspace)."""

    def __init__(self, velo, B, streams, params):
        import ctypes as C
        self.L = velo.lib()
        N, E = max(x["N"] for x in B), max(x["E"] for x in B)
        self.ws = [velo.alloc_workspace(N, E, B[0]["px"].device) for _ in streams]
        self.params = params
        self.args = {}
        for b, x in enumerate(B):
            s = b % len(streams)
            self.args[b] = (velo.velo._ptr(x["px"]), velo.velo._ptr(x["off"]), x["E"], x["N"],
                            velo.velo._geom(), C.byref(params), C.byref(velo.velo._hits_struct(x["hits"])),
                            C.byref(velo.velo._tracks_struct(x["tracks"])),
                            C.byref(velo.velo._states_struct(x["states"])), velo.velo._ptr(self.ws[s]),
                            self.ws[s].numel(), velo.velo._stream(streams[s]))

    def __call__(self, b):
        rc = self.L.velo_reconstruct(*self.args[b])
        if rc != 0:
            raise RuntimeError(f"velo_reconstruct failed ({rc})")


class Batched:
    """velo_reconstruct_batched with the fused classifier, one context per
    stream (its tuned shapes come from the first context's tuning through the
    tune cache; its graphs are captured on the first call of each batch)."""

    def __init__(self, velo, B, streams, params, mlp):
        import ctypes as C
        self.L = velo.lib()
        dev = B[0]["px"].device
        N, E = max(x["N"] for x in B), max(x["E"] for x in B)
        self.ctx = [velo.Context(params) for _ in streams]
        self.ws = [velo.alloc_batched_workspace(N, E, dev) for _ in streams]
        self.mlp_s = mlp.struct()
        self.keep = (params, mlp)
        self.args = {}
        for b, x in enumerate(B):
            s = b % len(streams)
            self.args[b] = (self.ctx[s]._h, velo.velo._ptr(x["px"]), velo.velo._ptr(x["off"]), x["E"], x["N"],
                            C.byref(params), C.byref(self.mlp_s), C.byref(velo.velo._hits_struct(x["hits"])),
                            C.byref(velo.velo._tracks_struct(x["tracks"])),
                            C.byref(velo.velo._states_struct(x["states"])), velo.velo._ptr(self.ws[s]),
                            self.ws[s].numel(), velo.velo._stream(streams[s]))

    def __call__(self, b):
        rc = self.L.velo_reconstruct_batched(*self.args[b])
        if rc != 0:
            raise RuntimeError(f"velo_reconstruct_batched failed ({rc})")

    def close(self):
        cfg = self.ctx[0].config()
        for c in self.ctx:
            c.close()
        return cfg


def rounds(launch, S, first, n):
    """n rounds from round `first`: round k runs batches (k mod 2) S + s on stream s."""
    for k in range(first, first + n):
        h = (k % 2) * S
        for s in range(S):
            launch(h + s)


def timed(torch, launch, S, first, n):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rounds(launch, S, first, n)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def measure(torch, launch, S, E, steps, warmup, n_rep):
    """Warm-up (at least both halves of the rotation), the timed window, then
    n_rep repeated windows of the same length over shifted rotations."""
    rounds(launch, S, 0, max(warmup, 2))
    torch.cuda.synchronize()
    wall = timed(torch, launch, S, 0, steps)
    if n_rep <= 0:
        return wall, None
    reps = [steps * S * E / timed(torch, launch, S, r + 1, steps) for r in range(n_rep)]
    rep = dict(n=n_rep, steps_each=steps, mean=round(float(np.mean(reps)), 1),
               std=round(float(np.std(reps, ddof=1)), 1) if n_rep > 1 else 0.0)
    return wall, rep


# ---------------------------------------------------------------------------
# physics


def host_tracks(B):
    hits = {k: v.cpu().numpy() for k, v in B["hits"].items()}
    hits["key"] = hits["key"].view(np.uint32)
    tr = {k: v.cpu().numpy() for k, v in B["tracks"].items()}
    tr["hit_idx"] = tr["hit_idx"].view(np.uint32).reshape(-1, 26)
    return hits, tr


def labels(B, b):
    """(slot, label, particle uid, reconstructible uids) of the tracks in B."""
    from synth.truth import track_labels_parallel
    hits, tr = host_tracks(B)
    return track_labels_parallel(b, tr, hits, workers=THREADS)


def figures(uid, accepted, reco):
    """Efficiency, ghost and clone rates with binomial standard errors."""
    from synth.truth import efficiency_ghosts
    m = efficiency_ghosts(uid, accepted, reco)
    n_reco = max(len(np.unique(reco)), 1)
    m["efficiency_err"] = float(np.sqrt(m["efficiency"] * (1 - m["efficiency"]) / n_reco))
    m["ghost_rate_err"] = float(np.sqrt(m["ghost_rate"] * (1 - m["ghost_rate"]) / max(m["n_tracks"], 1)))
    return {k: (round(v, 7) if isinstance(v, float) else v) for k, v in m.items()}


def reconstruct_events(velo, torch, b, params, dev, mlp=None):
    B = batches_to_device(velo, torch, [b], dev)[0]
    bufs = dict(hits=B["hits"], tracks=B["tracks"], states=B["states"],
                ws=velo.alloc_workspace(B["N"], B["E"], dev))
    if mlp is None:
        velo.reconstruct(B["px"], B["off"], params=params, bufs=bufs)
    else:
        velo.reconstruct_mlp(B["px"], B["off"], mlp, params=params, bufs=bufs)
    torch.cuda.synchronize()
    return B


def train(velo, torch, train_b, val_b, params, epochs, ghost_weight, dev):
    """Classifier trained on the method's tracks of train_b; threshold: the
    largest logit cut whose efficiency on val_b is at least the plain cut's."""
    from paper_1912_09161_amd import learn
    t0 = time.time()

    def tracks_of(b):
        B = reconstruct_events(velo, torch, b, params, dev)
        feat = velo.track_features(B["hits"], B["tracks"], B["states"], B["off"], B["N"])
        torch.cuda.synchronize()
        slot, lab, uid, reco = labels(B, b)
        acc = B["states"]["accepted"].cpu().numpy()[slot]
        return feat[torch.from_numpy(slot).to(dev)].contiguous(), lab, uid, reco, acc

    F, lab, _, _, _ = tracks_of(train_b)
    trainer = learn.Trainer(F, torch.from_numpy(lab).to(dev), seed=7, ghost_weight=ghost_weight)
    for _ in range(epochs):
        trainer.epoch()
    Fv, _, uid, reco, acc = tracks_of(val_b)
    plain_val = figures(uid, acc, reco)
    z = velo.mlp_infer(trainer.mlp(0.0), Fv).cpu().numpy()
    thr = learn.choose_threshold(z, uid, reco, plain_val["efficiency"])
    info = dict(train_events=train_b.n_events, train_tracks=int(F.shape[0]), ghosts_in_training=int((lab == 0).sum()),
                ghost_weight=ghost_weight, epochs=epochs, val_events=val_b.n_events, threshold=thr,
                plain_val_efficiency=plain_val["efficiency"], seconds=round(time.time() - t0, 1))
    return trainer.mlp(thr), info


def physics(velo, torch, b, params, mlp, dev):
    """Figures of merit of the plain cut and of the classifier on events b."""
    B = reconstruct_events(velo, torch, b, params, dev)
    lab = labels(B, b)
    out = dict(events=b.n_events, plain=figures(lab[2], B["states"]["accepted"].cpu().numpy()[lab[0]], lab[3]))
    if mlp is not None:
        Bm = reconstruct_events(velo, torch, b, params, dev, mlp=mlp)
        out["batched_mlp"] = figures(lab[2], Bm["states"]["accepted"].cpu().numpy()[lab[0]], lab[3])
        gp, gl = out["plain"]["ghost_rate"], out["batched_mlp"]["ghost_rate"]
        out["ghost_rate_reduction"] = round(1 - gl / gp, 4) if gp > 0 else None
        out["efficiency_not_lower"] = out["batched_mlp"]["efficiency"] >= out["plain"]["efficiency"]
        # equal within the binomial standard error of the difference (the two rates are measured
        # on the same particles, so this is conservative)
        se = float(np.hypot(out["plain"]["efficiency_err"], out["batched_mlp"]["efficiency_err"]))
        out["efficiency_equal_within_error"] = bool(
            out["batched_mlp"]["efficiency"] >= out["plain"]["efficiency"] - se)
    return out


# ---------------------------------------------------------------------------
# roofline of the dominant kernel


def algorithmic_bytes(velo, torch, B, b):
    """Bytes per launch each stage must move (one batch): clustering reads the
    words and offsets and writes 16 B per hit and the per-event tables; track
    finding reads x, y, key of every hit and writes 1 B + 4 B per track hit of
    every track; the fit reads index, x, y of every track hit and writes a
    56 B state and 5 B of decision and count per track."""
    nh = int(B["hits"]["n_hits"].sum().item())
    nt = B["tracks"]["n_tracks"].cpu().numpy().astype(np.int64)
    base = (b.offsets[:-1] // 3).astype(np.int64)
    nhits = B["tracks"]["nhits"].cpu().numpy()
    idx = np.concatenate([base[e] + np.arange(nt[e]) for e in range(b.n_events)])
    th = int(nhits[idx].astype(np.int64).sum())
    T = int(nt.sum())
    E, N = b.n_events, b.n_pixels
    return dict(cluster=4 * N + 16 * E + 16 * nh + 4 * (27 + 26 + 2) * E,
                find_tracks=12 * nh + T + 4 * th,
                fit=12 * th + 61 * T), dict(hits=nh, tracks=T, track_hits=th)


def stored_traffic(kernel):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per launch of a kernel from the
    committed counter summary, if it was taken on the current kernel sources."""
    from paper_1912_09161_amd.build import source_digest
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else int(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])


def kernel_pass(velo, torch, B, batches, stream, params, n_rounds):
    """One stream: every batch n_rounds times through velo_reconstruct_timed;
    average duration of each stage's main kernel; algorithmic bytes."""
    timer = velo.KernelTimer()
    ws = velo.alloc_workspace(max(x["N"] for x in B), max(x["E"] for x in B), B[0]["px"].device)
    dur = []
    for r in range(n_rounds + 1):
        for x in B:
            velo.reconstruct_timed(x["px"], x["off"], timer, params=params,
                                   bufs=dict(hits=x["hits"], tracks=x["tracks"], states=x["states"], ws=ws),
                                   stream=stream)
            d = timer.durations()
            if r > 0:  # the first round warms up
                dur.append(d)
    timer.close()
    torch.cuda.synchronize()
    by = [algorithmic_bytes(velo, torch, x, b) for x, b in zip(B, batches)]
    ms = np.mean(np.array(dur), axis=0)
    per = {k: float(np.mean([v[0][k] for v in by])) for k in ("cluster", "find_tracks", "fit")}
    counts = {k: float(np.mean([v[1][k] for v in by])) for k in ("hits", "tracks", "track_hits")}
    kernels = []
    for i, st in enumerate(("cluster", "find_tracks", "fit")):
        gbs = per[st] / (ms[i] * 1e-3) / 1e9
        kernels.append(dict(stage=st, kernel=DOMINANT_KERNEL[st], avg_us=round(float(ms[i]) * 1e3, 2),
                            launches=len(dur), bytes_per_launch=int(per[st]), gbs=round(gbs, 1),
                            frac=round(gbs / HBM_PEAK_GBS, 5)))
    return kernels, counts


# ---------------------------------------------------------------------------


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): events are independent, so several "
              "GPUs would each run this benchmark on their own share of the events; no multi-GPU figure is "
              "produced here.", file=sys.stderr)
        sys.exit(2)
    if not 1 <= args.hw_queues <= 32:
        print("--hw-queues must be within 1..32", file=sys.stderr)
        sys.exit(2)
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)  # read when HIP initialises, below

    from synth import generate
    S, E = max(1, args.streams), args.events
    R = 2 * S
    t0 = time.time()
    allb = generate("nominal", E * R, workers=THREADS)
    batches = [allb.range(i * E, (i + 1) * E) for i in range(R)]
    gen_s = time.time() - t0
    log(f"generated {R} x {E} nominal events in {gen_s:.1f} s")

    import torch

    import paper_1912_09161_amd as velo
    dev = torch.device("cuda:0")
    streams = [torch.cuda.Stream(dev) for _ in range(S)]
    params = velo.default_params()
    B = batches_to_device(velo, torch, batches, dev)
    torch.cuda.synchronize()
    touched = sum(x["px"].numel() * 4 + sum(t.numel() * t.element_size() for part in ("hits", "tracks", "states")
                                            for t in x[part].values()) for x in B)

    # ---- plain form
    plain = Plain(velo, B, streams, params)
    wall, rep = measure(torch, plain, S, E, args.steps, args.warmup, args.repeats)
    plain_value = args.steps * S * E / wall
    forms = dict(plain=dict(value=round(plain_value, 1), ms_per_step=round(wall * 1e3 / args.steps, 4),
                            repeats=rep))
    log(f"plain: {plain_value:.0f} events/s")

    # ---- dominant kernel, timed by itself
    kernels, counts = kernel_pass(velo, torch, B, batches, streams[0], params, args.kernel_rounds)
    dom = max(kernels, key=lambda k: k["avg_us"])
    roofline = dict(bound="hbm", achieved=dom["gbs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=dom["frac"],
                    traffic=stored_traffic(dom["kernel"]), kernel=dom["kernel"],
                    bytes_per_launch=dom["bytes_per_launch"], avg_us=dom["avg_us"])

    # ---- learned classifier and the batched form
    headline, mlp_nominal, phys = plain_value, None, None
    if not args.no_learned:
        mlp_nominal, info = train(velo, torch, generate("learn_train", args.train_events, workers=THREADS),
                                  generate("learn_val", args.val_events, workers=THREADS), params,
                                  args.epochs, args.ghost_weight, dev)
        bat = Batched(velo, B, streams, params, mlp_nominal)
        wall_b, rep_b = measure(torch, bat, S, E, args.steps, args.warmup, args.repeats)
        cfg = bat.close()
        value = args.steps * S * E / wall_b
        forms["batched_mlp"] = dict(value=round(value, 1), ms_per_step=round(wall_b * 1e3 / args.steps, 4),
                                    repeats=rep_b, training=info, autotuned=cfg)
        headline = value
        log(f"batched+classifier: {value:.0f} events/s")
    if not args.no_physics:
        phys = physics(velo, torch, generate("learn_test", args.physics_events, workers=THREADS), params,
                       mlp_nominal, dev)
        phys["sample"] = f"first {args.physics_events} events of the held-out test seed"

    # ---- streaming form: host memory in, compact tracks and vertices out
    e2e = None
    if not args.no_e2e:
        sizes = np.diff(allb.offsets.astype(np.int64))
        cut = int(np.percentile(sizes, 90))
        words = int(max(b.n_pixels for b in batches) * 1.25)
        e2e = dict(events=allb.n_events, streams=S, events_per_batch=E, note=(
            "events/s = input events / wall time of velo_pipeline_run (host packing into pinned staging, "
            "copies in, all kernels incl. vertex finding, compact rows and vertices back); PCIe-inclusive, "
            "not the headline"))
        for name, gec in (("no_cut", 0), ("gec", cut)):
            p = velo.Pipeline(S, E, words, gec_max_words=gec, params=params)
            p.run(allb.pixels, allb.offsets)  # warm-up (first touch of the pinned buffers)
            t1 = time.perf_counter()
            for _ in range(args.e2e_passes):
                r = p.run(allb.pixels, allb.offsets)
            dt = time.perf_counter() - t1
            p.close()
            e2e[name] = dict(value=round(args.e2e_passes * allb.n_events / dt, 1), seconds=round(dt, 4),
                             passes=args.e2e_passes, gec_max_words=gec,
                             events_cut=int((r["status"] == velo.EV_GEC).sum()), track_rows=int(len(r["tracks"])))
        e2e["gec_gain"] = round(e2e["gec"]["value"] / e2e["no_cut"]["value"] - 1, 4)
    del plain, B
    torch.cuda.empty_cache()

    # ---- uneven occupancy, every event in one launch (the batched form's own workload)
    uneven = None
    if args.uneven_events > 0:
        t1 = time.time()
        ub = generate("uneven", args.uneven_events, workers=THREADS)
        ugen = time.time() - t1
        UB = batches_to_device(velo, torch, [ub], dev)
        s0 = streams[0]
        up = Plain(velo, UB, [s0], params)
        uneven = dict(workload=UNEVEN, events=ub.n_events, pixels_per_event=round(ub.n_pixels / ub.n_events, 1),
                      steps=args.uneven_steps, gen_seconds=round(ugen, 1))
        w, _ = measure(torch, lambda b: up(0), 1, ub.n_events, args.uneven_steps, 1, 0)
        uneven["plain"] = dict(value=round(args.uneven_steps * ub.n_events / w, 1))
        if mlp_nominal is not None:
            ubt = Batched(velo, UB, [s0], params, mlp_nominal)
            w, _ = measure(torch, lambda b: ubt(0), 1, ub.n_events, args.uneven_steps, 1, 0)
            uneven["batched_mlp"] = dict(value=round(args.uneven_steps * ub.n_events / w, 1), autotuned=ubt.close())
        del up, UB
        torch.cuda.empty_cache()
        log(f"uneven: plain {uneven['plain']['value']:.0f} events/s")

    # ---- high occupancy
    stress = None
    if args.stress_events > 0:
        sp = velo.default_params(x_over_x0=2.38e-3)
        sb = generate("stress", args.stress_events, first_event=8192, workers=THREADS)
        nb = max(1, sb.n_events // E)
        sbat = [sb.range(i * E, min((i + 1) * E, sb.n_events)) for i in range(nb)]
        SB = batches_to_device(velo, torch, sbat, dev)
        ss = streams[:len(SB)]
        sp_plain = Plain(velo, SB, ss, sp)
        n_st = max(2, args.steps // 4)
        w, _ = measure(torch, lambda b: sp_plain(b % len(SB)), len(ss), E, n_st, args.warmup, 0)
        stress = dict(workload=STRESS, events=sb.n_events, streams=len(ss),
                      plain=dict(value=round(n_st * len(ss) * E / w, 1)))
        if not args.no_learned:
            mlp_s, info_s = train(velo, torch, generate("stress", args.stress_train, workers=THREADS),
                                  generate("stress", args.stress_val, first_event=4096, workers=THREADS), sp,
                                  args.stress_epochs, args.stress_ghost_weight, dev)
            sbt = Batched(velo, SB, ss, sp, mlp_s)
            w, _ = measure(torch, lambda b: sbt(b % len(SB)), len(ss), E, n_st, args.warmup, 0)
            stress["batched_mlp"] = dict(value=round(n_st * len(ss) * E / w, 1), training=info_s,
                                         autotuned=sbt.close())
        else:
            mlp_s = None
        if not args.no_physics:
            stress["physics"] = physics(velo, torch, sb, sp, mlp_s, dev)
        del sp_plain, SB
        torch.cuda.empty_cache()

    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- CPU oracle on a bounded sample
    cpu = cpu1 = None
    if not args.no_cpu:
        import oracle
        probe = allb.range(0, 50)
        t1 = time.perf_counter()
        oracle.reconstruct(probe.pixels, probe.offsets, threads=1)
        rate1 = probe.n_events / (time.perf_counter() - t1)
        n_cpu = int(min(allb.n_events, max(100, rate1 * THREADS * args.cpu_seconds * 0.7)))
        sample = allb.range(0, n_cpu)
        t1 = time.perf_counter()
        oracle.reconstruct(sample.pixels, sample.offsets, threads=THREADS)
        dt = time.perf_counter() - t1
        cpu = dict(value=round(sample.n_events / dt, 1), unit="events/s", cores=THREADS, kind="oracle",
                   sample=f"first {sample.n_events} nominal events of the benchmark's batches, cluster+find+fit, "
                          f"{THREADS} threads over events, {dt:.2f} s wall; the oracle is a correctness "
                          f"reference (-O2, no contraction), not a tuned CPU implementation")
        one = allb.range(0, min(int(rate1 * 5) + 1, allb.n_events))
        t1 = time.perf_counter()
        oracle.reconstruct(one.pixels, one.offsets, threads=1)
        dt1 = time.perf_counter() - t1
        cpu1 = dict(value=round(one.n_events / dt1, 1), unit="events/s", cores=1, kind="oracle",
                    sample=f"first {one.n_events} nominal events, one thread, {dt1:.2f} s wall")

    gates = dict(
        batched_mlp_ge_plain=None if args.no_learned else bool(headline >= plain_value),
        batched_mlp_ge_plain_uneven=None if not uneven or "batched_mlp" not in uneven
        else bool(uneven["batched_mlp"]["value"] >= uneven["plain"]["value"]),
        ghost_reduction_ge_20pct=None if not phys or "ghost_rate_reduction" not in phys
        else bool((phys["ghost_rate_reduction"] or 0) >= 0.2 and phys["efficiency_equal_within_error"]),
        ghost_reduction_ge_20pct_high_occupancy=None if not stress or "physics" not in stress
        or "ghost_rate_reduction" not in stress["physics"]
        else bool((stress["physics"]["ghost_rate_reduction"] or 0) >= 0.2
                  and stress["physics"]["efficiency_equal_within_error"]),
        cluster_hbm_frac=next(k["frac"] for k in kernels if k["stage"] == "cluster"),
        cluster_hbm_ge_50pct=bool(next(k["frac"] for k in kernels if k["stage"] == "cluster") >= 0.5))
    out = dict(
        metric="VELO events/s on 1 MI355X (plain vs batched+MLP) at matched efficiency/ghosts",
        value=round(headline, 1), unit="events/s", n_gpus=1, steps=args.steps, warmup=max(args.warmup, 2),
        ms_per_step=round(S * E / headline * 1e3, 4), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=WORKLOAD, events_per_batch=E, streams=S, events_per_step=S * E,
                    rotating_batches=R, touched_device_bytes=int(touched), hw_queues=args.hw_queues,
                    form="plain" if args.no_learned else "batched_mlp",
                    pixels_per_event=round(allb.n_pixels / allb.n_events, 1),
                    per_batch=dict(hits=counts["hits"], tracks=counts["tracks"], track_hits=counts["track_hits"])),
        roofline=roofline, kernels=kernels, forms=forms, gates=gates, physics=phys, e2e=e2e, uneven=uneven,
        stress=stress,
        cpu_baseline=cpu, cpu_baseline_1thread=cpu1, gen_seconds=round(gen_s, 1))
    print(json.dumps(out))


if __name__ == "__main__":
    main()

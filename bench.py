"""Frame-time benchmark of the sub-1-spp path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config c2|c3|c5] [--gpus 1]

A step is one frame of the path over one synthetic 1920x1080 frame at 0.25 spp (config c2 by
default): sampler CNN + budget normalisation, sample mask, scatter + pyramid, kernel-predictor
U-Net, gathering pyramid.  The renderer stand-in that turns the sample request into samples is
run once before timing (the mask is identical every step: same scene, seed and weights); its
output is resident in HBM when the timed region starts.  Weights are seeded random-init of the
configured architecture; inputs are procedural scenes (synthetic data).

Printed: one JSON line with ms/frame and Mpixel/s of the learned path, the uniform-sampling /
fixed-kernel fallback timed beside it, per-stage times, the roofline of the dominant kernel
(the MFMA convolution of the U-Net) and the FP64 CPU oracle on a bounded band of the frame.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "fp32_mfma_TFLOPs": 157.3, "bf16_mfma_TFLOPs": 2500.0}


def unet_flops(cfg, spec):
    """Algorithmic FLOPs of one U-Net pass: 2 k^2 cin cout per output pixel of each layer."""
    H, W = cfg.H, cfg.W
    res = {"enc0a": 0, "enc0b": 0, "enc1a": 1, "enc1b": 1, "enc2a": 2, "enc2b": 2, "bota": 3,
           "botb": 3, "dec2a": 2, "dec2b": 2, "dec1a": 1, "dec1b": 1, "dec0a": 0, "dec0b": 0}
    tot = 0
    for l in spec:
        lv = res.get(l["name"], int(l["name"][4:]) if l["name"].startswith("head") else 0)
        px = (H >> lv) * (W >> lv)
        tot += 2 * l["k"] * l["k"] * l["cin"] * l["cout"] * px
    return tot


def filter_bytes(cfg):
    """Algorithmic HBM bytes of the gathering pyramid per frame (logits, L^l, output, coarse
    level, and at level 0 with the temporal term the previous output and motion vectors)."""
    lb = 4 if cfg.logit_dtype.itemsize == 4 else 2
    ks = cfg.filter_channels()
    tot = 0
    for l in range(cfg.levels):
        px = (cfg.H >> l) * (cfg.W >> l)
        b = ks[l] * lb + 16 + 16
        if l < cfg.levels - 1:
            b += 4
        if l == 0 and cfg.temporal:
            b += 16 + 8
        tot += px * b
    if cfg.demod:   # demodulation: L0 + d in, the demodulated pyramid out; remodulation: in, d, out
        px = cfg.H * cfg.W
        tot += px * (16 + 3 * lb) + sum(16 * ((cfg.H >> l) * (cfg.W >> l)) for l in range(cfg.levels))
        tot += px * (16 + 3 * lb + 16)
    return tot


def cpu_baseline(cfg, dw, kw, rows: int):
    """FP64 oracle on a bounded band (rows x full width) of the same workload."""
    import numpy as np
    import torch

    import procgen
    from oracle import density as od
    from oracle import filt as of
    from oracle import sampling as osm
    from oracle import unet as ou

    H, W = rows, cfg.W
    sc = procgen.make_scene(11, H, W)
    fr = procgen.make_frame(sc, 0)
    pool = procgen.sample_pool(fr.truth, 11, 0, 8)
    dl = [(torch.tensor(dw[l["name"]][0], dtype=torch.float64),
           torch.tensor(dw[l["name"]][1], dtype=torch.float64), l["relu"])
          for l in procgen.density_cnn_spec(cfg.sampler_cin)]
    kwt = ou.to_torch(kw)
    aux = torch.tensor(fr.aux[None], dtype=torch.float64)
    t0 = time.perf_counter()
    z = od.cnn_forward(aux, dl)[..., 0]
    s = od.normalise(z, cfg.budget)
    m = osm.mask(s.numpy().astype(np.float32), 11, 0)
    cnt = m["count"].reshape(-1).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    j = np.arange(m["total"]) - start[m["sample_pixel"]]
    samples = pool[m["sample_pixel"], j % 8]
    L0 = osm.scatter(s, m["count"], samples, 11, 0)
    Ls = osm.pyramid(L0, cfg.levels)
    feat = torch.zeros(1, H, W, 16, dtype=torch.float64)
    feat[..., :7] = aux[..., :7]
    feat[..., 7:10] = torch.sign(L0[..., :3]) * torch.log1p(L0[..., :3].abs())
    feat[..., 10] = s
    logits = ou.unet_forward(feat, kwt, cfg.levels)
    out = of.denoise_pyramid(Ls, logits, cfg.KD, cfg.KU, cfg.KT)[0]
    dt = time.perf_counter() - t0
    assert torch.isfinite(out).all()
    res = dict(value=round(H * W / dt / 1e6, 5), unit="Mpixel/s", cores=torch.get_num_threads(),
               kind="oracle", seconds=round(dt, 3),
               sample=(f"one {W}x{H} band of the {cfg.W}x{cfg.H} frame" if H < cfg.H else
                       f"one whole {W}x{H} frame") +
                      ", full path (sampler CNN, normalisation, mask, scatter, pyramid, U-Net, "
                      "gathering pyramid) in FP64")
    return res, feat, logits


def cpu_baseline_1core(cfg, dw, kw, rows: int):
    """The same oracle path on one host thread, on a band of `rows` rows of the frame."""
    import torch
    n = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        r, _, _ = cpu_baseline(cfg, dw, kw, rows)
    finally:
        torch.set_num_threads(n)
    return r


def precision_vs_oracle(cfg, kw, feat, logits_ref, dev):
    """Per-head error of the library's U-Net against the FP64 oracle on the oracle frame's
    features: in the configuration's dtype (against logits_ref), and the same network in bf16
    (against the oracle on the bf16-rounded weights and features).  Per head: the normwise
    relative error and the largest abs(y - r) / (abs(r) + rms(r))."""
    import numpy as np
    import torch

    from oracle import unet as ou
    from paper_2602_08642_amd import ops, pipeline

    kspec = pipeline.kernel_spec(cfg)
    heads = cfg.head_channels()

    def errs(got, ref):
        out = []
        for l, K in enumerate(heads):
            y = got[l][..., :K].double().cpu().numpy()
            r = ref[l].numpy()
            rms = float(np.sqrt(np.mean(r * r)))
            out.append({"head": l, "K": K,
                        "normwise": float(f"{np.linalg.norm(y - r) / np.linalg.norm(r):.3e}"),
                        "max_elem": float(f"{np.max(np.abs(y - r) / (np.abs(r) + rms)):.3e}")})
        return out

    res = {"what": "U-Net logits of the oracle frame's features; per head: normwise relative error and "
                   "max abs(y - r) / (abs(r) + rms(r))"}
    for dt in (cfg.net_dtype, torch.bfloat16):
        key = "fp32" if dt == torch.float32 else "bf16"
        if key in res:
            continue
        net = ops.Net(kspec, kw, dt, dev)
        x = feat.to(dt)
        got = ops.kernel_predict(net, x.float().to(dev).to(dt), heads, dt)
        if dt == cfg.net_dtype and dt == torch.float32:
            ref = logits_ref
        else:
            wq = {k: (torch.tensor(a).to(dt).double(), torch.tensor(b).double()) for k, (a, b) in kw.items()}
            ref = ou.unet_forward(x.double(), wq, len(heads))
        res[key] = errs(got, ref)
        del net, got
    return res


def bench_config(name, steps, warmup, dev, seed=2602):
    """Time one frame configuration; returns the per-config result dict."""
    import torch

    import procgen
    from paper_2602_08642_amd import ops, pipeline

    cfg = pipeline.CONFIGS[name]
    dspec, kspec = pipeline.density_spec(cfg), pipeline.kernel_spec(cfg)
    dw = procgen.init_weights(dspec, 7)
    kw = procgen.init_weights(kspec, 8)
    sc = procgen.make_scene(seed, cfg.H, cfg.W)
    motion = procgen.camera_motion(seed)
    fr = procgen.make_frame(sc, 1 if cfg.temporal else 0, motion)
    aux = torch.tensor(fr.aux[None], device=dev)
    pool = torch.tensor(procgen.sample_pool(fr.truth, seed, 1, 8), device=dev)
    mv = torch.tensor(fr.mv[None], device=dev) if cfg.temporal else None
    prev = None
    if cfg.temporal:   # previous HDR output: the noise-free truth of frame 0 stands in for it
        f0 = procgen.make_frame(sc, 0, motion)
        pt = torch.zeros((1, cfg.H, cfg.W, 4), dtype=torch.float32)
        pt[0, ..., :3] = torch.tensor(f0.truth)
        prev = pt.to(dev)
    del fr, sc
    learned = pipeline.FrameRenderer(cfg, dw, kw, dev)
    uniform = pipeline.FrameRenderer(cfg, None, None, dev, uniform=True)
    frame = 1
    # pre-render the (deterministic) sample requests of both paths
    s_l = learned.density(aux, prev, mv)
    req_l = learned.request(s_l, seed, frame)
    smp_l = ops.fixture_render(pool, req_l["count"], req_l["pixel_offset"], req_l["capacity"])
    s_u = uniform.density(aux)
    req_u = uniform.request(s_u, seed, frame)
    smp_u = ops.fixture_render(pool, req_u["count"], req_u["pixel_offset"], req_u["capacity"])
    del pool
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def run(r, smp, events=None):
        def mark(k):
            if events is not None:
                events[k].record(stream)
        mark(0)
        s = r.density(aux, prev, mv)
        mark(1)
        req = r.request(s, seed, frame)
        mark(2)
        Ls = ops.scatter_samples(s, req["count"], req["pixel_offset"], smp, cfg.levels, "hard",
                                 10.0, seed, frame, u_tex=r.u_tex)
        mark(3)
        if r.knet is not None:
            feat = ops.assemble_features("kernel", aux, Ls[0], s, prev, mv, cfg.kernel_cin, cfg.net_dtype,
                                         lat=r._lat(prev))
        mark(4)
        zmap = None
        if r.knet is not None:
            z, zmap = r.kernel_logits(feat)
        else:
            z = r.logits(aux, Ls[0], s)
        mark(5)
        out = r.filter(Ls, z, prev, mv, zmap=zmap)
        mark(6)
        return out

    def timed(r, smp):
        for _ in range(warmup):
            run(r, smp)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            run(r, smp, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stages = [[evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)] for i in range(6)]
        frame_ms = [evs[k][0].elapsed_time(evs[k][6]) for k in range(steps)]
        return wall, frame_ms, stages

    wall_l, fms_l, st_l = timed(learned, smp_l)
    wall_u, fms_u, st_u = timed(uniform, smp_u)
    mean = lambda v: sum(v) / len(v)
    ms = wall_l * 1e3 / steps
    names = ["density", "mask", "scatter_pyramid", "features", "unet", "filter"]
    flops = unet_flops(cfg, kspec)
    unet_ms = mean(st_l[4])
    filt_ms = mean(st_l[5])
    fbytes = filter_bytes(cfg)
    fp32 = cfg.net_dtype == torch.float32
    peak = PEAK["fp32_mfma_TFLOPs"] if fp32 else PEAK["bf16_mfma_TFLOPs"]
    achieved = flops / (unet_ms * 1e-3) / 1e12
    fgbs = fbytes / (filt_ms * 1e-3) / 1e9
    return dict(
        cfg=cfg, dw=dw, kw=kw, ms=ms, fps=1e3 / ms, mpx=cfg.H * cfg.W / (ms * 1e3),
        event_ms=mean(fms_l), stages={n: round(mean(v), 4) for n, v in zip(names, st_l)},
        uniform={"ms_per_frame": round(wall_u * 1e3 / steps, 4),
                 "Mpixel_per_s": round(cfg.H * cfg.W / (wall_u * 1e6 / steps), 3),
                 "stages_ms": {n: round(mean(v), 4) for n, v in zip(names, st_u)},
                 "what": "s = B everywhere, all-zero logits (box-weighted pyramid)"},
        roofline={"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                  "frac": round(achieved / peak, 4), "traffic": measured_traffic(name),
                  "kernel": ("U-Net MFMA convolutions (row-sweep and tiled implicit-GEMM 3x3, 1x1 heads), "
                             "all launches of one frame"),
                  "algorithmic_flop_per_frame": flops},
        filter_roofline={"bound": "hbm", "achieved": round(fgbs, 1), "peak": PEAK["hbm_GBps"],
                         "unit": "GB/s", "frac": round(fgbs / PEAK["hbm_GBps"], 4),
                         "algorithmic_bytes_per_frame": fbytes},
        workload=(f"{cfg.name}: {cfg.W}x{cfg.H} frame, {cfg.budget} spp, {cfg.levels}-level kd "
                  f"{cfg.KD}x{cfg.KD} / ku {cfg.KU}x{cfg.KU}"
                  + (f" / kt {cfg.KT}x{cfg.KT}" if cfg.temporal else "")
                  + f", U-Net 32-64-128-256 with {cfg.levels} heads ({'fp32' if fp32 else 'bf16'} MFMA)"
                  + (", sampler at quarter resolution" if cfg.density_scale == 2 else "")
                  + (", blue-noise u" if cfg.u_noise == "blue" else "")
                  + (", learned demodulation" if cfg.demod else "")
                  + (", recurrent latents" if cfg.latents else "")))


def bench_train(dev, steps=3, warmup=1):
    """One C4 training step (batch of 4 clips of 8 frames at 256x256, 0.25 spp budget range,
    bf16 networks with fp32 masters): every frame forward and backward through both networks,
    the relaxed sampling step, the filter and the loss, then AdamW.  The clips are generated
    before timing.  FLOPs: the U-Net and sampler forward per frame times 3 (forward, data
    gradient and weight gradient), the forward recomputation inside the filter backward not
    counted."""
    import torch

    from paper_2602_08642_amd import pipeline, train
    cfg = pipeline.CONFIGS["c4"]
    tc = train.TrainConfig(steps=warmup + steps, batch=4, frames=8, n_train_clips=4)
    tr = train.Trainer(cfg, tc, dev)
    tr.clips(0)
    for _ in range(warmup):
        tr.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    dspec, kspec = pipeline.density_spec(cfg), pipeline.kernel_spec(cfg)
    px = cfg.H * cfg.W
    fwd = unet_flops(cfg, kspec) + sum(2 * l["k"] * l["k"] * l["cin"] * l["cout"] * px for l in dspec)
    flops = 3 * fwd * tc.batch * tc.frames
    achieved = flops / (ms * 1e-3) / 1e12
    return {"workload": f"c4: {tc.batch} clips x {tc.frames} frames of {cfg.W}x{cfg.H}, bf16 networks, "
                        "relaxed sampling step, window-2 truncated back-propagation, AdamW",
            "ms_per_step": round(ms, 2), "steps": steps, "warmup": warmup,
            "mfma": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["bf16_mfma_TFLOPs"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["bf16_mfma_TFLOPs"], 4),
                     "flop_per_step": flops}}


WEIGHTS = os.path.join(ROOT, "paper_2602_08642_amd", "weights", "c4_trained.npz")
CSRC = os.path.join(ROOT, "paper_2602_08642_amd", "csrc")
TRAFFIC_SOURCES = ("aps_common.h", "mfma_frag.h", "conv.hip", "net.hip")


def source_digest(names=TRAFFIC_SOURCES):
    """Digest of the sources the U-Net's convolution launches are built from."""
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(config):
    """HBM bytes per U-Net pass from the committed PMC summary of this configuration
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings), or None when there is none
    or the convolution sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"unet_{config}_pmc_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":", 1)[0].strip() in ("digest", "traffic_bytes_per_frame"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("digest") != source_digest():
        return None
    return int(fields["traffic_bytes_per_frame"])


def quality(dev):
    """Learned vs uniform vs fallback error of the trained C4 weights on 16 held-out procedural
    clips (256x256, 8 frames, 0.25 spp): the paired per-clip PSNR gain with its 95 % interval,
    and the uniform budget that matches the learned error."""
    from paper_2602_08642_amd import evaluate
    if not os.path.exists(WEIGHTS):
        return None
    return evaluate.compare_trained(WEIGHTS, device=dev)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--also", default="c3,c5,paper", help="other configurations timed beside (or '')")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the frame the CPU oracle processes (0: the whole frame)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-train", action="store_true", help="skip the C4 training-step timing")
    ap.add_argument("--only-train", action="store_true", help="only the C4 training-step timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scales the HBM "
                         "traffic counters FETCH_SIZE / WRITE_SIZE of a profiled run)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "repeats": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding a frame over "
                                   "several GPUs is not built"}))
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only_train:
        print(json.dumps({"training_step": bench_train(dev, steps=args.steps, warmup=args.warmup)}))
        return
    r = bench_config(args.config, args.steps, args.warmup, dev)
    cfg = r["cfg"]
    res = {
        "metric": "ms/frame & Mpixel/s at 1080p 0.25spp, learned vs uniform sampling at equal error",
        "value": round(r["mpx"], 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg.net_dtype == torch.float32 else "bf16",
        "data": "synthetic (procedural blobs+polygons scene, seeded random-init weights)",
        "config": {"workload": r["workload"], "global_batch": 1, "frames_per_step": 1},
        "frames_per_s": round(r["fps"], 2),
        "ms_per_frame_event_mean": round(r["event_ms"], 4),
        "stages_ms": r["stages"],
        "uniform_fallback": r["uniform"],
        "roofline": r["roofline"],
        "filter_roofline": r["filter_roofline"],
    }
    also = {}
    for name in [a for a in args.also.split(",") if a and a != args.config]:
        o = bench_config(name, max(3, args.steps // 2), max(1, args.warmup // 2), dev)
        also[name] = {"workload": o["workload"], "ms_per_frame": round(o["ms"], 4),
                      "frames_per_s": round(o["fps"], 2), "Mpixel_per_s": round(o["mpx"], 3),
                      "stages_ms": o["stages"], "uniform_fallback": o["uniform"],
                      "roofline": o["roofline"], "filter_roofline": o["filter_roofline"]}
        del o
        torch.cuda.empty_cache()
    if also:
        res["also_timed"] = also
    if not args.no_train:
        res["training_step"] = bench_train(dev)
        torch.cuda.empty_cache()
    if not args.no_quality:
        q = quality(dev)
        if q is not None:
            res["learned_vs_uniform"] = q
    if not args.no_cpu_baseline:
        cb, feat, logits = cpu_baseline(cfg, r["dw"], r["kw"], args.cpu_rows or cfg.H)
        # one thread on a band of about an eighth of the rows (a multiple of 8 for the U-Net)
        cb["one_core"] = cpu_baseline_1core(cfg, r["dw"], r["kw"], max(8, (args.cpu_rows or cfg.H) // 64 * 8))
        res["cpu_baseline"] = cb
        res["precision_vs_fp64"] = precision_vs_oracle(cfg, r["kw"], feat, logits, dev)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

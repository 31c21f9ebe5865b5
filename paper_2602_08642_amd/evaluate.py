"""Learned density vs uniform sampling at equal spp, and the equal-error budget ratio.

    python -m paper_2602_08642_amd.evaluate --steps 300 --out results.json [--save weights.npz]
    python -m paper_2602_08642_amd.evaluate --steps 400 --estimators relaxed,straight_through,gumbel,dasr

Three reconstructions on held-out procedural clips (scene seeds disjoint from training):
  learned   sampler CNN + kernel U-Net trained jointly (relaxed stochastic rounding)
  uniform   s = B everywhere, kernel U-Net trained with uniform sampling ("Ours Uniform")
  fallback  s = B everywhere, all-zero logits (box-weighted pyramid), no training
Then the uniform variant is evaluated at larger budgets; the budget at which it matches the
learned variant's error at B (linear interpolation of PSNR in the budget) gives the sample
saving at equal error.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np
import torch

from . import pipeline, train


def save_weights(path, dnet, knet_l, knet_u):
    arrs = {}
    for tag, net in (("density", dnet), ("kernel_learned", knet_l), ("kernel_uniform", knet_u)):
        if net is None:
            continue
        for name, (w, b) in net.weights().items():
            arrs[f"{tag}/{name}/w"] = w
            arrs[f"{tag}/{name}/b"] = b
    np.savez_compressed(path, **arrs)


def load_weights(path):
    z = np.load(path)
    out = {}
    for key in z.files:
        tag, name, kind = key.split("/")
        d = out.setdefault(tag, {})
        w, b = d.get(name, (None, None))
        d[name] = (z[key], b) if kind == "w" else (w, z[key])
    return out


# held-out scene seeds (training uses seeds 0..1023)
HELD_OUT = tuple(range(10000, 10016))


def paired_gain(a, b):
    """Paired per-clip PSNR differences a - b (same clips, same sample pools): mean, standard
    deviation, two-sided 95 % Student-t interval of the mean, and the clips where a is better."""
    from scipy import stats
    d = np.asarray(a["psnr_per_clip"], np.float64) - np.asarray(b["psnr_per_clip"], np.float64)
    n = d.size
    m, sd = float(d.mean()), float(d.std(ddof=1))
    h = float(stats.t.ppf(0.975, n - 1)) * sd / np.sqrt(n)
    return {"clips": int(n), "mean_db": round(m, 4), "sd_db": round(sd, 4),
            "ci95_db": [round(m - h, 4), round(m + h, 4)], "clips_better": int((d > 0).sum())}


def equal_error_budget(target_psnr, sweep):
    """Uniform budget whose PSNR equals target_psnr (linear interpolation of PSNR over the
    budget sweep), or None outside the sweep."""
    for a, b in zip(sweep[:-1], sweep[1:]):
        if a["psnr"] <= target_psnr <= b["psnr"] and b["psnr"] > a["psnr"]:
            return a["budget"] + (target_psnr - a["psnr"]) / (b["psnr"] - a["psnr"]) * (b["budget"] - a["budget"])
    return None


def compare_trained(weights_path, seeds=HELD_OUT, frames=8, device="cuda",
                    budgets=(0.25, 0.3, 0.35, 0.4, 0.5, 0.6, 0.75, 1.0)):
    """The shipped C4 weights on held-out clips at 0.25 spp: learned (sampler + kernels), uniform
    sampling with its own kernels ("Ours Uniform", Sec. 7) and the fixed-kernel fallback; the
    paired learned - uniform PSNR gain with its 95 % interval, and the uniform budget of equal
    error."""
    w = load_weights(weights_path)
    cfg = pipeline.CONFIGS["c4"]
    dnet = train.TrainNet(pipeline.density_spec(cfg), w["density"], cfg.net_dtype, device)
    kl = train.TrainNet(pipeline.kernel_spec(cfg), w["kernel_learned"], cfg.net_dtype, device)
    ku = train.TrainNet(pipeline.kernel_spec(cfg), w["kernel_uniform"], cfg.net_dtype, device)
    seeds = list(seeds)
    res = {"workload": f"held-out procedural {cfg.W}x{cfg.H} clips (scene seeds {seeds[0]}-{seeds[-1]}) x "
                       f"{frames} frames, {cfg.budget} spp, hard mask",
           "learned": train.evaluate(cfg, dnet, kl, seeds, frames, device),
           "uniform": train.evaluate(cfg, None, ku, seeds, frames, device, uniform=True),
           "fallback": train.evaluate(cfg, None, None, seeds, frames, device, uniform=True)}
    sweep = [res["uniform"]] + [train.evaluate(cfg, None, ku, seeds, frames, device, uniform=True, budget=b)
                                for b in budgets if b != cfg.budget]
    eq = equal_error_budget(res["learned"]["psnr"], sweep)
    res["paired_gain_vs_uniform"] = paired_gain(res["learned"], res["uniform"])
    res["paired_gain_vs_fallback"] = paired_gain(res["learned"], res["fallback"])
    res["uniform_budget_sweep_psnr"] = {str(e["budget"]): round(e["psnr"], 3) for e in sweep}
    res["equal_error_uniform_spp"] = None if eq is None else round(eq, 4)
    res["equal_error_sample_ratio"] = None if eq is None else round(eq / cfg.budget, 3)
    for k in ("learned", "uniform", "fallback"):
        res[k] = {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in res[k].items()
                  if kk != "psnr_per_clip"}
    return res


def run(steps=300, batch=4, frames=8, lr=1e-3, eval_seeds=tuple(range(10000, 10008)),
        budgets=(0.25, 0.3, 0.35, 0.4, 0.5, 0.6, 0.75, 1.0), device="cuda", cfg_name="c4", log=print,
        H=None):
    cfg = pipeline.CONFIGS[cfg_name]
    if H is not None:
        cfg = dataclasses.replace(cfg, H=H, W=H)
    res = {"config": cfg_name, "H": cfg.H, "W": cfg.W, "budget": cfg.budget, "steps": steps,
           "batch": batch, "frames": frames}
    t0 = time.time()
    dnet, knet_l, hist_l = train.train(cfg, train.TrainConfig(steps=steps, batch=batch, frames=frames, lr=lr),
                                       device, log=lambda m: log("[learned] " + m))
    res["train_learned_s"] = round(time.time() - t0, 1)
    t1 = time.time()
    _, knet_u, hist_u = train.train(cfg, train.TrainConfig(steps=steps, batch=batch, frames=frames, lr=lr,
                                                           uniform=True),
                                    device, log=lambda m: log("[uniform] " + m))
    res["train_uniform_s"] = round(time.time() - t1, 1)
    res["loss_learned"] = [hist_l[0]["loss"], float(np.mean([h["loss"] for h in hist_l[-10:]]))]
    res["loss_uniform"] = [hist_u[0]["loss"], float(np.mean([h["loss"] for h in hist_u[-10:]]))]
    seeds = list(eval_seeds)
    res["learned"] = train.evaluate(cfg, dnet, knet_l, seeds, frames, device)
    res["uniform"] = train.evaluate(cfg, None, knet_u, seeds, frames, device, uniform=True)
    res["fallback"] = train.evaluate(cfg, None, None, seeds, frames, device, uniform=True)
    sweep = [train.evaluate(cfg, None, knet_u, seeds, frames, device, uniform=True, budget=b)
             for b in budgets]
    res["uniform_budget_sweep"] = sweep
    target = res["learned"]["psnr"]
    eq = None
    for a, b in zip(sweep[:-1], sweep[1:]):
        if a["psnr"] <= target <= b["psnr"] and b["psnr"] > a["psnr"]:
            f = (target - a["psnr"]) / (b["psnr"] - a["psnr"])
            eq = a["budget"] + f * (b["budget"] - a["budget"])
            break
    res["equal_error_uniform_budget"] = eq
    res["equal_error_sample_ratio"] = None if eq is None else eq / cfg.budget
    if eq is None and all(s["psnr"] < target for s in sweep):
        res["equal_error_sample_ratio_lower_bound"] = budgets[-1] / cfg.budget
    res["psnr_gain_db"] = res["learned"]["psnr"] - res["uniform"]["psnr"]
    return res, (dnet, knet_l, knet_u)


def compare_estimators(estimators=("relaxed", "straight_through", "gumbel", "dasr"), steps=400, batch=4,
                       frames=8, lr=1e-3, eval_seeds=tuple(range(10000, 10008)), device="cuda",
                       cfg_name="c4", tau=0.5, log=print):
    """Train the learned variant (sampler + kernels) with each gradient estimator of the sampling
    step under the same schedule, and evaluate each with its own test-time forward (the hard mask;
    deterministic rounding for DASR) at the configuration's budget."""
    cfg = pipeline.CONFIGS[cfg_name]
    res = {"config": cfg_name, "H": cfg.H, "W": cfg.W, "budget": cfg.budget, "steps": steps,
           "batch": batch, "frames": frames, "tau": tau, "estimators": {}}
    for est in estimators:
        t0 = time.time()
        dnet, knet, hist = train.train(cfg, train.TrainConfig(steps=steps, batch=batch, frames=frames, lr=lr,
                                                              estimator=est, tau=tau),
                                       device, log=lambda m, e=est: log(f"[{e}] " + m))
        ev = train.evaluate(cfg, dnet, knet, list(eval_seeds), frames, device,
                            mode="dasr" if est == "dasr" else "hard")
        ev["train_s"] = round(time.time() - t0, 1)
        ev["loss_first_last10"] = [hist[0]["loss"], float(np.mean([h["loss"] for h in hist[-10:]]))]
        res["estimators"][est] = ev
        log(f"[{est}] psnr {ev['psnr']:.3f} relmse {ev['relmse']:.4f}")
    return res


VARIANTS = {
    "plain": {},
    "demod": {"demod": True},
    "demod_latents": {"demod": True, "latents": 4},
}


def compare_variants(variants=("plain", "demod", "demod_latents"), steps=400, batch=4, frames=8, lr=1e-3,
                     eval_seeds=tuple(range(10000, 10008)), device="cuda", cfg_name="c4", log=print):
    """Train the learned variant (sampler + kernels, relaxed estimator) with and without learned
    demodulation (Sec. 6.2) and the recurrent latents (Sec. 3) under the same schedule, and
    evaluate each on the same held-out clips (hard mask) at the configuration's budget."""
    base = pipeline.CONFIGS[cfg_name]
    res = {"config": cfg_name, "H": base.H, "W": base.W, "budget": base.budget, "steps": steps,
           "batch": batch, "frames": frames, "variants": {}}
    for name in variants:
        cfg = dataclasses.replace(base, **VARIANTS[name])
        t0 = time.time()
        dnet, knet, hist = train.train(cfg, train.TrainConfig(steps=steps, batch=batch, frames=frames, lr=lr),
                                       device, log=lambda m, v=name: log(f"[{v}] " + m))
        ev = train.evaluate(cfg, dnet, knet, list(eval_seeds), frames, device)
        ev["train_s"] = round(time.time() - t0, 1)
        ev["loss_first_last10"] = [hist[0]["loss"], float(np.mean([h["loss"] for h in hist[-10:]]))]
        res["variants"][name] = ev
        log(f"[{name}] psnr {ev['psnr']:.3f} relmse {ev['relmse']:.4f}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None)
    ap.add_argument("--estimators", default=None,
                    help="comma list (relaxed,straight_through,gumbel,dasr): train and compare them")
    ap.add_argument("--variants", default=None,
                    help="comma list (plain,demod,demod_latents): train and compare them")
    a = ap.parse_args()
    if a.variants:
        res = compare_variants(tuple(a.variants.split(",")), a.steps, a.batch, a.frames, a.lr,
                               log=lambda m: print(m, flush=True))
        print(json.dumps(res))
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)
        return
    if a.estimators:
        res = compare_estimators(tuple(a.estimators.split(",")), a.steps, a.batch, a.frames, a.lr,
                                 log=lambda m: print(m, flush=True))
        print(json.dumps(res))
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)
        return
    res, nets = run(a.steps, a.batch, a.frames, a.lr, H=a.size, log=lambda m: print(m, flush=True))
    print(json.dumps(res))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    if a.save:
        save_weights(a.save, *nets)


if __name__ == "__main__":
    main()

"""Training of the sampler CNN and the kernel-predictor U-Net on frames the pipeline itself
generates (procedural clips, renderer stand-in), with the library's forward and backward
kernels behind torch.autograd.Function (Sec. 6.3).

* Relaxed stochastic rounding in training (Sec. 4.3, lambda = 10); the hard mask at test time.
* Loss per frame: tonemapped max(1.25 temporal, spatial) with randomised filmic parameters.
* Sliding window of two frames: frame t takes frame t-1's output (with its graph) as history;
  the gradient of frame t's loss reaches frame t-1's networks but stops there (a gate closes
  once frame t-1's own loss has been propagated).
* AdamW, betas (0.8, 0.985), weight decay 0.02, cosine learning-rate decay, fp32 master weights
  re-packed into the bf16 (or fp32) working copies after every step.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import autograd as ag
from . import ops
from .pipeline import FrameConfig, density_spec, kernel_spec

F32 = torch.float32


# ------------------------------------------------------------------ data

@dataclasses.dataclass
class ClipBatch:
    aux: torch.Tensor     # [T, N, H, W, 8]
    ref: torch.Tensor     # [T, N, H, W, 4]  noise-free radiance
    mv: torch.Tensor      # [T, N, H, W, 2]
    params: torch.Tensor  # [N, 5] tonemapper (k, alpha, beta, s, h)
    seeds: list


def make_clips(seeds, H, W, T, device, randomise_tmo=True, rng_seed=0):
    import procgen
    N = len(seeds)
    aux = np.zeros((T, N, H, W, 8), np.float32)
    ref = np.zeros((T, N, H, W, 4), np.float32)
    mv = np.zeros((T, N, H, W, 2), np.float32)
    prm = np.zeros((N, 5), np.float32)
    rng = np.random.default_rng([rng_seed, 0x7A0])
    for n, sd in enumerate(seeds):
        frames = procgen.make_clip(sd, H, W, T)
        for t, fr in enumerate(frames):
            aux[t, n] = fr.aux
            ref[t, n, ..., :3] = fr.truth
            mv[t, n] = fr.mv
        kc = -float(np.median(np.log(np.maximum(frames[0].truth, 0) + 1e-4)))
        if randomise_tmo:
            prm[n] = [kc + rng.uniform(-0.5, 0.5), rng.uniform(0.25, 0.6), rng.uniform(0.8, 1.2),
                      rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9)]
        else:
            prm[n] = [kc, 0.4, 1.0, 0.5, 0.5]
    d = lambda a: torch.tensor(a, device=device)
    return ClipBatch(d(aux), d(ref), d(mv), d(prm), list(seeds))


def sample_pool(ref_t, gen, J=8):
    """Renderer stand-in on the device: J noisy samples per pixel, truth * (1 + n),
    n = lognormal(0, 0.8) - E[lognormal(0, 0.8)] (input generation, not the method)."""
    N, H, W, _ = ref_t.shape
    g = torch.randn((N * H * W, J), generator=gen, device=ref_t.device)
    one_n = torch.exp(0.8 * g) - math.exp(0.32) + 1.0
    pool = ref_t.reshape(N * H * W, 1, 4) * one_n.unsqueeze(-1)
    pool[..., 3] = 0
    return pool.contiguous()


# ------------------------------------------------------------------ networks

class TrainNet:
    def __init__(self, spec, weights, dtype, device):
        self.spec = [dict(l) for l in spec]
        self.layers = {}
        self.state = {}
        for l in self.spec:
            w, b = weights[l["name"]]
            wt = torch.tensor(w, dtype=F32, device=device).requires_grad_(True)
            bt = torch.tensor(b, dtype=F32, device=device).requires_grad_(True)
            self.layers[l["name"]] = ag.LayerRef(l, wt, bt, dtype)
            self.state[l["name"]] = [(torch.zeros_like(wt), torch.zeros_like(wt)),
                                     (torch.zeros_like(bt), torch.zeros_like(bt))]

    def params(self):
        for name, lr in self.layers.items():
            yield name, lr.w, self.state[name][0]
            yield name, lr.b, self.state[name][1]

    def refresh(self):
        for lr in self.layers.values():
            lr.refresh()

    def weights(self):
        return {n: (lr.w.detach().cpu().numpy(), lr.b.detach().cpu().numpy()) for n, lr in self.layers.items()}


def density_forward(net: TrainNet, cfg: FrameConfig, aux, prev, mv, lat=None):
    if cfg.density_scale != 1:
        raise NotImplementedError("training runs the sampler at full resolution")
    feat = ag.Features.apply("sampler", aux, None, None, prev, mv, cfg.sampler_cin, cfg.net_dtype, lat)
    L = net.layers
    h = ag.conv(feat, L["d0"])
    h = ag.conv(h, L["d1"])
    z = ag.conv(h, L["d2"], out_dtype=F32, ldy=1)
    N, H, W, _ = z.shape
    return ag.Normalize.apply(z.view(N, H, W), cfg.budget, cfg.uniform_frac)


def unet_forward(net: TrainNet, cfg: FrameConfig, feat):
    L = net.layers
    t = ag.conv(feat, L["enc0a"])
    e0 = ag.conv(t, L["enc0b"])
    t = ag.conv(e0, L["enc1a"], "pool2")
    e1 = ag.conv(t, L["enc1b"])
    t = ag.conv(e1, L["enc2a"], "pool2")
    e2 = ag.conv(t, L["enc2b"])
    t = ag.conv(e2, L["bota"], "pool2")
    e3 = ag.conv(t, L["botb"])
    t = ag.conv(e3, L["dec2a"], "up2cat", x2=e2)
    d2 = ag.conv(t, L["dec2b"])
    t = ag.conv(d2, L["dec1a"], "up2cat", x2=e1)
    d1 = ag.conv(t, L["dec1b"])
    t = ag.conv(d1, L["dec0a"], "up2cat", x2=e0)
    d0 = ag.conv(t, L["dec0b"])
    feats = [d0, d1, d2, e3, e3]
    ks = cfg.head_channels()
    return [ag.conv(feats[l], L[f"head{l}"], "pool2" if l == 4 else "direct", out_dtype=cfg.logit_dtype,
                    ldy=ops.round_kstride(ks[l], cfg.logit_dtype)) for l in range(cfg.levels)]


class _Gate(torch.autograd.Function):
    """Identity whose backward passes the gradient only while the gate is open."""

    @staticmethod
    def forward(ctx, x, gate):
        ctx.gate = gate
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return (g if ctx.gate["open"] else None), None


def frame_forward(dnet, knet, cfg, aux, prev, mv, pool, seed, frame, mode="relaxed",
                  uniform=False, lam=10.0, history=None, want_history=False, tau=0.5, ref=None,
                  lat=None, want_latent=False):
    """One frame with autograd.  prev: the previous output (network inputs); history: the filter's
    temporal input (prev when None; with learned demodulation the previous demodulated
    reconstruction, which want_history returns as a third value).  mode: the sampling step's
    estimator (hard at test time; relaxed, straight_through, gumbel or dasr in training; dasr
    needs the reference radiance ref for its surrogate gradient and is also its own test-time
    forward, deterministic rounding)."""
    N = aux.shape[0]
    lat_in = lat if (cfg.latents and prev is not None) else None
    if uniform or dnet is None:
        s = torch.full((N, cfg.H, cfg.W), cfg.budget, dtype=F32, device=aux.device)
    else:
        s = density_forward(dnet, cfg, aux, prev, mv, lat_in)
    cap = int(N * cfg.H * cfg.W * (cfg.budget + 1)) + 1024
    req = ops.sample_mask(s.detach(), seed, frame, capacity=cap, rounding=ops.MODE_ROUNDING[mode])
    samples = ops.fixture_render(pool, req["count"], req["pixel_offset"], cap)
    if mode == "dasr" and ref is None:
        raise ValueError("the DASR surrogate needs the reference radiance")
    Ls = ag.Scatter.apply(s, req, samples, cfg.levels, mode, lam, seed, frame, tau, ref)
    if knet is None:
        ks = cfg.head_channels()
        logits = [torch.zeros((N, cfg.H >> l, cfg.W >> l, ops.round_kstride(ks[l], cfg.logit_dtype)),
                              dtype=cfg.logit_dtype, device=aux.device) for l in range(cfg.levels)]
    else:
        feat = ag.Features.apply("kernel", aux, Ls[0], s, prev, mv, cfg.kernel_cin, cfg.net_dtype, lat_in)
        logits = unet_forward(knet, cfg, feat)
    hist = prev if history is None else history
    if cfg.demod:
        k0 = cfg.filter_channels()[0]
        Ld = ag.Demod.apply(Ls[0], logits[0], k0, cfg.levels)
        out_h = ag.denoise(list(Ld), logits, cfg.KD, cfg.KU, cfg.KT, hist, mv)
        out = ag.Remod.apply(out_h, logits[0], k0)
    else:
        out = out_h = ag.denoise(list(Ls), logits, cfg.KD, cfg.KU, cfg.KT, hist, mv)
    res = (out, s) + ((out_h,) if want_history else ())
    if want_latent:   # this frame's latents: the four level-0 head channels after the map
        k0 = cfg.filter_channels()[0] + 3
        res += ((logits[0][..., k0:k0 + 4].float().contiguous() if cfg.latents else None),)
    return res


# ------------------------------------------------------------------ training

@dataclasses.dataclass
class TrainConfig:
    steps: int = 200
    batch: int = 4
    frames: int = 8
    lr: float = 1e-3
    train_density: bool = True
    uniform: bool = False
    n_train_clips: int = 64
    seed: int = 0
    log_every: int = 10
    # one model covers a range of budgets (Sec. 6.3): B log-uniform in [lo, hi] per step
    budget_range: tuple = (0.125, 1.0)
    # gradient estimator of the sampling step (Sec. 4.3 and the compared ones); tau for gumbel
    estimator: str = "relaxed"
    tau: float = 0.5


def cosine_lr(step, total, peak):
    return 0.5 * peak * (1.0 + math.cos(math.pi * min(step, total) / max(total, 1)))


class Trainer:
    """The training loop's state (networks, AdamW moments, step count, clip cache) and one step.

    A step trains on one batch of clips: every frame forward and backward through the library's
    kernels (window-2 truncated back-propagation through the temporal loop), then AdamW on the
    fp32 masters with the gradients averaged over the frames.  The gradient-norm guard reduces
    every parameter's sum of squares into one device vector that is read back once per step,
    together with the frame losses; a step with a non-finite norm is skipped."""

    def __init__(self, cfg: FrameConfig, tc: TrainConfig, device="cuda", dw=None, kw=None):
        import procgen
        self.cfg, self.tc, self.device = cfg, tc, device
        dspec, kspec = density_spec(cfg), kernel_spec(cfg)
        dw = dw or procgen.init_weights(dspec, 7)
        if kw is None:
            kw = procgen.init_weights(kspec, 8)
            if cfg.demod or cfg.latents:
                # the demodulation map and the latents start at zero (d = 1: the plain path), so
                # training departs from the path without them instead of from a random map
                hname = kspec[-1]["name"] if cfg.kernel_net == "cnn3" else "head0"
                k0 = cfg.filter_channels()[0]
                w, b = kw[hname]
                w, b = w.copy(), b.copy()
                w[k0:] = 0.0
                b[k0:] = 0.0
                kw = dict(kw)
                kw[hname] = (w, b)
        self.dnet = None if tc.uniform else TrainNet(dspec, dw, cfg.net_dtype, device)
        self.knet = TrainNet(kspec, kw, cfg.net_dtype, device)
        self.nets = [self.knet] + ([] if self.dnet is None else [self.dnet])
        self.params = [(p, mv) for net in self.nets for _, p, mv in net.params()]
        self.pool_clips = [list(range(c * tc.batch, (c + 1) * tc.batch))
                           for c in range(tc.n_train_clips // tc.batch)]
        self.data = {}
        self.gen = torch.Generator(device=device).manual_seed(tc.seed)
        self.step_no = 0
        self.history = []

    def clips(self, ci):
        if ci not in self.data:
            self.data[ci] = make_clips(self.pool_clips[ci], self.cfg.H, self.cfg.W, self.tc.frames,
                                       self.device, rng_seed=ci)
        return self.data[ci]

    def step(self):
        cfg, tc = self.cfg, self.tc
        self.step_no += 1
        step = self.step_no
        cb = self.clips((step - 1) % len(self.pool_clips))
        prev, prev_h, prev_lat, prev_ref, gate = None, None, None, None, None
        losses = []
        lo, hi = tc.budget_range
        bstep = float(math.exp(np.random.default_rng([tc.seed, step]).uniform(math.log(lo), math.log(hi))))
        cfg_s = dataclasses.replace(cfg, budget=bstep)
        for t in range(tc.frames):
            pool = sample_pool(cb.ref[t], self.gen)
            pin = None if prev is None else _Gate.apply(prev, gate)
            hin = None if prev_h is None else (pin if prev_h is prev else _Gate.apply(prev_h, gate))
            lin = None if prev_lat is None else _Gate.apply(prev_lat, gate)
            mv = cb.mv[t] if prev is not None else None
            seed = 1_000_003 * step + t
            out, s, out_h, lat = frame_forward(self.dnet, self.knet, cfg_s, cb.aux[t], pin, mv, pool, seed,
                                               t, "relaxed" if tc.uniform else tc.estimator,
                                               uniform=tc.uniform, history=hin, want_history=True,
                                               tau=tc.tau, ref=cb.ref[t], lat=lin, want_latent=True)
            loss = ag.TMOLoss.apply(out, pin, cb.ref[t], prev_ref, mv, cb.params)
            loss.backward(retain_graph=True)
            if gate is not None:
                gate["open"] = False        # frame t-2 stays out of later windows
            losses.append(loss.detach().reshape(1))
            prev, prev_h, prev_lat, prev_ref, gate = out, out_h, lat, cb.ref[t], {"open": True}
        del prev, prev_h, prev_lat, out, out_h, lat, loss, pin
        # gradient-norm guard: every parameter's sum of squares into one device vector, read back
        # once with the frame losses
        sq = torch.zeros(len(self.params), dtype=F32, device=self.device)
        for i, (p, _) in enumerate(self.params):
            if p.grad is not None:
                ops.sumsq(p.grad, out=sq[i:i + 1])
        host = torch.cat(losses + [sq]).cpu().numpy().astype(np.float64)
        lval, gn = float(host[:len(losses)].mean()), float(host[len(losses):].sum())
        finite = math.isfinite(gn)
        lr = cosine_lr(step - 1, tc.steps, tc.lr)
        if finite:
            for p, (m, v) in self.params:
                if p.grad is not None:
                    ops.adamw_step(p.data, m, v, p.grad, lr, step, grad_scale=1.0 / tc.frames)
            for net in self.nets:
                net.refresh()
        for p, _ in self.params:
            p.grad = None
        rec = dict(step=step, loss=lval, grad_norm=math.sqrt(gn) if finite else float("nan"), lr=lr,
                   budget=bstep, skipped=not finite)
        self.history.append(rec)
        return rec

    # ---- checkpoint / resume: masters, AdamW moments and the step count (the clip cache and
    # the per-step budgets and seeds are functions of the step and the configuration)
    def state_dict(self):
        out = {"step": np.array(self.step_no), "gen": self.gen.get_state().numpy()}
        for tag, net in (("k", self.knet), ("d", self.dnet)):
            if net is None:
                continue
            for name, lr in net.layers.items():
                (mw, vw), (mb, vb) = net.state[name]
                for key, t in (("w", lr.w), ("b", lr.b), ("mw", mw), ("vw", vw), ("mb", mb), ("vb", vb)):
                    out[f"{tag}/{name}/{key}"] = t.detach().cpu().numpy()
        return out

    def save(self, path):
        np.savez(path, **self.state_dict())

    def load(self, path):
        z = np.load(path)
        self.step_no = int(z["step"])
        self.gen.set_state(torch.tensor(z["gen"]))
        for tag, net in (("k", self.knet), ("d", self.dnet)):
            if net is None:
                continue
            for name, lr in net.layers.items():
                (mw, vw), (mb, vb) = net.state[name]
                with torch.no_grad():
                    for key, t in (("w", lr.w), ("b", lr.b), ("mw", mw), ("vw", vw), ("mb", mb), ("vb", vb)):
                        t.copy_(torch.tensor(z[f"{tag}/{name}/{key}"]))
            net.refresh()


def train(cfg: FrameConfig, tc: TrainConfig, device="cuda", log=print, dw=None, kw=None):
    tr = Trainer(cfg, tc, device, dw, kw)
    t0 = time.time()
    for _ in range(tc.steps):
        rec = tr.step()
        step = rec["step"]
        if step % tc.log_every == 0 or step == 1:
            log(f"step {step:4d} loss {rec['loss']:.5f} |g| {rec['grad_norm']:.3e} lr {rec['lr']:.2e} "
                f"{time.time() - t0:.1f}s")
    return tr.dnet, tr.knet, tr.history


# ------------------------------------------------------------------ evaluation

def psnr_tonemapped(out, ref, params):
    """PSNR of the evaluation-tonemapped images (metric only, computed with the loss kernel's
    tonemapper via a zero-temporal call is not needed: plain torch on the outputs)."""
    k, a = params[:, 0].view(-1, 1, 1, 1), params[:, 1].view(-1, 1, 1, 1)

    def tm(x):
        y = torch.log(torch.clamp(x[..., :3], min=0) + 1e-4)
        xx = a * (y + k)
        t = torch.where(xx < -0.5, 0.25 * torch.exp((xx + 0.5) / 0.5),
                        torch.where(xx < 0.5, 0.5 * (1 + xx), 1 - 0.25 * torch.exp(-(xx - 0.5) / 0.5)))
        t = torch.clamp(t, 0, 1)
        return torch.where(t <= 0.0031308, 12.92 * t, 1.055 * torch.pow(torch.clamp(t, min=0.0031308), 1 / 2.4) - 0.055)

    mse = ((tm(out) - tm(ref)) ** 2).mean(dim=(1, 2, 3))
    return (10 * torch.log10(1.0 / mse)).cpu().numpy()


@torch.no_grad()
def evaluate(cfg: FrameConfig, dnet, knet, seeds, frames=8, device="cuda", uniform=False,
             budget=None, gen_seed=123, mode="hard"):
    """Mean tonemapped PSNR and relMSE over held-out clips, hard mask (test time; mode "dasr":
    deterministic rounding, the test-time forward of a DASR-trained sampler); psnr_per_clip:
    each clip's PSNR averaged over its frames, in the order of seeds."""
    if budget is not None:
        cfg = dataclasses.replace(cfg, budget=budget)
    cb = make_clips(seeds, cfg.H, cfg.W, frames, device, randomise_tmo=False)
    gen = torch.Generator(device=device).manual_seed(gen_seed)
    prev = hist = lat = None
    ps, rm = [], []
    for t in range(frames):
        pool = sample_pool(cb.ref[t], gen)
        mv = cb.mv[t] if prev is not None else None
        out, _, hist, lat = frame_forward(None if uniform else dnet, knet, cfg, cb.aux[t], prev, mv, pool,
                                          7_000_001 + t, t, mode, uniform=uniform, history=hist,
                                          want_history=True, ref=cb.ref[t], lat=lat, want_latent=True)
        prev = out
        ps.append(psnr_tonemapped(out, cb.ref[t], cb.params))
        r = cb.ref[t][..., :3]
        rm.append((((out[..., :3] - r) ** 2) / (r ** 2 + 1e-2)).mean().item())
    per_clip = np.mean(np.stack(ps), axis=0)
    return dict(psnr=float(per_clip.mean()), relmse=float(np.mean(rm)), budget=cfg.budget,
                psnr_per_clip=[float(v) for v in per_clip])

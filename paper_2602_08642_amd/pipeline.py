"""Per-frame path: sampler CNN -> budget normalisation -> sample mask -> (renderer) ->
s-normalised scatter + pyramid -> kernel prediction -> gathering pyramid.

Each stage is one or more libaps calls on the current stream; this module only chooses the
configuration and passes buffers between them.
"""
from __future__ import annotations

import dataclasses

import torch

from . import _lib, ops

F32, BF16 = torch.float32, torch.bfloat16


@dataclasses.dataclass(frozen=True)
class FrameConfig:
    name: str
    H: int
    W: int
    budget: float          # samples per pixel, B
    levels: int            # pyramid levels L
    KD: int
    KU: int
    KT: int
    temporal: bool
    net_dtype: torch.dtype    # convolution storage / MFMA input type (fp32 accumulation)
    logit_dtype: torch.dtype
    widths: tuple = (32, 64, 128, 256)
    uniform_frac: float = 1.0 / 8.0   # Sec. 3: 1/8 of the budget spread uniformly
    kernel_net: str = "unet"          # "unet" or "cnn3" (single-level 3-layer CNN)
    density_scale: int = 1            # 2: sampler at a quarter of the pixels (Sec. 7)
    u_noise: str = "philox"           # u of the mask: "philox" or "blue" (void-and-cluster texture)
    demod: bool = False               # learned demodulation (Sec. 6.2): 3 more level-0 head channels
    latents: int = 0                  # recurrent latents shared by both networks (Sec. 3): 0 or 4

    @property
    def sampler_cin(self) -> int:
        return 16 if self.temporal else 8

    @property
    def kernel_cin(self) -> int:
        return 24 if self.latents else 16

    def filter_channels(self):
        """Kernel logits per level (the joint softmax of App. A)."""
        out = []
        for l in range(self.levels):
            k = self.KD * self.KD + (self.KU * self.KU if l < self.levels - 1 else 0)
            if l == 0 and self.temporal:
                k += self.KT * self.KT
            out.append(k)
        return out

    def head_channels(self):
        """U-Net head outputs per level: the kernel logits, and at level 0 the three channels of
        the demodulation map after them when demod is on."""
        out = self.filter_channels()
        if self.demod:
            out[0] += 3
        out[0] += self.latents       # the latent channels follow (they ride with demodulation)
        return out


CONFIGS = {
    # 128x128 single frame, FP32, single-level 5x5 softmax kernel from a 3-layer CNN
    "c1": FrameConfig("c1", 128, 128, 0.25, 1, 5, 3, 3, False, F32, F32, kernel_net="cnn3"),
    # 1080p, 0.25 spp, FP32 throughout, U-Net kernels, 3-level pyramid 5x5, ku 3x3
    "c2": FrameConfig("c2", 1080, 1920, 0.25, 3, 5, 3, 3, False, F32, F32),
    # 1080p, BF16 MFMA U-Net, FP32 filtering, temporal kt 3x3
    "c3": FrameConfig("c3", 1080, 1920, 0.25, 3, 5, 3, 3, True, BF16, BF16),
    # training crops: 256x256, C3's reconstruction
    "c4": FrameConfig("c4", 256, 256, 0.25, 3, 5, 3, 3, True, BF16, BF16),
    # 4K, 0.125 spp, 4-level 7x7 pyramid, BF16 U-Net, temporal
    "c5": FrameConfig("c5", 2160, 3840, 0.125, 4, 7, 3, 3, True, BF16, BF16),
    # the paper's own reconstruction (App. A): 5 levels, kd 5x5 everywhere, literal 2x2 ku,
    # kt 5x5 (54-way softmax at level 0), with the quarter-resolution density map of Sec. 7;
    # 1080 rows are not divisible by 2^4, so the frame is 1080p padded to 1088 rows
    "paper": FrameConfig("paper", 1088, 1920, 0.25, 5, 5, 2, 5, True, BF16, BF16, density_scale=2,
                         u_noise="blue", demod=True, latents=4),
}


def density_spec(cfg: FrameConfig):
    import procgen
    return procgen.density_cnn_spec(cfg.sampler_cin)


def kernel_spec(cfg: FrameConfig):
    import procgen
    if cfg.kernel_net == "cnn3":
        return procgen.small_kernel_cnn_spec(cfg.kernel_cin, 16, cfg.head_channels()[0])
    return procgen.unet_spec(cfg.kernel_cin, cfg.head_channels(), cfg.widths)


class FrameRenderer:
    """Runs the path for one configuration with given network weights.

    uniform=True is the fallback: s = B everywhere (no sampler), and, when no kernel network is
    given, all-zero logits (box-weighted pyramid).
    """

    def __init__(self, cfg: FrameConfig, density_weights=None, kernel_weights=None,
                 device="cuda", uniform=False):
        self.cfg = cfg
        self.device = torch.device(device)
        self.uniform = uniform
        self.dnet = None
        if not uniform:
            self.dnet = ops.Net(density_spec(cfg), density_weights, cfg.net_dtype, self.device)
        self.knet = None
        if kernel_weights is not None:
            self.knet = ops.Net(kernel_spec(cfg), kernel_weights, cfg.net_dtype, self.device)
        if cfg.latents and (cfg.latents != 4 or not cfg.demod or not cfg.temporal):
            raise ValueError("recurrent latents are 4 channels and need demodulation and a temporal config")
        self._const_logits = None
        self.history = None
        self.latent = None      # the latest frame's latents [N,H,W,4], read by the next frame
        self.zmap = None        # the latest frame's compact demodulation map (kernel_logits)
        self.u_tex = None
        if cfg.u_noise == "blue":   # a 64x64 void-and-cluster threshold texture (Sec. 6.3)
            import procgen
            self.u_tex = torch.tensor(procgen.blue_noise_thresholds(64), device=self.device)
        elif cfg.u_noise != "philox":
            raise ValueError(cfg.u_noise)

    # -- stage 1: density ------------------------------------------------------------
    def density(self, aux, prev=None, mv=None):
        cfg = self.cfg
        N = aux.shape[0]
        if self.uniform:
            return torch.full((N, cfg.H, cfg.W), cfg.budget, dtype=F32, device=self.device)
        feat = ops.assemble_features("sampler", aux, prev=prev, mv=mv, C_out=cfg.sampler_cin,
                                     dtype=cfg.net_dtype, lat=self._lat(prev))
        if cfg.density_scale == 2:
            # quarter resolution: the budget per pixel is unchanged, so sum(s) stays Npx * B
            _, s_q = ops.density_predict(self.dnet, ops.avgpool2(feat), cfg.budget, cfg.uniform_frac)
            return ops.upsample_nearest2(s_q)
        _, s = ops.density_predict(self.dnet, feat, cfg.budget, cfg.uniform_frac)
        return s

    # -- stage 2: sample request ---------------------------------------------------------
    def request(self, s, seed: int, frame: int):
        N = s.shape[0]
        cap = int(N * self.cfg.H * self.cfg.W * (self.cfg.budget + 1.0)) + 1024
        return ops.sample_mask(s, seed, frame, capacity=cap, u_tex=self.u_tex)

    # -- stage 3: reconstruction -----------------------------------------------------------
    def logits(self, aux, L0, s, prev=None, mv=None):
        cfg = self.cfg
        N = aux.shape[0]
        if self.knet is None:
            if self._const_logits is None or self._const_logits[0].shape[0] != N:
                ks = cfg.head_channels()
                self._const_logits = [
                    torch.zeros((N, cfg.H >> l, cfg.W >> l, ops.round_kstride(ks[l], cfg.logit_dtype)),
                                dtype=cfg.logit_dtype, device=self.device) for l in range(cfg.levels)]
            return self._const_logits
        feat = ops.assemble_features("kernel", aux, L0, s, prev, mv, cfg.kernel_cin, cfg.net_dtype,
                                     lat=self._lat(prev))
        if cfg.kernel_net == "cnn3":
            h = feat
            for l in self.knet.spec:
                sp, pk, b = self.knet.layer(l["name"])
                last = l is self.knet.spec[-1]
                ld = ops.round_kstride(l["cout"], cfg.logit_dtype) if last else None
                h = ops.conv2d(h, sp, pk, b, out_dtype=cfg.logit_dtype if last else None, ldy=ld)
            return [h]
        z, self.zmap = self.kernel_logits(feat)
        return z

    def kernel_logits(self, feat):
        """U-Net logits, and with learned demodulation the compact [N,H,W,4] map that the fused
        level-0 head writes beside them (None where that head cannot write it: the map is then
        read from the logit rows)."""
        cfg = self.cfg
        if cfg.demod and cfg.logit_dtype == cfg.net_dtype:
            try:
                return ops.kernel_predict(self.knet, feat, cfg.head_channels(), cfg.logit_dtype,
                                          side_offset=cfg.filter_channels()[0])
            except _lib.ApsError as e:
                if e.status != _lib.APS_ERR_UNSUPPORTED:
                    raise
        return ops.kernel_predict(self.knet, feat, cfg.head_channels(), cfg.logit_dtype), None

    def reconstruct(self, aux, s, req, samples, seed: int, frame: int, prev=None, mv=None,
                    mode="hard", lam=10.0, history=None):
        cfg = self.cfg
        Ls = ops.scatter_samples(s, req["count"], req["pixel_offset"], samples, cfg.levels, mode,
                                 lam, seed, frame, u_tex=self.u_tex)
        use_prev = prev if cfg.temporal else None
        use_mv = mv if cfg.temporal else None
        self.zmap = None
        z = self.logits(aux, Ls[0], s, use_prev, use_mv)
        hist = (history if history is not None else prev) if cfg.temporal else None
        out, self.history = self.filter(Ls, z, hist, use_mv, want_history=True, zmap=self.zmap)
        return out, Ls, z

    def _lat(self, prev):
        """The previous frame's latents, when there is a previous frame."""
        if not self.cfg.latents or prev is None or self.latent is None:
            return None
        return self.latent

    def filter(self, Ls, z, history=None, mv=None, want_history=False, zmap=None):
        """Gathering pyramid.  With learned demodulation the pyramid of L0 / d is filtered and the
        result multiplied by d (d from the level-0 head channels after the kernel logits); the
        filter then works in demodulated space throughout, so its temporal input (history) is the
        previous frame's demodulated reconstruction, which want_history also returns.  zmap: the
        compact copy of those three channels (kernel_logits), else they are read from z[0]."""
        cfg = self.cfg
        if cfg.demod:
            k0 = cfg.filter_channels()[0]
            if zmap is not None:
                Ld = ops.demodulate(Ls[0], zmap, 0, cfg.levels)
            else:
                Ld = ops.demodulate(Ls[0], z[0], k0, cfg.levels)
            out_d = torch.empty_like(Ls[0])
            lat = None
            if cfg.latents:   # copied from the level-0 logit rows the map is read from
                lat = torch.empty_like(Ls[0])
            # remodulation (and the latent copy) happen in the level-0 filter kernel
            out = ops.denoise_pyramid(Ld, z, cfg.KD, cfg.KU, cfg.KT, history, mv, demod_offset=k0,
                                      lat_offset=k0 + 3 if cfg.latents else -1, out_demod=out_d,
                                      lat_out=lat)
            if lat is not None:
                self.latent = lat
            return (out, out_d) if want_history else out
        out = ops.denoise_pyramid(Ls, z, cfg.KD, cfg.KU, cfg.KT, history, mv)
        return (out, out) if want_history else out

    def step(self, aux, render, seed: int, frame: int, prev=None, mv=None, history=None):
        """One frame; render(req) -> samples [capacity, 4] stands in for the path tracer.  prev is
        the previous output (network inputs); history the filter's temporal input (the previous
        "history" entry; prev when not given)."""
        s = self.density(aux, prev if self.cfg.temporal else None, mv if self.cfg.temporal else None)
        req = self.request(s, seed, frame)
        samples = render(req)
        out, Ls, z = self.reconstruct(aux, s, req, samples, seed, frame, prev, mv, history=history)
        return dict(out=out, history=self.history, s=s, req=req, L=Ls, logits=z)

"""torch.autograd.Function wrappers: every forward and backward is a libaps call.

Conv          one conv layer (fused pool / upsample+concat input, bias, ReLU); gradients for
              its input(s), fp32 master weight and bias (dgrad on MFMA with the transposed
              operator, wgrad on MFMA with a deterministic split-K).
Normalize     budget normalisation z -> s.
Scatter       s -> pyramid levels of the s-normalised estimate (hard or relaxed holdout);
              gradient w.r.t. s only (the renderer is not differentiated, as in the paper).
Features      network-input assembly; gradients to L0, s and the previous output.
Denoise       the gathering pyramid; coarse levels recomputed in the backward.
TMOLoss       tonemapped spatial + temporal loss of one frame.
"""
from __future__ import annotations

import torch

from . import ops

F32, BF16 = torch.float32, torch.bfloat16


def _esize(dt):
    return 2 if dt == BF16 else 4


class LayerRef:
    """Packed forward / data-gradient operators of one layer, refreshed after optimizer steps."""

    def __init__(self, spec, w_master, b_master, dtype):
        self.spec, self.w, self.b, self.dtype = spec, w_master, b_master, dtype
        self.refresh()

    def refresh(self):
        lib = ops.L.load()
        n = lib.aps_conv_packed_elems(self.spec["cout"], self.spec["k"], self.spec["cin"])
        if not hasattr(self, "packed") or self.packed.numel() != n:
            self.packed = torch.empty(n, dtype=self.dtype, device=self.w.device)
        ops.L.check(lib.aps_conv_pack_weights(ops._p(self.w.detach()), self.spec["cout"], self.spec["k"],
                                              self.spec["cin"], ops._dt(self.dtype), ops._p(self.packed),
                                              ops._stream()), "pack_weights")
        self.packed_T = ops.pack_dgrad(self.spec, self.w.detach(), self.dtype)


class Conv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, x2, w, b, layer: LayerRef, mode: str, out_dtype, ldy):
        y = ops.conv2d(x, layer.spec, layer.packed, b.detach(), mode, x2, out_dtype=out_dtype, ldy=ldy)
        ctx.layer, ctx.mode = layer, mode
        ctx.save_for_backward(x, x2, y)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, x2, y = ctx.saved_tensors
        layer = ctx.layer
        spec = layer.spec
        gy = gy.contiguous()
        ymask = y if spec["relu"] else None
        ld = gy.shape[-1]
        if gy.dtype != x.dtype or (ld * _esize(x.dtype)) % 16:
            ld8 = (ld + 7) // 8 * 8
            gy = ops.copy_channels(gy, x.dtype, ld8, ld)
        dx, dx2, dw, db = ops.conv2d_bwd(x, x2, ctx.mode, spec, layer.packed_T, gy, ymask,
                                         need_dx=ctx.needs_input_grad[0],
                                         need_dx2=x2 is not None and ctx.needs_input_grad[1])
        return dx, dx2, dw, db, None, None, None, None


def conv(x, layer: LayerRef, mode="direct", x2=None, out_dtype=None, ldy=None):
    return Conv.apply(x, x2, layer.w, layer.b, layer, mode, out_dtype, ldy)


class Normalize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, budget: float, uniform_frac: float):
        ctx.budget, ctx.f = budget, uniform_frac
        ctx.save_for_backward(z)
        return ops.normalize_density(z, budget, uniform_frac)

    @staticmethod
    def backward(ctx, gs):
        (z,) = ctx.saved_tensors
        return ops.normalize_density_bwd(z, ctx.budget, gs.contiguous(), ctx.f), None, None


class Scatter(torch.autograd.Function):
    """The s-normalised scatter with the estimator of `mode` (hard, relaxed, straight_through,
    gumbel with temperature tau, dasr with the reference radiance L_ref for its surrogate)."""

    @staticmethod
    def forward(ctx, s, req: dict, samples, levels: int, mode: str, lam: float, seed: int, frame: int,
                tau: float = 0.5, L_ref=None):
        Ls = ops.scatter_samples(s, req["count"], req["pixel_offset"], samples, levels, mode, lam,
                                 seed, frame, tau=tau)
        ctx.req, ctx.mode, ctx.lam, ctx.seed, ctx.frame, ctx.tau = req, mode, lam, seed, frame, tau
        ctx.L_ref = L_ref
        ctx.save_for_backward(s, samples)
        return tuple(Ls)

    @staticmethod
    def backward(ctx, *gLs):
        s, samples = ctx.saved_tensors
        N, H, W = s.shape
        g = [gl.contiguous() if gl is not None else
             torch.zeros((N, H >> l, W >> l, 4), dtype=F32, device=s.device) for l, gl in enumerate(gLs)]
        gs = ops.scatter_samples_bwd(s, ctx.req["count"], ctx.req["pixel_offset"], samples, g,
                                     ctx.mode, ctx.lam, ctx.seed, ctx.frame, tau=ctx.tau, L_ref=ctx.L_ref)
        return gs, None, None, None, None, None, None, None, None, None


class Features(torch.autograd.Function):
    """Network inputs; lat: the previous frame's recurrent latents [N,H,W,4] (optional)."""

    @staticmethod
    def forward(ctx, kind: str, aux, L0, s, prev, mv, C: int, dtype, lat=None):
        ctx.kind = kind
        ctx.has_lat = lat is not None
        ctx.save_for_backward(L0, prev, mv)
        return ops.assemble_features(kind, aux, L0, s, prev, mv, C, dtype,
                                     lat=None if lat is None else lat.contiguous())

    @staticmethod
    def backward(ctx, gf):
        L0, prev, mv = ctx.saved_tensors
        gf = gf.contiguous()
        gL0 = torch.zeros_like(L0) if (L0 is not None and ctx.needs_input_grad[2]) else None
        gs = (torch.zeros(gf.shape[:3], dtype=F32, device=gf.device)
              if ctx.kind == "kernel" and ctx.needs_input_grad[3] else None)
        gp = torch.zeros_like(prev) if (prev is not None and ctx.needs_input_grad[4]) else None
        gl = (torch.zeros((*gf.shape[:3], 4), dtype=F32, device=gf.device)
              if ctx.has_lat and ctx.needs_input_grad[8] else None)
        ops.assemble_features_bwd(ctx.kind, gf, L0, prev, mv, gL0, gs, gp, has_lat=ctx.has_lat,
                                  grad_lat=gl)
        return None, None, gL0, gs, gp, None, None, None, gl


class Denoise(torch.autograd.Function):
    @staticmethod
    def forward(ctx, KD, KU, KT, mv, prev, levels: int, *tensors):
        Ls, logits = list(tensors[:levels]), list(tensors[levels:])
        out = ops.denoise_pyramid(Ls, logits, KD, KU, KT, prev, mv)
        ctx.k = (KD, KU, KT, levels)
        ctx.save_for_backward(mv, prev, *tensors)
        return out

    @staticmethod
    def backward(ctx, gout):
        KD, KU, KT, levels = ctx.k
        mv, prev, *tensors = ctx.saved_tensors
        Ls, logits = tensors[:levels], tensors[levels:]
        glog, gL, gprev = ops.denoise_pyramid_bwd(list(Ls), list(logits), KD, KU, KT, prev, mv,
                                                  gout.contiguous(), want_prev=prev is not None
                                                  and ctx.needs_input_grad[4])
        return (None, None, None, None, gprev, None, *gL, *glog)


def denoise(Ls, logits, KD, KU, KT, prev=None, mv=None):
    return Denoise.apply(KD, KU, KT, mv, prev, len(Ls), *Ls, *logits)


def _z_grad(z0, k0, gz):
    """dLoss/dz of the three demodulation channels as a gradient of the whole level-0 logits."""
    g = torch.zeros_like(z0)
    g[..., k0:k0 + 3] = gz.to(z0.dtype)
    return g


class Demod(torch.autograd.Function):
    """Learned demodulation (Sec. 6.2): the pyramid of L0 / d, d from the level-0 logits."""

    @staticmethod
    def forward(ctx, L0, z0, k0: int, levels: int):
        ctx.k = (k0, levels)
        ctx.save_for_backward(L0, z0)
        return tuple(ops.demodulate(L0, z0, k0, levels))

    @staticmethod
    def backward(ctx, *gLd):
        k0, levels = ctx.k
        L0, z0 = ctx.saved_tensors
        g = [t.contiguous() if t is not None else torch.zeros((L0.shape[0], L0.shape[1] >> l, L0.shape[2] >> l, 4),
                                                             dtype=torch.float32, device=L0.device)
             for l, t in enumerate(gLd)]
        gL0, gz = ops.demodulate_bwd(L0, z0, k0, g)
        return gL0, _z_grad(z0, k0, gz), None, None


class Remod(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, z0, k0: int):
        ctx.k0 = k0
        ctx.save_for_backward(x, z0)
        return ops.remodulate(x, z0, k0)

    @staticmethod
    def backward(ctx, gout):
        x, z0 = ctx.saved_tensors
        gx, gz = ops.remodulate_bwd(x, z0, ctx.k0, gout.contiguous())
        return gx, _z_grad(z0, ctx.k0, gz), None


class TMOLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, out, prev_out, ref, prev_ref, mv, params):
        loss, gout, gprev = ops.tmo_loss(out, ref, params, prev_out, prev_ref, mv,
                                         want_prev=prev_out is not None)
        ctx.save_for_backward(gout, gprev)
        return loss

    @staticmethod
    def backward(ctx, gl):
        gout, gprev = ctx.saved_tensors
        gl = gl.contiguous().reshape(1).to(F32)
        gout = ops.scale_by(gout.clone(), gl)
        if gprev is not None:
            gprev = ops.scale_by(gprev.clone(), gl)
        return gout, gprev, None, None, None, None

"""Learned demodulation (Sec. 6.2, learned demodulation), FP64.

The denoiser predicts a three-channel map d per pixel; the noisy radiance is divided by d before
the pyramid is built and filtered, and the reconstruction is multiplied by d afterwards.  The
paper does not fix how d is parameterised; here d = exp(z) for three extra channels z of the
level-0 logits, with z clamped to [-8, 8] (d = 1 when z = 0, so an untrained head leaves the
radiance as it is).
"""
import torch

ZMAX = 8.0


def demod_map(z):
    """z [..., 3] -> d = exp(clamp(z, -8, 8))."""
    return torch.exp(torch.clamp(z, -ZMAX, ZMAX))


def demodulate(L0, z, levels: int):
    """L0 [N, H, W, 4] (A unused), z [N, H, W, 3] -> pyramid of L0 / d (App. A eq. app-pyramid
    applied to the demodulated radiance): level l = mean over 2^l x 2^l blocks of level 0."""
    d = demod_map(z)
    Ld = torch.cat([L0[..., :3] / d, torch.zeros_like(L0[..., 3:])], -1)
    out = [Ld]
    for _ in range(1, levels):
        x = out[-1]
        N, H, W, C = x.shape
        out.append(x.reshape(N, H // 2, 2, W // 2, 2, C).mean(dim=(2, 4)))
    return out


def remodulate(out_d, z):
    """out = d * out_d (RGB; A = 0)."""
    d = demod_map(z)
    return torch.cat([out_d[..., :3] * d, torch.zeros_like(out_d[..., 3:])], -1)

"""Differentiable filmic tonemapper and training loss (Sec. 5; Sec. 6.3 eqs.
loss_spatial, loss_temporal, loss_combined), FP64.

I = sRGB(tau(alpha * (sat_beta(log(max(L, 0) + eps)) + k); s, h)), with sat_beta
scaling each channel's log value about the per-pixel log-RGB mean, and the piecewise
curve tau: exponential toe below s-1, line (1+x)/2, exponential shoulder from 1-h.
sRGB is the IEC 61966-2-1 transfer function.
"""
import torch

EPS = 1e-4


def tau(x, s: float, h: float):
    toe = 0.5 * s * torch.exp((x + 1.0 - s) / s)
    lin = 0.5 * (1.0 + x)
    sho = 1.0 - 0.5 * h * torch.exp(-(x + h - 1.0) / h)
    return torch.where(x < s - 1.0, toe, torch.where(x < 1.0 - h, lin, sho))


def srgb(v):
    v = torch.clamp(v, 0.0, 1.0)
    lo = 12.92 * v
    hi = 1.055 * torch.pow(torch.clamp(v, min=0.0031308), 1.0 / 2.4) - 0.055
    return torch.where(v <= 0.0031308, lo, hi)


def tonemap(L, params):
    """L [..., >=3] HDR -> I [..., 3] display values; params = dict(k, alpha, beta, s, h)."""
    y = torch.log(torch.clamp(L[..., :3], min=0.0) + EPS)
    m = y.mean(dim=-1, keepdim=True)
    y = m + params["beta"] * (y - m)
    x = params["alpha"] * (y + params["k"])
    return srgb(tau(x, params["s"], params["h"]))


def frame_loss(I, I_ref, I_prev_w=None, I_ref_prev_w=None, valid=None):
    """mean over pixels and channels of max(1.25 * |dI - dI_ref|, |I - I_ref|) (mask m = 1).
    Without a previous frame only the spatial term remains; the temporal term is zero at
    pixels whose back-projection left the frame."""
    ls = (I - I_ref).abs()
    if I_prev_w is None:
        return ls.mean()
    lt = ((I - I_prev_w) - (I_ref - I_ref_prev_w)).abs()
    if valid is not None:
        lt = lt * valid.unsqueeze(-1).to(lt.dtype)
    return torch.maximum(1.25 * lt, ls).mean()

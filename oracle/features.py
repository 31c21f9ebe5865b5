"""Network inputs, FP64 (Sec. 3, Overview: the sampler sees the GBuffer and the reprojected
tonemapped previous output; the denoiser additionally sees the noisy image).

Channel layout (zero padded to C):
  sampler: albedo 3, normal 3, log-depth 1, then with history: tonemap(W prev) 3, valid 1
  kernel : albedo 3, normal 3, log-depth 1, slog1p(L_noisy) 3, s 1, then with history:
           slog1p(W prev) 3, valid 1
slog1p(v) = sign(v) log(1 + |v|) (samples, hence L, can be negative); tonemap = the filmic
curve of Sec. 5 at s = h = 0.5, contrast 0.4, exposure 0, saturation 1, then sRGB; valid = the
back-projected position x + mv lies inside the frame.
"""
import torch

from .filt import warp
from .tmo import srgb, tau

F64 = torch.float64


def slog1p(v):
    return torch.sign(v) * torch.log1p(v.abs())


def tonemap_eval(L):
    return srgb(tau(0.4 * torch.log(torch.clamp(L, min=0.0) + 1e-4), 0.5, 0.5))


def valid_from_mv(mv):
    N, H, W, _ = mv.shape
    px = torch.arange(W, dtype=F64).reshape(1, 1, W) + mv[..., 0]
    py = torch.arange(H, dtype=F64).reshape(1, H, 1) + mv[..., 1]
    return ((px >= -0.5) & (px <= W - 0.5) & (py >= -0.5) & (py <= H - 0.5)).to(F64)


def _assemble(cols, C):
    N, H, W = cols[0].shape[:3]
    out = torch.zeros(N, H, W, C, dtype=F64)
    o = 0
    parts = []
    for c in cols:
        parts.append(c if c.dim() == 4 else c.unsqueeze(-1))
    x = torch.cat(parts, -1)
    return torch.cat([x, out[..., x.shape[-1]:]], -1)


def sampler_features(aux, prev=None, mv=None, C: int = 8, lat=None):
    """lat: the previous frame's four recurrent latents (Sec. 3: a latent space shared by the
    sampler and the denoiser, fed forward across frames), warped like prev and appended."""
    aux = torch.as_tensor(aux, dtype=F64)
    cols = [aux[..., :7]]
    if prev is not None:
        wp = warp(torch.as_tensor(prev, dtype=F64), mv)
        cols += [tonemap_eval(wp[..., :3]), valid_from_mv(torch.as_tensor(mv, dtype=F64))]
        if lat is not None:
            cols += [warp(torch.as_tensor(lat, dtype=F64), mv)[..., :4]]
    return _assemble(cols, C)


def kernel_features(aux, L0, s, prev=None, mv=None, C: int = 16, lat=None):
    aux = torch.as_tensor(aux, dtype=F64)
    cols = [aux[..., :7], slog1p(L0[..., :3]), s]
    if prev is not None:
        wp = warp(prev, mv)
        cols += [slog1p(wp[..., :3]), valid_from_mv(torch.as_tensor(mv, dtype=F64))]
        if lat is not None:
            cols += [warp(torch.as_tensor(lat, dtype=F64), mv)[..., :4]]
    return _assemble(cols, C)

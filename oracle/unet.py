"""Kernel-predictor U-Net in FP64 (Sec. 6.3 names a U-Net encoder-decoder; its layer
widths and depth here are the 4-level 32-64-128-256 configuration with 3x3 convs).

enc_l: two 3x3 conv + ReLU (level 0 on the input, deeper levels on the 2x2 average pool
of the level above); dec_l: two 3x3 conv + ReLU on concat[nearest-2x(deeper), enc_l];
head_l: 1x1 conv (no activation) on dec_l (on the bottleneck for level 3) giving the
kernel logits of pyramid level l (App. A, kernel prediction).  The five-level pyramid of
App. A (pyramid construction, L = 5) needs logits at 1/16 resolution as well: head 4 reads
the 2x2 average pool of the bottleneck (the paper does not specify its networks; this is
the reading used here).
"""
import torch

from .density import conv2d_nhwc


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(dim=(2, 4))


def up2(x):
    return x.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)


def _cr(x, wb):
    w, b = wb
    return torch.relu(conv2d_nhwc(x, w, b))


def unet_forward(x, wts, n_heads: int):
    """x [N, H, W, Cin] (H, W divisible by 8, by 16 for 5 heads); wts: {name: (w, b)} float64
    tensors."""
    e0 = _cr(_cr(x, wts["enc0a"]), wts["enc0b"])
    e1 = _cr(_cr(avgpool2(e0), wts["enc1a"]), wts["enc1b"])
    e2 = _cr(_cr(avgpool2(e1), wts["enc2a"]), wts["enc2b"])
    e3 = _cr(_cr(avgpool2(e2), wts["bota"]), wts["botb"])
    d2 = _cr(_cr(torch.cat([up2(e3), e2], -1), wts["dec2a"]), wts["dec2b"])
    d1 = _cr(_cr(torch.cat([up2(d2), e1], -1), wts["dec1a"]), wts["dec1b"])
    d0 = _cr(_cr(torch.cat([up2(d1), e0], -1), wts["dec0a"]), wts["dec0b"])
    feats = [d0, d1, d2, e3]
    if n_heads > 4:
        feats.append(avgpool2(e3))
    out = []
    for l in range(n_heads):
        w, b = wts[f"head{l}"]
        out.append(conv2d_nhwc(feats[l], w, b))
    return out


def to_torch(wts, dtype=torch.float64, requires_grad=False):
    out = {}
    for k, (w, b) in wts.items():
        wt = torch.tensor(w, dtype=dtype, requires_grad=requires_grad)
        bt = torch.tensor(b, dtype=dtype, requires_grad=requires_grad)
        out[k] = (wt, bt)
    return out

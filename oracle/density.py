"""Sampler network and budget normalisation, FP64 (torch CPU, autograd-capable).

Sec. 3 (Overview): the sampler predicts one output channel; a softmax over the image
turns it into a distribution; 1/8 of the budget is spread uniformly and 7/8 follows the
softmax, so that the per-pixel density s sums to the frame budget.
"""
import torch

F64 = torch.float64


def conv2d_nhwc(x, w, b):
    """Zero-padded 'same' convolution written as an explicit sum over taps.

    x [N, H, W, Ci], w [Co, k, k, Ci], b [Co]  ->  [N, H, W, Co]
    out[n, y, x, o] = b[o] + sum_{ky, kx, c} w[o, ky, kx, c] * x[n, y + ky - r, x + kx - r, c]
    with r = k // 2 and x = 0 outside the image.
    """
    N, H, W, Ci = x.shape
    Co, k, _, _ = w.shape
    r = k // 2
    xp = torch.nn.functional.pad(x, (0, 0, r, r, r, r))   # pads W then H (NHWC)
    out = b.reshape(1, 1, 1, Co).expand(N, H, W, Co).clone()
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, ky:ky + H, kx:kx + W, :]
            out = out + torch.einsum("nhwc,oc->nhwo", patch, w[:, ky, kx, :])
    return out


def cnn_forward(x, layers):
    """layers: list of (w, b, relu) applied in order (ReLU after each flagged layer)."""
    for w, b, relu in layers:
        x = conv2d_nhwc(x, w, b)
        if relu:
            x = torch.relu(x)
    return x


def normalise(z, budget: float, uniform_frac: float = 1.0 / 8.0):
    """s_i = f*B + (1-f)*B*Npx*softmax(z)_i, softmax over the H*W pixels of each frame.

    z [N, H, W] -> s [N, H, W];  sum_i s_i = Npx * B and s_i >= f*B.
    """
    N = z.shape[0]
    zf = z.reshape(N, -1)
    npx = zf.shape[1]
    m = zf.max(dim=1, keepdim=True).values
    e = torch.exp(zf - m)
    sm = e / e.sum(dim=1, keepdim=True)
    s = uniform_frac * budget + (1.0 - uniform_frac) * budget * npx * sm
    return s.reshape(z.shape)


def block_mean2(x):
    """2x2 block mean of NHWC features: out[n, y, x] = mean of x[n, 2y + j, 2x + i], i, j in {0, 1}."""
    N, H, W, C = x.shape
    out = torch.zeros((N, H // 2, W // 2, C), dtype=x.dtype)
    for j in range(2):
        for i in range(2):
            out = out + x[:, j::2, i::2, :]
    return out / 4.0


def density_quarter(x, layers, budget: float, uniform_frac: float = 1.0 / 8.0):
    """Sampler run at a quarter of the pixels (Sec. 7, density-map resolution ablation): the
    CNN sees the 2x2 block means of the features, its logits are normalised over the
    (H/2)x(W/2) map with the same per-pixel budget B, and every full-resolution pixel takes
    the density of its block: s[n, y, x] = s_q[n, y // 2, x // 2].  Each block of 4 pixels
    then carries 4 s_q, so sum(s) = Npx * B as at full resolution.

    x [N, H, W, C] (H, W even) -> (z_q [N, H/2, W/2], s [N, H, W])
    """
    zq = cnn_forward(block_mean2(x), layers)[..., 0]
    sq = normalise(zq, budget, uniform_frac)
    s = sq.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)
    return zq, s

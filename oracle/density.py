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
